/*
 * GridSPT reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of what the GPU library
 * computes, written from Taruya, Nishimichi & Jeong (2018), "GridSPT:
 * grid-based calculation for perturbation theory of large-scale structure"
 * (arXiv:1807.04215).  Only the test-suite, the package smoke entry and the
 * benchmark's CPU-baseline leg may load this file; the product library never
 * links or calls it.  It shares no code with the GPU library: its own DFT, its
 * own counter-based generator, its own spectrum and estimator loops.
 *
 * Conventions (Sec. II C, Eq. 17):
 *   grid       N^3 cells, box side L, cell x_j = j L / N with j in [0, N)
 *   modes      k = (2 pi / L) n, n_i = i for i < N/2, i - N otherwise
 *   forward    F(k) = N^-3 sum_x f(x) exp(-i k.x)
 *   inverse    f(x) = sum_k F(k) exp(+i k.x)
 *   masks      a mode is kept when n_x^2 + n_y^2 + n_z^2 <= n2max (integer)
 * Derivative multipliers i k_j use k_j = 0 at the Nyquist index i = N/2.
 * Spectra handed back to the caller use the half layout [ix][iy][iz],
 * iz in [0, N/2], interleaved complex; internally the oracle keeps full
 * complex N^3 arrays, which is wasteful and simple.
 *
 * Two forms of the source terms of the recursion (Eq. 10):
 *   P-form  the paper's own products, built from the 17 derived real fields of
 *           Eq. 15/16 (gradients of delta and theta, u, and d_i u_j);
 *   D-form  the same sources rewritten with div u = theta and u = grad phi:
 *           S_delta = div sum_m delta_m u_{n-m},
 *           S_theta = (1/2) lap sum_m u_m . u_{n-m}.
 * Both agree mode by mode whenever no product aliases (the 2/3 rule of
 * Sec. II C); under wider cuts they differ by aliased terms.
 *
 * Parity is pinned by the tests (closed forms, brute-force mode sums, the
 * one-dimensional Zel'dovich series, library routines); see tests/.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.28318530717958647692528676655900577;

/* ------------------------------------------------------------------------ */
/* threads                                                                    */
/* ------------------------------------------------------------------------ */

int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* 1D DFT: recursive mixed-radix decimation in time                           */
/* ------------------------------------------------------------------------ */

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* tw[j] = exp(sign * 2 pi i j / n0); the length-n twiddle w_n^e is
 * tw[(e mod n) * (n0 / n)]. */
static cplx *make_table(int n0, int sign)
{
    cplx *tw = malloc(sizeof(cplx) * (size_t)n0);
    for (int j = 0; j < n0; ++j) {
        double a = sign * TWO_PI * (double)j / (double)n0;
        tw[j] = cos(a) + I * sin(a);
    }
    return tw;
}

/* out[k] = sum_{j<n} in[j*s] w_n^{j k}.  Split x into the p subsequences
 * x[r + p q], transform each (length m = n/p), then combine
 * X[k + t m] = sum_r w_n^{r (k + t m)} Y_r[k]. */
static void dft_rec(const cplx *in, long s, cplx *out, int n,
                    const cplx *tw, int n0, cplx *work)
{
    if (n == 1) { out[0] = in[0]; return; }
    const int step = n0 / n;
    const int p = smallest_factor(n);
    if (p == n) {
        for (int k = 0; k < n; ++k) {
            cplx acc = 0;
            for (int j = 0; j < n; ++j)
                acc += in[j * s] * tw[(int)(((long)j * k) % n) * step];
            work[k] = acc;
        }
        memcpy(out, work, sizeof(cplx) * (size_t)n);
        return;
    }
    const int m = n / p;
    for (int r = 0; r < p; ++r)
        dft_rec(in + r * s, s * p, out + r * m, m, tw, n0, work);
    for (int k = 0; k < m; ++k)
        for (int t = 0; t < p; ++t) {
            const int kk = k + t * m;
            cplx acc = 0;
            for (int r = 0; r < p; ++r)
                acc += out[r * m + k] * tw[(int)(((long)r * kk) % n) * step];
            work[kk] = acc;
        }
    memcpy(out, work, sizeof(cplx) * (size_t)n);
}

/* Unnormalised 1D transform of n points spaced by `stride` in a[]. */
static void dft_strided(cplx *a, long stride, int n, const cplx *tw,
                        cplx *buf, cplx *res, cplx *work)
{
    for (int j = 0; j < n; ++j) buf[j] = a[j * stride];
    dft_rec(buf, 1, res, n, tw, n, work);
    for (int j = 0; j < n; ++j) a[j * stride] = res[j];
}

/* Unnormalised 3D transform of a full complex N^3 array [x][y][z],
 * sign -1 forward, +1 inverse.  One 1D transform per pencil, axis by axis. */
static void fft3d(cplx *a, int N, int sign)
{
    cplx *tw = make_table(N, sign);
    const long NN = (long)N * N;
    for (int axis = 0; axis < 3; ++axis) {
        const long stride = axis == 0 ? 1 : (axis == 1 ? N : NN);
#pragma omp parallel
        {
            cplx *buf = malloc(sizeof(cplx) * (size_t)N * 3);
            cplx *res = buf + N, *work = buf + 2 * N;
#pragma omp for schedule(static)
            for (long pencil = 0; pencil < NN; ++pencil) {
                const long i0 = pencil / N, i1 = pencil % N;
                long base;
                if (axis == 0) base = (i0 * N + i1) * N;       /* z pencils */
                else if (axis == 1) base = i0 * NN + i1;       /* y pencils */
                else base = i0 * N + i1;                       /* x pencils */
                dft_strided(a + base, stride, N, tw, buf, res, work);
            }
            free(buf);
        }
    }
    free(tw);
}

/* Exported for the tests: unnormalised 3D DFT of a full complex array. */
void or_fft3d(int N, cplx *a, int sign) { fft3d(a, N, sign < 0 ? -1 : 1); }

/* ------------------------------------------------------------------------ */
/* grid helpers                                                               */
/* ------------------------------------------------------------------------ */

static inline int sgn_index(int i, int N) { return i < N / 2 ? i : i - N; }
/* derivative wavenumber index: zero at the Nyquist index */
static inline int der_index(int i, int N) { return i == N / 2 ? 0 : sgn_index(i, N); }

static inline long long mode_n2(int ix, int iy, int iz, int N)
{
    long long a = sgn_index(ix, N), b = sgn_index(iy, N), c = sgn_index(iz, N);
    return a * a + b * b + c * c;
}

static cplx *cnew(int N) { return calloc((size_t)N * N * N, sizeof(cplx)); }
static double *rnew(int N) { return calloc((size_t)N * N * N, sizeof(double)); }

/* F = N^-3 sum_x f(x) e^{-ik.x} (Eq. 17, in three dimensions) */
static void forward_real(const double *f, cplx *F, int N)
{
    const long M = (long)N * N * N;
    for (long i = 0; i < M; ++i) F[i] = f[i];
    fft3d(F, N, -1);
    const double s = 1.0 / (double)M;
    for (long i = 0; i < M; ++i) F[i] *= s;
}

/* f = Re sum_k F(k) e^{+ik.x}; tmp is a complex scratch array */
static void inverse_real(const cplx *F, double *f, cplx *tmp, int N)
{
    const long M = (long)N * N * N;
    memcpy(tmp, F, sizeof(cplx) * (size_t)M);
    fft3d(tmp, N, +1);
    for (long i = 0; i < M; ++i) f[i] = creal(tmp[i]);
}

/* copy the iz <= N/2 half of a full spectrum to the caller's half layout */
static void store_half(const cplx *F, cplx *H, int N)
{
    const int Nh = N / 2 + 1;
    for (int ix = 0; ix < N; ++ix)
        for (int iy = 0; iy < N; ++iy)
            for (int iz = 0; iz < Nh; ++iz)
                H[((long)ix * N + iy) * Nh + iz] = F[((long)ix * N + iy) * N + iz];
}

/* ------------------------------------------------------------------------ */
/* counter-based generator: Philox4x64-10 (Salmon, Moraes, Dror & Shaw,      */
/* SC'11, "Parallel random numbers: as easy as 1, 2, 3")                     */
/* ------------------------------------------------------------------------ */

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {                      /* Weyl key schedule */
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Unit Gaussians of the four cells 4q .. 4q+3 of realisation `stream`:
 * Philox(counter = (q, stream, 0, 0), key = (seed, 0)); word pairs (w0, w1)
 * and (w2, w3) become uniforms in (0, 1) with 53 random bits, and Box-Muller
 * turns each pair into two Gaussians, cosine branch first.  Cell 4q + r
 * takes pair r / 2, branch r % 2. */
void or_group_gaussians(uint64_t seed, uint64_t stream, uint64_t q, double g[4])
{
    const uint64_t ctr[4] = {q, stream, 0, 0};
    const uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    or_philox4x64_10(ctr, key, w);
    for (int pair = 0; pair < 2; ++pair) {
        const double u1 = ((double)(w[2 * pair] >> 11) + 0.5) * 0x1p-53;
        const double u2 = ((double)(w[2 * pair + 1] >> 11) + 0.5) * 0x1p-53;
        const double r = sqrt(-2.0 * log(u1));
        g[2 * pair] = r * cos(TWO_PI * u2);
        g[2 * pair + 1] = r * sin(TWO_PI * u2);
    }
}

double or_unit_gaussian(uint64_t seed, uint64_t stream, uint64_t cell)
{
    double g[4];
    or_group_gaussians(seed, stream, cell >> 2, g);
    return g[cell & 3];
}

/* ------------------------------------------------------------------------ */
/* linear spectrum: P0(k) = A k^ns T_BBKS(k / Gamma)^2                         */
/* ------------------------------------------------------------------------ */

/* Bardeen, Bond, Kaiser & Szalay (1986), Eq. G3; q = k / (Gamma h/Mpc). */
double or_bbks(double q)
{
    if (q <= 0.0) return 1.0;
    const double a = 2.34 * q;
    const double poly = 1.0 + 3.89 * q + pow(16.1 * q, 2) + pow(5.46 * q, 3) + pow(6.71 * q, 4);
    return log1p(a) / a * pow(poly, -0.25);
}

double or_p0(double k, double A, double ns, double gamma)
{
    if (k <= 0.0) return 0.0;
    const double t = or_bbks(k / gamma);
    return A * pow(k, ns) * t * t;
}

/* sigma^2(R) = (1 / 2 pi^2) int dk k^2 P(k) W(kR)^2, top-hat W; composite
 * Simpson in ln k over [1e-6, 1e4] h/Mpc. */
double or_sigma_r(double R, double A, double ns, double gamma)
{
    const int n = 200000;
    const double a = log(1e-6), b = log(1e4), h = (b - a) / n;
    double acc = 0.0;
    for (int i = 0; i <= n; ++i) {
        const double k = exp(a + i * h), x = k * R;
        double w;
        if (x < 1e-3) w = 1.0 - x * x / 10.0;
        else w = 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
        const double f = k * k * k * or_p0(k, A, ns, gamma) * w * w; /* dk = k dlnk */
        const double c = (i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        acc += c * f;
    }
    acc *= h / 3.0;
    return sqrt(acc / (2.0 * M_PI * M_PI));
}

/* amplitude A giving sigma(8 Mpc/h) = sigma8 for the uncut spectrum */
double or_sigma8_amp(double sigma8, double ns, double gamma)
{
    const double s = or_sigma_r(8.0, 1.0, ns, gamma);
    return sigma8 * sigma8 / (s * s);
}

/* linear growth D(z)/D(0) for Omega_m, Omega_L (curvature 1 - Om - OL):
 * D(a) propto E(a) int_0^a da' / (a' E(a'))^3, composite Simpson. */
static double growth_unnorm(double a, double Om, double OL)
{
    const double Ok = 1.0 - Om - OL;
    const int n = 200000;
    const double h = a / n;
    double acc = 0.0;
    for (int i = 0; i <= n; ++i) {
        const double x = i * h;
        double f;
        if (x == 0.0) f = 0.0;                 /* integrand ~ x^{3/2} -> 0 */
        else {
            const double E = sqrt(Om / (x * x * x) + Ok / (x * x) + OL);
            f = 1.0 / pow(x * E, 3);
        }
        const double c = (i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        acc += c * f;
    }
    acc *= h / 3.0;
    const double Ea = sqrt(Om / (a * a * a) + Ok / (a * a) + OL);
    return Ea * acc;
}

double or_growth(double Om, double OL, double z)
{
    return growth_unnorm(1.0 / (1.0 + z), Om, OL) / growth_unnorm(1.0, Om, OL);
}

/* ------------------------------------------------------------------------ */
/* step (1) of Sec. II C: Gaussian linear field                               */
/* ------------------------------------------------------------------------ */

/* delta1(x) = inverse of W1(k) sqrt(P0(k) N^3 / L^3) D w(k), with w(k) the
 * forward transform of unit white noise w(x), so that
 * L^3 <|delta1(k)|^2> = D^2 P0(k) on kept modes; delta1(k = 0) = 0. */
int or_linear_field(int N, double L, double A, double ns, double gamma,
                    double growth, int64_t n2max1, uint64_t seed, uint64_t stream,
                    double *delta1)
{
    const long M = (long)N * N * N;
    cplx *F = cnew(N), *tmp = cnew(N);
    double *w = rnew(N);
    if (!F || !tmp || !w) { free(F); free(tmp); free(w); return -1; }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < M; ++c) w[c] = or_unit_gaussian(seed, stream, (uint64_t)c);
    forward_real(w, F, N);
    const double kF = TWO_PI / L;
    const double vol = (double)M / (L * L * L);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < M; ++c) {
        const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
        const long long n2 = mode_n2(ix, iy, iz, N);
        if (n2 == 0 || n2 > n2max1) { F[c] = 0; continue; }
        const double k = kF * sqrt((double)n2);
        F[c] *= sqrt(or_p0(k, A, ns, gamma) * vol) * growth;
    }
    inverse_real(F, delta1, tmp, N);
    free(F); free(tmp); free(w);
    return 0;
}

/* The same field evaluated at single modes, straight from the definition:
 * out[j] = W1(k_j) sqrt(P0(k_j) N^3 / L^3) D N^-3 sum_x w(x) e^{-i k_j.x}
 * for signed integer modes k_j = modes[3j..3j+2], one pass over all N^3 cells
 * (compensated summation), without any FFT.  For sampling very large grids. */
int or_linear_modes(int N, double L, double A, double ns, double gamma, double growth, int64_t n2max1,
                    uint64_t seed, uint64_t stream, int nm, const int *modes, cplx *out)
{
    const long M = (long)N * N * N;
    cplx *tab = malloc(sizeof(cplx) * (size_t)nm * 3 * N);      /* e^{-2 pi i m x / N} per axis */
    for (int j = 0; j < nm; ++j)
        for (int a = 0; a < 3; ++a)
            for (int x = 0; x < N; ++x) {
                const long e = ((long)modes[3 * j + a] * x) % N;
                const double ang = -TWO_PI * (double)(e < 0 ? e + N : e) / (double)N;
                tab[((long)j * 3 + a) * N + x] = cos(ang) + I * sin(ang);
            }
    cplx *sum = calloc((size_t)nm, sizeof(cplx)), *cmp = calloc((size_t)nm, sizeof(cplx));
#pragma omp parallel
    {
        cplx *ls = calloc((size_t)nm, sizeof(cplx)), *lc = calloc((size_t)nm, sizeof(cplx));
#pragma omp for schedule(static)
        for (long q = 0; q < M / 4; ++q) {
            double g[4];
            or_group_gaussians(seed, stream, (uint64_t)q, g);
            for (int r = 0; r < 4; ++r) {
                const long c = 4 * q + r;
                const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                for (int j = 0; j < nm; ++j) {
                    const cplx t = g[r] * tab[((long)j * 3 + 0) * N + ix] * tab[((long)j * 3 + 1) * N + iy] *
                                   tab[((long)j * 3 + 2) * N + iz];
                    const cplx y = t - lc[j];          /* Kahan */
                    const cplx s2 = ls[j] + y;
                    lc[j] = (s2 - ls[j]) - y;
                    ls[j] = s2;
                }
            }
        }
#pragma omp critical
        for (int j = 0; j < nm; ++j) {
            const cplx y = ls[j] - cmp[j];
            const cplx s2 = sum[j] + y;
            cmp[j] = (s2 - sum[j]) - y;
            sum[j] = s2;
        }
        free(ls); free(lc);
    }
    const double kF = TWO_PI / L, vol = (double)M / (L * L * L);
    for (int j = 0; j < nm; ++j) {
        const long long a = modes[3 * j], b = modes[3 * j + 1], c = modes[3 * j + 2];
        const long long n2 = a * a + b * b + c * c;
        if (n2 == 0 || n2 > n2max1) { out[j] = 0; continue; }
        const double k = kF * sqrt((double)n2);
        out[j] = sum[j] / (double)M * sqrt(or_p0(k, A, ns, gamma) * vol) * growth;
    }
    free(tab); free(sum); free(cmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* recursion (Eq. 10, 11)                                                     */
/* ------------------------------------------------------------------------ */

/* c_n = 2 / ((2n + 3)(n - 1)); the 2x2 matrix [[n + 1/2, 1], [3/2, n]]. */
static void order_combine(int n, cplx sd, cplx st, cplx *dn, cplx *tn)
{
    const double c = 2.0 / ((2.0 * n + 3.0) * (n - 1.0));
    *dn = c * ((n + 0.5) * sd + st);
    *tn = c * (1.5 * sd + n * st);
}

/* spectral multiplier -i k_j / k^2 (Eq. 5), zero at k = 0 */
static cplx uvec_mult(int ix, int iy, int iz, int j, int N, double kF)
{
    const int d[3] = {der_index(ix, N), der_index(iy, N), der_index(iz, N)};
    const long long n2 = mode_n2(ix, iy, iz, N);
    if (n2 == 0) return 0;
    return -I * (double)d[j] / ((double)n2 * kF);
}

/* Linear order: delta1(k) = theta1(k) = W1 F[delta1_in], k = 0 removed. */
static void linear_spectrum(const double *d1_in, cplx *d1k, int N, int64_t n2max1)
{
    forward_real(d1_in, d1k, N);
    const long M = (long)N * N * N;
    for (long c = 0; c < M; ++c) {
        const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
        const long long n2 = mode_n2(ix, iy, iz, N);
        if (n2 == 0 || n2 > n2max1) d1k[c] = 0;
    }
}

/* u(x) = inverse of (-i k / k^2) theta(k), three components */
static void velocity_from_theta(const cplx *tk, double *u[3], cplx *tmp, cplx *tmp2,
                                int N, double kF)
{
    const long M = (long)N * N * N;
    for (int j = 0; j < 3; ++j) {
        for (long c = 0; c < M; ++c) {
            const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
            tmp2[c] = uvec_mult(ix, iy, iz, j, N, kF) * tk[c];
        }
        inverse_real(tmp2, u[j], tmp, N);
    }
}

/*
 * D-form recursion.  Inputs: grid (N, L), nmax in [1, 5+], masks n2max1
 * (linear field) and n2max2 (orders >= 2), delta1_in (N^3 real, any field;
 * W1 is applied here).  Outputs: delta, theta as nmax consecutive N^3 real
 * fields; optional half-layout spectra delta_k, theta_k (nmax * N*N*(N/2+1)).
 */
int or_orders_dform(int N, double L, int nmax, int64_t n2max1, int64_t n2max2,
                    const double *delta1_in, double *delta, double *theta,
                    cplx *delta_k, cplx *theta_k)
{
    const long M = (long)N * N * N, Mh = (long)N * N * (N / 2 + 1);
    const double kF = TWO_PI / L;
    double **u = calloc((size_t)nmax * 3, sizeof(double *));
    cplx *dk = cnew(N), *tk = cnew(N), *tmp = cnew(N), *tmp2 = cnew(N);
    cplx *Vk[3] = {cnew(N), cnew(N), cnew(N)}, *Wk = cnew(N);
    double *V = rnew(N), *W = rnew(N);
    for (int i = 0; i < 3 * (nmax - 1); ++i) u[i] = rnew(N);

    /* order 1 */
    linear_spectrum(delta1_in, dk, N, n2max1);
    inverse_real(dk, delta, tmp, N);
    memcpy(theta, delta, sizeof(double) * (size_t)M);
    if (delta_k) store_half(dk, delta_k, N);
    if (theta_k) store_half(dk, theta_k, N);
    if (nmax > 1) velocity_from_theta(dk, u, tmp, tmp2, N, kF);

    for (int n = 2; n <= nmax; ++n) {
        /* V = sum_m delta_m u_{n-m},  W = sum_m u_m . u_{n-m} */
        for (int j = 0; j < 3; ++j) {
            memset(V, 0, sizeof(double) * (size_t)M);
            for (int m = 1; m <= n - 1; ++m) {
                const double *dm = delta + (long)(m - 1) * M;
                const double *un = u[3 * (n - m - 1) + j];
                for (long c = 0; c < M; ++c) V[c] += dm[c] * un[c];
            }
            forward_real(V, Vk[j], N);
        }
        memset(W, 0, sizeof(double) * (size_t)M);
        for (int m = 1; m <= n - 1; ++m)
            for (int j = 0; j < 3; ++j) {
                const double *a = u[3 * (m - 1) + j], *b = u[3 * (n - m - 1) + j];
                for (long c = 0; c < M; ++c) W[c] += a[c] * b[c];
            }
        forward_real(W, Wk, N);

        /* S_delta = i k . V(k), S_theta = -(k^2 / 2) W(k); mask W2 */
        for (long c = 0; c < M; ++c) {
            const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
            const long long n2 = mode_n2(ix, iy, iz, N);
            if (n2 == 0 || n2 > n2max2) { dk[c] = 0; tk[c] = 0; continue; }
            const double kx = kF * der_index(ix, N), ky = kF * der_index(iy, N),
                         kz = kF * der_index(iz, N);
            const cplx sd = I * (kx * Vk[0][c] + ky * Vk[1][c] + kz * Vk[2][c]);
            const cplx st = -0.5 * kF * kF * (double)n2 * Wk[c];
            order_combine(n, sd, st, &dk[c], &tk[c]);
        }
        inverse_real(dk, delta + (long)(n - 1) * M, tmp, N);
        inverse_real(tk, theta + (long)(n - 1) * M, tmp, N);
        if (delta_k) store_half(dk, delta_k + (long)(n - 1) * Mh, N);
        if (theta_k) store_half(tk, theta_k + (long)(n - 1) * Mh, N);
        if (n < nmax) velocity_from_theta(tk, u + 3 * (n - 1), tmp, tmp2, N, kF);
    }

    for (int i = 0; i < 3 * (nmax - 1); ++i) free(u[i]);
    free(u); free(dk); free(tk); free(tmp); free(tmp2);
    for (int j = 0; j < 3; ++j) free(Vk[j]);
    free(Wk); free(V); free(W);
    return 0;
}

/*
 * P-form recursion: the products exactly as printed in Eq. 10, built from the
 * real fields of Eq. 15/16 for every earlier order m:
 *   delta_m, theta_m, grad delta_m, grad theta_m, u_m, d_i (u_m)_j.
 * Same arguments and outputs as or_orders_dform.
 */
int or_orders_pform(int N, double L, int nmax, int64_t n2max1, int64_t n2max2,
                    const double *delta1_in, double *delta, double *theta,
                    cplx *delta_k, cplx *theta_k)
{
    const long M = (long)N * N * N, Mh = (long)N * N * (N / 2 + 1);
    const double kF = TWO_PI / L;
    /* per order: gd[3], gt[3], u[3], du[9] (d_i u_j, row-major i*3+j) */
    enum { GD = 0, GT = 3, U = 6, DU = 9, NDER = 18 };
    double **der = calloc((size_t)nmax * NDER, sizeof(double *));
    cplx *dk = cnew(N), *tk = cnew(N), *tmp = cnew(N), *tmp2 = cnew(N);
    cplx *Sdk = cnew(N), *Stk = cnew(N);
    double *Sd = rnew(N), *St = rnew(N);

    for (int n = 1; n <= nmax; ++n) {
        if (n == 1) {
            linear_spectrum(delta1_in, dk, N, n2max1);
            memcpy(tk, dk, sizeof(cplx) * (size_t)M);
        } else {
            memset(Sd, 0, sizeof(double) * (size_t)M);
            memset(St, 0, sizeof(double) * (size_t)M);
            for (int m = 1; m <= n - 1; ++m) {
                const int a = m - 1, b = n - m - 1;
                const double *dm = delta + (long)a * M, *tb = theta + (long)b * M;
                double *const *Da = der + (long)a * NDER, *const *Db = der + (long)b * NDER;
                for (long c = 0; c < M; ++c) {
                    /* (grad delta_m) . u_{n-m} + delta_m theta_{n-m} */
                    double s = dm[c] * tb[c];
                    for (int j = 0; j < 3; ++j) s += Da[GD + j][c] * Db[U + j][c];
                    Sd[c] += s;
                    /* [d_j (u_m)_k][d_k (u_{n-m})_j] + u_m . grad theta_{n-m} */
                    double t = 0.0;
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k)
                            t += Da[DU + 3 * j + k][c] * Db[DU + 3 * k + j][c];
                    for (int j = 0; j < 3; ++j) t += Da[U + j][c] * Db[GT + j][c];
                    St[c] += t;
                }
            }
            forward_real(Sd, Sdk, N);
            forward_real(St, Stk, N);
            for (long c = 0; c < M; ++c) {
                const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                const long long n2 = mode_n2(ix, iy, iz, N);
                if (n2 == 0 || n2 > n2max2) { dk[c] = 0; tk[c] = 0; continue; }
                order_combine(n, Sdk[c], Stk[c], &dk[c], &tk[c]);
            }
        }
        inverse_real(dk, delta + (long)(n - 1) * M, tmp, N);
        inverse_real(tk, theta + (long)(n - 1) * M, tmp, N);
        if (delta_k) store_half(dk, delta_k + (long)(n - 1) * Mh, N);
        if (theta_k) store_half(tk, theta_k + (long)(n - 1) * Mh, N);
        if (n == nmax) break;

        /* derived fields of order n (Eq. 15/16) */
        double **D = der + (long)(n - 1) * NDER;
        for (int i = 0; i < NDER; ++i) D[i] = rnew(N);
        for (int j = 0; j < 3; ++j) {
            for (int which = 0; which < 3; ++which) {   /* grad delta, grad theta, u */
                for (long c = 0; c < M; ++c) {
                    const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                    const int d[3] = {der_index(ix, N), der_index(iy, N), der_index(iz, N)};
                    if (which == 0) tmp2[c] = I * kF * d[j] * dk[c];
                    else if (which == 1) tmp2[c] = I * kF * d[j] * tk[c];
                    else tmp2[c] = uvec_mult(ix, iy, iz, j, N, kF) * tk[c];
                }
                inverse_real(tmp2, D[(which == 0 ? GD : which == 1 ? GT : U) + j], tmp, N);
            }
            for (int i = 0; i < 3; ++i) {                /* d_i u_j = (k_i k_j / k^2) theta */
                for (long c = 0; c < M; ++c) {
                    const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                    const int d[3] = {der_index(ix, N), der_index(iy, N), der_index(iz, N)};
                    tmp2[c] = I * kF * d[i] * uvec_mult(ix, iy, iz, j, N, kF) * tk[c];
                }
                inverse_real(tmp2, D[DU + 3 * i + j], tmp, N);
            }
        }
    }

    for (long i = 0; i < (long)nmax * NDER; ++i) free(der[i]);
    free(der); free(dk); free(tk); free(tmp); free(tmp2); free(Sdk); free(Stk);
    free(Sd); free(St);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* linear field from a given noise field, and the reverse-mode gradient      */
/* ------------------------------------------------------------------------ */

/* W1(k) sqrt(P0(k) N^3 / L^3) D at integer mode n2 (zero at k = 0 and outside W1) */
static double noise_amplitude(long long n2, double kF, double A, double ns, double gamma, double growth,
                              double vol, int64_t n2max1)
{
    if (n2 == 0 || n2 > n2max1) return 0.0;
    return sqrt(or_p0(kF * sqrt((double)n2), A, ns, gamma) * vol) * growth;
}

/* Step (1) of Sec. II C with the white noise w(x) given instead of drawn:
 * delta1 = inverse of W1(k) sqrt(P0(k) N^3 / L^3) D F[w](k). */
int or_noise_field(int N, double L, double A, double ns, double gamma, double growth, int64_t n2max1,
                   const double *w, double *delta1)
{
    const long M = (long)N * N * N;
    cplx *F = cnew(N), *tmp = cnew(N);
    if (!F || !tmp) { free(F); free(tmp); return -1; }
    const double kF = TWO_PI / L, vol = (double)M / (L * L * L);
    forward_real(w, F, N);
    for (long c = 0; c < M; ++c) {
        const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
        F[c] *= noise_amplitude(mode_n2(ix, iy, iz, N), kF, A, ns, gamma, growth, vol, n2max1);
    }
    inverse_real(F, delta1, tmp, N);
    free(F); free(tmp);
    return 0;
}

/*
 * Reverse mode of (noise -> delta_1 -> D-form orders 2..nmax).  Given
 * gdelta = dJ/d delta_n(x) (nmax consecutive N^3 real fields) for a scalar J,
 * returns gw = dJ/dw(x).  Every step of the forward map is a real-linear
 * spectral multiply x -> F^-1[m(k) F[x]] (adjoint: the multiplier conj(m(k)),
 * since m(-k) = conj(m(k)) for real output) or a pointwise product:
 *   order n >= 2:  (delta_n, theta_n)^ = W2 c_n M (S_delta, S_theta),
 *                  M = [[n + 1/2, 1], [3/2, n]], S_delta = i k.V^, S_theta = -(k^2/2) W^,
 *                  u_n = F^-1[(-i k / k^2) theta_n^]
 *   adjoint:       G_d = F[g delta_n], G_t = sum_j (+i k_j / k^2) F[g u_n,j],
 *                  (a, b) = W2 c_n M^T (G_d, G_t),
 *                  g V_j = F^-1[-i k_j a],  g W = F^-1[-(k^2/2) b]
 *   products:      V = sum_m delta_m u_{n-m}, W = sum_m u_m . u_{n-m}, so for j < n
 *                  g delta_j += gV . u_{n-j},  g u_{n-j} += gV delta_j,  g u_j += 2 gW u_{n-j}
 *   order 1:       delta_1 = theta_1 = F^-1[a1(k) F[w]], a1 = noise_amplitude;
 *                  gw = F^-1[a1 (F[g delta_1] + sum_j (+i k_j / k^2) F[g u_1,j])]
 * The forward fields delta_m, u_m (m < nmax) are recomputed here first.
 */
int or_adjoint_dform(int N, double L, double A, double ns, double gamma, double growth, int nmax,
                     int64_t n2max1, int64_t n2max2, const double *w, const double *gdelta, double *gw)
{
    if (nmax < 1) return -1;
    const long M = (long)N * N * N;
    const double kF = TWO_PI / L, vol = (double)M / (L * L * L);
    const int nm = nmax - 1;                       /* orders with stored delta_m, u_m */
    double **dl = calloc((size_t)(nm + 1), sizeof(double *));
    double **u = calloc((size_t)(3 * nm + 3), sizeof(double *));
    double **gd = calloc((size_t)(nmax + 1), sizeof(double *));
    double **gu = calloc((size_t)(3 * nm + 3), sizeof(double *));
    cplx *dk = cnew(N), *tk = cnew(N), *tmp = cnew(N), *tmp2 = cnew(N), *Gd = cnew(N), *Gt = cnew(N);
    cplx *Vk[3] = {cnew(N), cnew(N), cnew(N)}, *Wk = cnew(N);
    double *V = rnew(N), *W = rnew(N), *gV[3] = {rnew(N), rnew(N), rnew(N)}, *gW = rnew(N);
    for (int m = 1; m <= nm; ++m) {
        dl[m] = rnew(N);
        for (int j = 0; j < 3; ++j) { u[3 * m + j] = rnew(N); gu[3 * m + j] = rnew(N); }
    }
    for (int m = 1; m <= nmax; ++m) {
        gd[m] = rnew(N);
        memcpy(gd[m], gdelta + (long)(m - 1) * M, sizeof(double) * (size_t)M);
    }

    /* ---- forward: delta_m and u_m for m < nmax ---- */
    if (nm >= 1) {
        forward_real(w, dk, N);
        for (long c = 0; c < M; ++c) {
            const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
            dk[c] *= noise_amplitude(mode_n2(ix, iy, iz, N), kF, A, ns, gamma, growth, vol, n2max1);
        }
        inverse_real(dk, dl[1], tmp, N);
        velocity_from_theta(dk, u + 3, tmp, tmp2, N, kF);
    }
    for (int n = 2; n <= nm; ++n) {
        for (int j = 0; j < 3; ++j) {
            memset(V, 0, sizeof(double) * (size_t)M);
            for (int m = 1; m <= n - 1; ++m)
                for (long c = 0; c < M; ++c) V[c] += dl[m][c] * u[3 * (n - m) + j][c];
            forward_real(V, Vk[j], N);
        }
        memset(W, 0, sizeof(double) * (size_t)M);
        for (int m = 1; m <= n - 1; ++m)
            for (int j = 0; j < 3; ++j)
                for (long c = 0; c < M; ++c) W[c] += u[3 * m + j][c] * u[3 * (n - m) + j][c];
        forward_real(W, Wk, N);
        for (long c = 0; c < M; ++c) {
            const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
            const long long n2 = mode_n2(ix, iy, iz, N);
            if (n2 == 0 || n2 > n2max2) { dk[c] = 0; tk[c] = 0; continue; }
            const double kx = kF * der_index(ix, N), ky = kF * der_index(iy, N), kz = kF * der_index(iz, N);
            const cplx sd = I * (kx * Vk[0][c] + ky * Vk[1][c] + kz * Vk[2][c]);
            const cplx st = -0.5 * kF * kF * (double)n2 * Wk[c];
            order_combine(n, sd, st, &dk[c], &tk[c]);
        }
        inverse_real(dk, dl[n], tmp, N);
        velocity_from_theta(tk, u + 3 * n, tmp, tmp2, N, kF);
    }

    /* ---- reverse ---- */
    for (int n = nmax; n >= 2; --n) {
        forward_real(gd[n], Gd, N);
        memset(Gt, 0, sizeof(cplx) * (size_t)M);
        if (n <= nm)
            for (int j = 0; j < 3; ++j) {
                forward_real(gu[3 * n + j], tmp2, N);
                for (long c = 0; c < M; ++c) {
                    const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                    Gt[c] += conj(uvec_mult(ix, iy, iz, j, N, kF)) * tmp2[c];
                }
            }
        const double cn = 2.0 / ((2.0 * n + 3.0) * (n - 1.0));
        for (long c = 0; c < M; ++c) {       /* a -> dk, b -> tk */
            const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
            const long long n2 = mode_n2(ix, iy, iz, N);
            if (n2 == 0 || n2 > n2max2) { dk[c] = 0; tk[c] = 0; continue; }
            dk[c] = cn * ((n + 0.5) * Gd[c] + 1.5 * Gt[c]);
            tk[c] = cn * (Gd[c] + n * Gt[c]);
        }
        for (int j = 0; j < 3; ++j) {
            for (long c = 0; c < M; ++c) {
                const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                const int d[3] = {der_index(ix, N), der_index(iy, N), der_index(iz, N)};
                tmp2[c] = -I * kF * d[j] * dk[c];
            }
            inverse_real(tmp2, gV[j], tmp, N);
        }
        for (long c = 0; c < M; ++c) {
            const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
            tmp2[c] = -0.5 * kF * kF * (double)mode_n2(ix, iy, iz, N) * tk[c];
        }
        inverse_real(tmp2, gW, tmp, N);
        for (int j = 1; j <= n - 1; ++j)
            for (long c = 0; c < M; ++c) {
                double s = 0.0;
                for (int q = 0; q < 3; ++q) {
                    s += gV[q][c] * u[3 * (n - j) + q][c];
                    gu[3 * (n - j) + q][c] += gV[q][c] * dl[j][c];
                    gu[3 * j + q][c] += 2.0 * gW[c] * u[3 * (n - j) + q][c];
                }
                gd[j][c] += s;
            }
    }
    /* order 1 */
    forward_real(gd[1], Gd, N);
    if (nm >= 1)
        for (int j = 0; j < 3; ++j) {
            forward_real(gu[3 + j], tmp2, N);
            for (long c = 0; c < M; ++c) {
                const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
                Gd[c] += conj(uvec_mult(ix, iy, iz, j, N, kF)) * tmp2[c];
            }
        }
    for (long c = 0; c < M; ++c) {
        const int ix = (int)(c / ((long)N * N)), iy = (int)((c / N) % N), iz = (int)(c % N);
        Gd[c] *= noise_amplitude(mode_n2(ix, iy, iz, N), kF, A, ns, gamma, growth, vol, n2max1);
    }
    inverse_real(Gd, gw, tmp, N);

    for (int m = 1; m <= nm; ++m) {
        free(dl[m]);
        for (int j = 0; j < 3; ++j) { free(u[3 * m + j]); free(gu[3 * m + j]); }
    }
    for (int m = 1; m <= nmax; ++m) free(gd[m]);
    free(dl); free(u); free(gd); free(gu);
    free(dk); free(tk); free(tmp); free(tmp2); free(Gd); free(Gt);
    for (int j = 0; j < 3; ++j) { free(Vk[j]); free(gV[j]); }
    free(Wk); free(V); free(W); free(gW);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* estimators                                                                 */
/* ------------------------------------------------------------------------ */

static int find_bin(long long n2, int nbins, const int64_t *edges)
{
    for (int b = 0; b < nbins; ++b)
        if (n2 >= edges[b] && n2 < edges[b + 1]) return b;
    return -1;
}

/*
 * Shell-averaged cross spectra, the estimators of Eq. 19-21 with the volume
 * factor: P_ab(bin) = L^3 sum w Re[F_a F_b^*] / sum w over half-layout modes,
 * w = 1 on the iz = 0 and iz = N/2 planes (their mirror images are stored
 * too) and 2 elsewhere.  kmean = sum w |k| / sum w, nmodes = sum w.
 */
int or_power(int N, double L, int nfields, const cplx *const *fk,
             int npairs, const int *pairs, int nbins, const int64_t *edges,
             double *pk, double *kmean, double *nmodes)
{
    const int Nh = N / 2 + 1;
    const double kF = TWO_PI / L;
    double *acc = calloc((size_t)npairs * nbins, sizeof(double));
    double *cnt = calloc((size_t)nbins, sizeof(double)), *ks = calloc((size_t)nbins, sizeof(double));
    for (int p = 0; p < npairs; ++p)
        if (pairs[2 * p] < 0 || pairs[2 * p] >= nfields || pairs[2 * p + 1] < 0 ||
            pairs[2 * p + 1] >= nfields) { free(acc); free(cnt); free(ks); return -1; }
    for (int ix = 0; ix < N; ++ix)
        for (int iy = 0; iy < N; ++iy)
            for (int iz = 0; iz < Nh; ++iz) {
                const long long n2 = mode_n2(ix, iy, iz, N);
                const int b = find_bin(n2, nbins, edges);
                if (b < 0) continue;
                const double w = (iz == 0 || iz == N / 2) ? 1.0 : 2.0;
                const long c = ((long)ix * N + iy) * Nh + iz;
                cnt[b] += w;
                ks[b] += w * kF * sqrt((double)n2);
                for (int p = 0; p < npairs; ++p) {
                    const cplx a = fk[pairs[2 * p]][c], bb = fk[pairs[2 * p + 1]][c];
                    acc[(long)p * nbins + b] += w * creal(a * conj(bb));
                }
            }
    const double vol = L * L * L;
    for (int b = 0; b < nbins; ++b) {
        if (nmodes) nmodes[b] = cnt[b];
        if (kmean) kmean[b] = cnt[b] > 0 ? ks[b] / cnt[b] : 0.0;
        for (int p = 0; p < npairs; ++p)
            pk[(long)p * nbins + b] = cnt[b] > 0 ? vol * acc[(long)p * nbins + b] / cnt[b] : 0.0;
    }
    free(acc); free(cnt); free(ks);
    return 0;
}

/* value of a real field's spectrum at signed mode (a, b, c) from the half
 * layout, using F(-k) = F(k)^*; the mode must lie on the grid. */
static cplx half_value(const cplx *H, int N, int a, int b, int c)
{
    const int Nh = N / 2 + 1;
    int conjugate = 0;
    if (c < 0 || (c == -N / 2)) { a = -a; b = -b; c = -c; conjugate = 1; }
    const int ix = ((a % N) + N) % N, iy = ((b % N) + N) % N, iz = c;
    const cplx v = H[((long)ix * N + iy) * Nh + iz];
    return conjugate ? conj(v) : v;
}

static int on_grid(int v, int N) { return v >= -N / 2 && v < N / 2; }

/*
 * Closed-triangle bispectrum sums of Eq. 22/23 by direct enumeration:
 * for term t = (fa, fb, fc, tri) with shells (b1, b2, b3) of triangle `tri`,
 *   T = sum_{k1 in b1, k2 in b2, k3 = -k1-k2 in b3} F_fa(k1) F_fb(k2) F_fc(k3)
 * over all grid modes (both half-spaces), with exact (unwrapped) closure;
 *   ntriangles[tri] = number of such ordered (k1, k2, k3),
 *   bk[t] = L^6 Re T / ntriangles[tri].
 */
int or_bispectrum(int N, double L, int nfields, const cplx *const *fk,
                  int ntri, const int *bins, int nterms, const int *terms,
                  int nbins, const int64_t *edges, double *bk, double *ntriangles)
{
    /* shell member lists over the full grid */
    long *count = calloc((size_t)nbins, sizeof(long));
    for (int a = -N / 2; a < N / 2; ++a)
        for (int b = -N / 2; b < N / 2; ++b)
            for (int c = -N / 2; c < N / 2; ++c) {
                const int s = find_bin((long long)a * a + (long long)b * b + (long long)c * c, nbins, edges);
                if (s >= 0) count[s]++;
            }
    int **shell = calloc((size_t)nbins, sizeof(int *));
    long *fill = calloc((size_t)nbins, sizeof(long));
    for (int s = 0; s < nbins; ++s) shell[s] = malloc(sizeof(int) * 3 * (size_t)(count[s] + 1));
    for (int a = -N / 2; a < N / 2; ++a)
        for (int b = -N / 2; b < N / 2; ++b)
            for (int c = -N / 2; c < N / 2; ++c) {
                const int s = find_bin((long long)a * a + (long long)b * b + (long long)c * c, nbins, edges);
                if (s < 0) continue;
                int *e = shell[s] + 3 * fill[s]++;
                e[0] = a; e[1] = b; e[2] = c;
            }
    const double vol2 = L * L * L * L * L * L;
    int rc = 0;
    for (int t = 0; t < ntri; ++t) {
        const int b1 = bins[3 * t], b2 = bins[3 * t + 1], b3 = bins[3 * t + 2];
        if (b1 < 0 || b1 >= nbins || b2 < 0 || b2 >= nbins || b3 < 0 || b3 >= nbins) { rc = -1; goto out; }
        double ntr = 0.0;
        for (long i = 0; i < count[b1]; ++i)
            for (long j = 0; j < count[b2]; ++j) {
                const int *p = shell[b1] + 3 * i, *q = shell[b2] + 3 * j;
                const int a = -(p[0] + q[0]), b = -(p[1] + q[1]), c = -(p[2] + q[2]);
                if (!on_grid(a, N) || !on_grid(b, N) || !on_grid(c, N)) continue;
                if (find_bin((long long)a * a + (long long)b * b + (long long)c * c, nbins, edges) == b3) ntr += 1.0;
            }
        ntriangles[t] = ntr;
    }
    for (int u = 0; u < nterms; ++u) {
        const int fa = terms[4 * u], fb = terms[4 * u + 1], fc = terms[4 * u + 2], t = terms[4 * u + 3];
        if (fa < 0 || fa >= nfields || fb < 0 || fb >= nfields || fc < 0 || fc >= nfields ||
            t < 0 || t >= ntri) { rc = -1; goto out; }
        const int b1 = bins[3 * t], b2 = bins[3 * t + 1], b3 = bins[3 * t + 2];
        cplx acc = 0;
        for (long i = 0; i < count[b1]; ++i)
            for (long j = 0; j < count[b2]; ++j) {
                const int *p = shell[b1] + 3 * i, *q = shell[b2] + 3 * j;
                const int a = -(p[0] + q[0]), b = -(p[1] + q[1]), c = -(p[2] + q[2]);
                if (!on_grid(a, N) || !on_grid(b, N) || !on_grid(c, N)) continue;
                if (find_bin((long long)a * a + (long long)b * b + (long long)c * c, nbins, edges) != b3) continue;
                acc += half_value(fk[fa], N, p[0], p[1], p[2]) * half_value(fk[fb], N, q[0], q[1], q[2]) *
                       half_value(fk[fc], N, a, b, c);
            }
        bk[u] = ntriangles[t] > 0 ? vol2 * creal(acc) / ntriangles[t] : 0.0;
    }
out:
    for (int s = 0; s < nbins; ++s) free(shell[s]);
    free(shell); free(fill); free(count);
    return rc;
}

/* sum_n coef[n] delta_n(x) (Sec. III A, the truncated series of Eq. 8) */
void or_sum_orders(long ncell, int nmax, const double *delta, const double *coef, double *out)
{
    for (long c = 0; c < ncell; ++c) {
        double s = 0.0;
        for (int n = 0; n < nmax; ++n) s += coef[n] * delta[(long)n * ncell + c];
        out[c] = s;
    }
}

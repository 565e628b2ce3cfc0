/*
 * gridspt.h -- C ABI of libgridspt, a GPU (gfx950) implementation of the
 * GridSPT hot path of Taruya, Nishimichi & Jeong (2018), "GridSPT: grid-based
 * calculation for perturbation theory of large-scale structure",
 * arXiv:1807.04215.
 *
 * What it computes.  From a Gaussian linear density field on an N^3 periodic
 * grid (Sec. II C, step 1), the standard-perturbation-theory fields delta_n and
 * theta_n for n = 1..nmax <= 5 by the real-space recursion of Eq. 10 with the
 * linear order of Eq. 11, evaluated with FFTs as in steps 2-6 of Sec. II C,
 * and the estimators built on them: shell-averaged cross spectra (Eq. 19-21)
 * and closed-triangle bispectra (Eq. 22-23, FFT estimator).
 *
 * Conventions.
 *   - Grid: N^3 cells, box side L [Mpc/h]; x_j = j L / N, j in [0, N).
 *   - Modes: k = (2 pi / L) n with integer n; forward transform
 *     F(k) = N^-3 sum_x f(x) e^{-i k.x}, inverse f(x) = sum_k F(k) e^{i k.x}
 *     (Eq. 17, three-dimensional).
 *   - Sharp-k masks are integer: a mode is kept when |n|^2 <= n2max.  Every
 *     mask must satisfy n2max < (N/2)^2 (the cut lies below Nyquist).
 *   - Real fields: float32 or float64 [x][y][z], z fastest, N^3 elements.
 *   - Spectra ("cube layout"): the masked fields have no mode with
 *     |n_i| > Kc, Kc = grid.kc; a spectrum is stored as interleaved complex
 *     [kz][ky][kx] with kz in [0, Kc] and ky, kx in "fftfreq" order over
 *     2Kc + 1 values (index i <= Kc is mode +i, index i > Kc is mode i - 2Kc - 1),
 *     (Kc + 1)(2Kc + 1)^2 complex elements.  Only kz >= 0 is stored; the
 *     rest follows from F(-k) = F(k)^*.
 *   - Units: L in Mpc/h, k in h/Mpc, P in (Mpc/h)^3, B in (Mpc/h)^6;
 *     fields are dimensionless, u in Mpc/h.
 *   - D-form sources: the recursion uses div u = theta and u = grad phi to
 *     write the sources of Eq. 10 as S_delta = div(sum_m delta_m u_{n-m}) and
 *     S_theta = (1/2) lap(sum_m u_m . u_{n-m}); identical to the printed form
 *     whenever products do not alias (the 2/3 rule of Sec. II C).
 *
 * Memory.  Every pointer is a caller-owned device pointer unless marked
 * "host".  The library allocates no device memory: scratch comes in `work`
 * (device, 256-byte aligned) of at least the size the matching
 * *_workspace_bytes call returns.  Device pointers must be 256-byte aligned.
 * Calls are asynchronous on the stream given to gridspt_create; results are
 * ready when that stream has reached them (gridspt_sync waits).
 *
 * Errors.  Every entry point validates its arguments on the host before any
 * work is enqueued and returns a negative gridspt_status on failure, in which
 * case nothing has been written.  No exception crosses this interface.
 * A context is not thread-safe; use one per host thread and stream.
 */
#ifndef GRIDSPT_H
#define GRIDSPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GRIDSPT_OK = 0,
    GRIDSPT_EINVAL = -1,       /* an argument is out of range or inconsistent */
    GRIDSPT_EUNSUPPORTED = -2, /* valid, but not built: N not 2^a in [16, 1024] or 3 2^a in [48, 768], ... */
    GRIDSPT_EWORKSPACE = -3,   /* work is null or smaller than required */
    GRIDSPT_EALIGN = -4,       /* a device pointer is null or not 256-byte aligned */
    GRIDSPT_EHIP = -5,         /* the HIP runtime reported an error */
    GRIDSPT_ENONFINITE = -6    /* an input field holds a NaN or an infinity (only with GRIDSPT_CHECK_FINITE) */
} gridspt_status;

typedef enum { GRIDSPT_F32 = 0, GRIDSPT_F64 = 1 } gridspt_dtype;

typedef struct {
    int32_t n;     /* cells per side N: 2^a with 16 <= N <= 1024, or 3 2^a with 48 <= N <= 768 */
    int32_t dtype; /* gridspt_dtype of every real field and spectrum */
    double box;    /* side L > 0 [Mpc/h] */
    int32_t kc;    /* half-width of the spectral cube, 1 <= kc < N/2; every mask
                      used with this grid needs floor(sqrt(n2max)) <= kc */
    uint32_t flags; /* 0, or GRIDSPT_CHECK_FINITE; other bits are GRIDSPT_EINVAL */
} gridspt_grid;

/* Grid flags.
 * GRIDSPT_CHECK_FINITE: gridspt_forward, gridspt_orders, gridspt_orders_pform,
 *   gridspt_noise_field and gridspt_adjoint first check every real input field
 *   (delta1, field, noise, gdelta) on the device and return
 *   GRIDSPT_ENONFINITE, with nothing else enqueued, if any value is a NaN or
 *   an infinity.  The check waits for the context's stream (the call is then
 *   not asynchronous) and reads each input once more; it uses the first 256
 *   bytes of `work`.  Batches ignore the flag (they have no input fields). */
enum { GRIDSPT_CHECK_FINITE = 1 };

/* Linear power spectrum P0(k) = amp k^ns T_BBKS(k / gamma)^2 (k in h/Mpc,
 * Bardeen et al. 1986 transfer function), the growth factor multiplying the
 * field, the mask W1 and the seed of the white noise (Sec. II C, step 1). */
typedef struct {
    double amp;      /* A [(Mpc/h)^(3 + ns)] */
    double ns;       /* spectral index */
    double gamma;    /* shape parameter Gamma [h/Mpc] */
    double growth;   /* D, multiplies delta_1 */
    int64_t n2max;   /* W1: keep 0 < |n|^2 <= n2max */
    uint64_t seed;   /* Philox4x64-10 key word 0 */
    uint64_t stream; /* Philox counter word 1: realisation index */
} gridspt_linpk;

typedef struct gridspt_ctx gridspt_ctx;

/* Create a context bound to a HIP stream (hipStream_t passed as void*, NULL
 * for the null stream).  Needs no GPU; the device is the one current at the
 * first enqueue. */
int gridspt_create(gridspt_ctx** out, void* hip_stream);
void gridspt_destroy(gridspt_ctx* ctx);
/* Waits for the context's stream; GRIDSPT_EHIP if an asynchronous error occurred. */
int gridspt_sync(gridspt_ctx* ctx);
const char* gridspt_status_string(int status);
/* Library version (major * 10000 + minor * 100 + patch). */
int32_t gridspt_version(void);

/* ---- host helpers (exact integer arithmetic where ties are possible) ---- */

/* Mask threshold for a cut: kcut <= 0 selects the strict 2/3 rule of Sec. II C
 * (keep |n| < N/3: n2max = ceil(N^2 / 9) - 1); otherwise the absolute cut
 * |k| <= kcut: n2max = floor((kcut L / 2 pi)^2).  Returns < 0 on bad input. */
int64_t gridspt_cut_n2max(int32_t n, double box, double kcut);
/* floor(sqrt(n2max)), the cube half-width a mask needs; < 0 on bad input. */
int32_t gridspt_cube_kc(int64_t n2max);
/* Complex elements of one spectrum in the cube layout of `g`. */
int64_t gridspt_cube_elems(const gridspt_grid* g);
/* Linear bins on [0, k_max], k_max = (kmax_num / kmax_den) k_F, left-closed, the
 * last bin closed at min(k_max, cut): edge_n2[0] = 1 (k = 0 excluded),
 * edge_n2[b] = ceil((b k_max / nbins / k_F)^2), edge_n2[nbins] =
 * min(floor((k_max / k_F)^2) + 1, n2max + 1).  Bin b holds
 * edge_n2[b] <= |n|^2 < edge_n2[b+1].  edge_n2 is host memory of nbins + 1. */
int gridspt_linear_edges(int32_t nbins, int64_t kmax_num, int64_t kmax_den, int64_t n2max, int64_t* edge_n2);
/* Amplitude A giving sigma(R = 8 Mpc/h) = sigma8 for the uncut P0 (top-hat). */
int gridspt_sigma8_amp(double sigma8, double ns, double gamma, double* amp);
/* Linear growth D(z) / D(0) for matter and vacuum densities om, ol. */
int gridspt_growth(double om, double ol, double z, double* d);

/* ---- hot path ---- */

/* Device scratch needed by gridspt_linear_field, gridspt_forward,
 * gridspt_orders(nmax) and gridspt_orders_linear(nmax) on grid g, for calls
 * made with the grid flags `flags | g->flags` (unknown bits:
 * GRIDSPT_EINVAL).  Every workspace of this library already holds the 256
 * bytes GRIDSPT_CHECK_FINITE uses, so no current flag changes the size. */
int64_t gridspt_workspace_bytes(const gridspt_grid* g, int32_t nmax, uint32_t flags);

/* Step (1) of Sec. II C.  delta1(x) = inverse transform of
 * W1(k) sqrt(P0(k) N^3 / L^3) D w(k), where w(k) is the forward transform of
 * unit white noise w(x).  Cells c = (x N + y) N + z come in groups of four:
 * group q = c / 4 draws Philox4x64-10(counter = (q, stream, 0, 0),
 * key = (seed, 0)); its word pairs (w0, w1), (w2, w3) become 53-bit uniforms
 * in (0, 1) and Box-Muller gives two Gaussians per pair (cosine first); cell
 * 4q + r takes pair r / 2, branch r % 2.  So that
 * L^3 <|delta1(k)|^2> = D^2 P0(k) on kept modes and delta1(k=0) = 0.
 * delta1: N^3 real out.  delta1_k: cube-layout spectrum out, or NULL. */
int gridspt_linear_field(gridspt_ctx* ctx, const gridspt_grid* g, const gridspt_linpk* lp, void* delta1,
                         void* delta1_k, void* work, int64_t work_bytes);

/* Masked forward transform of any real field into the cube layout:
 * field_k(k) = [0 < |n|^2 <= n2max] N^-3 sum_x field(x) e^{-ik.x}. */
int gridspt_forward(gridspt_ctx* ctx, const gridspt_grid* g, int64_t n2max, const void* field, void* field_k,
                    void* work, int64_t work_bytes);

/* A cube-layout spectrum in the usual half layout of a real-to-complex
 * transform (the coefficients of Eq. 17): half is interleaved complex
 * [ix][iy][iz], N x N x (N/2 + 1) elements, ix and iy the grid positions of
 * signed modes (position i < N/2 is mode i, else i - N), iz = kz >= 0; every
 * mode outside the cube (|n_i| > Kc, and the Nyquist planes) is written as
 * zero.  For consumers that expect that layout (an inverse transform of
 * another library, numpy's irfftn); the library's own estimators read cubes.
 * The cube layout stays the library's output because every masked spectrum
 * lives inside it: at 1024^3 with the strict 2/3 cut a cube is 1.28 GB in
 * FP32 against 4.3 GB for the half layout. */
int gridspt_spectrum_half(gridspt_ctx* ctx, const gridspt_grid* g, const void* cube, void* half);

/* The recursion of Eq. 10 (n >= 2) and Eq. 11 (n = 1) up to nmax in [1, 5].
 * delta1: N^3 real input (any field; the mask W1 = n2max1 and the removal of
 *   k = 0 are applied here).  It may alias delta[0].
 * delta, theta: host arrays of nmax device pointers to N^3 real outputs;
 *   delta[0] receives the masked delta_1, theta[0] (may be NULL or alias
 *   delta[0]) the same field (theta_1 = delta_1).
 * delta_k, theta_k: NULL, or host arrays of nmax device pointers (entries may
 *   be NULL) receiving the cube-layout spectra of delta_n and theta_n.
 * Orders n >= 2 are masked with W2 (n2max2); both masks need
 * floor(sqrt(n2max)) <= g->kc. */
int gridspt_orders(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nmax, int64_t n2max1, int64_t n2max2,
                   const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
                   void* const* theta_k, void* work, int64_t work_bytes);

/* Device scratch of gridspt_orders_pform: the transform buffers, 15 real
 * fields per order below nmax, two real fields and two spectra. */
int64_t gridspt_pform_workspace_bytes(const gridspt_grid* g, int32_t nmax);

/* The recursion with the sources exactly as printed in Eq. 10 (the P-form):
 * S_delta = sum_m (grad delta_m).u_{n-m} + delta_m theta_{n-m},
 * S_theta = sum_m [d_j u_{m,k}][d_k u_{n-m,j}] + u_m.grad theta_{n-m},
 * built pointwise from the derived fields of Eq. 15/16 of every earlier
 * order (steps 2 and 5 of Sec. II C), then transformed and combined as in
 * gridspt_orders.  Same arguments and layouts as gridspt_orders (for n >= 2
 * delta_k[n-1] and theta_k[n-1] must differ).  It equals gridspt_orders
 * mode by mode when no product aliases (both masks inside the 2/3 rule) and
 * differs by the aliased terms otherwise (e.g. the paper's cuts of 1 and
 * 4/3 h/Mpc on 512^3 with L = 1000 Mpc/h). */
int gridspt_orders_pform(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nmax, int64_t n2max1, int64_t n2max2,
                         const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
                         void* const* theta_k, void* work, int64_t work_bytes);

/* Gaussian smoothing (Sec. III A-B) of cube-layout spectra into real fields:
 * out[j](x) = F^-1[exp(-k^2 R^2 / 2) S_j(k)], S_j = sum_{i <= j} coef[i] F_i
 * (cumulative != 0: the truncated series of Eq. 8, e.g. coef[i] = D^(i+1)) or
 * S_j = coef[j] F_j.  fields_k, out: host arrays of nfields <= 5 device
 * pointers; coef: host; radius R in Mpc/h (0: no smoothing).  Workspace as
 * gridspt_workspace_bytes(g, 1). */
int gridspt_smooth(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                   const double* coef, int32_t cumulative, double radius, void* const* out, void* work,
                   int64_t work_bytes);

/* Device scratch of gridspt_field_stats. */
int64_t gridspt_stats_workspace_bytes(int32_t nfields, int32_t nbins, int32_t nbins2);

/* One-point statistics of nfields <= 8 real fields of grid g (Sec. III B):
 *   moments  [nfields][4]: mean, variance (1/N^3), skewness, excess kurtosis;
 *   corr     [nfields][nfields]: Pearson correlation coefficients;
 *   counts   [nfields][nbins]: histogram, bin b = floor((x - lo) nbins / (hi - lo))
 *            evaluated in FP64, values with b outside [0, nbins) dropped (nbins <= 1024);
 *   joint    [nfields - 1][nbins2][nbins2]: joint histogram of field 0 (first index)
 *            and field j + 1 on the same range with nbins2 <= 64 bins per axis.
 * Each output pointer (device) may be NULL to skip it.  Sums are FP64 in a fixed
 * order; counts are exact integers (as doubles). */
int gridspt_field_stats(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nfields, const void* const* fields,
                        int32_t nbins, double lo, double hi, int32_t nbins2, double* moments, double* corr,
                        double* counts, double* joint, void* work, int64_t work_bytes);

/* gridspt_linear_field followed by gridspt_orders in one pass sequence: the
 * seeded linear field of lp (W1 = lp->n2max) is formed in Fourier space and
 * delta_1, u_1 are made from it directly (no inverse and forward transform of
 * delta_1 in between).  Outputs as gridspt_orders (delta[0] receives delta_1);
 * equal to the two calls up to rounding.  Workspace as gridspt_workspace_bytes. */
int gridspt_orders_linear(gridspt_ctx* ctx, const gridspt_grid* g, const gridspt_linpk* lp, int32_t nmax,
                          int64_t n2max2, void* const* delta, void* const* theta, void* const* delta_k,
                          void* const* theta_k, void* work, int64_t work_bytes);

/* Autotuner of the transform passes: runs gridspt_orders_linear once per
 * compiled launch variant of grid g (rows per block, radix split; FP32 grids
 * of 64..1024 and 96..384 have several) with every pass in that variant,
 * times each pass kind with HIP events, waits, and keeps the fastest variant
 * per kind in the context for this grid size and precision.  Later calls of
 * the context on such grids use it (results equal up to rounding).  Same
 * arguments as gridspt_orders_linear (the outputs are overwritten).  Returns
 * the number of variants tried. */
int gridspt_tune_orders(gridspt_ctx* ctx, const gridspt_grid* g, const gridspt_linpk* lp, int32_t nmax,
                        int64_t n2max2, void* const* delta, void* const* theta, void* const* delta_k,
                        void* const* theta_k, void* work, int64_t work_bytes);
/* Pins launch variant `variant` for every pass kind of grids of g's size and
 * precision in this context, replacing any autotuner choice.  The variant
 * changes only block shapes and radix splits, never results beyond rounding.
 * Variant 0 is always compiled; FP32 N = 64 .. 1024 (powers of two) also have
 * 1, 4, 5 and FP32 N = 96, 192, 384 have 1, 2.  Returns GRIDSPT_EINVAL for a
 * variant not compiled for the grid. */
int gridspt_set_tuning(gridspt_ctx* ctx, const gridspt_grid* g, int32_t variant);

/* The context's choice per tuned pass kind for grid g (variant 0 when not
 * tuned), with the tuner's time; names as for gridspt_profile_read. */
int gridspt_tuning(const gridspt_ctx* ctx, const gridspt_grid* g, int32_t max, char* names, int32_t* variant,
                   double* ms);

/* Final sum of orders (the truncated series of Eq. 8):
 * out(x) = sum_{n=1..nmax} coef[n-1] delta_n(x), accumulated in FP64.
 * delta: host array of nmax device pointers; coef: host array of nmax;
 * out: N^3 float64, device.  nmax <= 8. */
int gridspt_sum_orders(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nmax, const void* const* delta,
                       const double* coef, double* out);

/* Device scratch needed by gridspt_power: per-block partial sums and their
 * reduction for the most products one launch accumulates, which nbins sets
 * (npairs is checked but does not change the size). */
int64_t gridspt_power_workspace_bytes(const gridspt_grid* g, int32_t npairs, int32_t nbins);

/* Shell-averaged cross spectra, the estimators of Eq. 19-21 with the volume
 * factor: P_ab(bin) = L^3 sum_k w Re[F_a(k) F_b(k)^*] / sum_k w over stored
 * (kz >= 0) modes of the bin, w = 1 on kz = 0 and 2 elsewhere (so N_k counts
 * k and -k).  fields_k: host array of nfields (<= 16) device cube spectra.
 * pairs: host, 2 * npairs field indices (npairs <= 64).  edge_n2: host,
 * nbins + 1 non-decreasing integers, edge_n2[0] >= 1, nbins <= 256.
 * pk: device [npairs][nbins]; kmean, nmodes: device [nbins] or NULL.
 * Empty bins report 0.  Sums are FP64 in a fixed order. */
int gridspt_power(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                  int32_t npairs, const int32_t* pairs, int32_t nbins, const int64_t* edge_n2, double* pk,
                  double* kmean, double* nmodes, void* work, int64_t work_bytes);

/* gridspt_power for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments and results, without `work`.  Its scratch is a
 * library-owned array of 16 MiB per GPU (every GPU the library runs on holds
 * it until the process ends), enough for every valid call (at most about
 * 14.7 MB is used); a call needing more returns GRIDSPT_EWORKSPACE.  The call
 * allocates nothing.  All calls on one GPU share that GPU's array: calls that
 * overlap in time on one GPU (several streams or threads) race and must be
 * ordered by the caller. */
int gridspt_power_static(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                         int32_t npairs, const int32_t* pairs, int32_t nbins, const int64_t* edge_n2, double* pk,
                         double* kmean, double* nmodes);

/* Device scratch needed by gridspt_bispectrum for these triangles and terms
 * (room for the FP64 indicator transforms included). */
int64_t gridspt_bispectrum_workspace_bytes(const gridspt_grid* g, int32_t ntri, const int32_t* tri_bins,
                                           int32_t nterms, const int32_t* terms);

/* Closed-triangle bispectra of Eq. 22-23 by the FFT estimator:
 * I_a^b(x) = inverse transform of F_a restricted to shell b, J^b the same for
 * the indicator of shell b; for term (fa, fb, fc, tri) with shells (b1, b2, b3)
 *   T = N^-3 sum_x I_fa^b1 I_fb^b2 I_fc^b3,  ntriangles = N^-3 sum_x J^b1 J^b2 J^b3,
 *   bk = L^6 T / ntriangles.
 * The sum over x counts the triangles that close modulo N; Eq. 22-23 ask for
 * exact closure, k1 + k2 + k3 = 0.  The two agree when every component of
 * the sum lies in (-N, N), which holds when the outer radii of the three
 * shells (r_b = floor(sqrt(edge_n2[b + 1] - 1)), the largest |n| of shell b)
 * add up to less than N.  A triangle whose radii reach N or more is rejected
 * with GRIDSPT_EINVAL (under the strict 2/3 cut every shell has r_b < N/3 and
 * never is).
 * ntriangles is an exact integer count of ordered closed triangles: the
 * indicator transforms and their triple sums run in FP64 whatever the grid's
 * precision, and the count is rounded to the nearest integer.
 * tri_bins: host 3 * ntri bin indices (ntri <= 4096); terms: host 4 * nterms
 * (fa, fb, fc, tri), nterms <= 16384;
 * edge_n2 as for gridspt_power.  bk: device [nterms]; ntriangles: device
 * [ntri].  Sums are FP64 in a fixed order. */
int gridspt_bispectrum(gridspt_ctx* ctx, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                       int32_t ntri, const int32_t* tri_bins, int32_t nterms, const int32_t* terms, int32_t nbins,
                       const int64_t* edge_n2, double* bk, double* ntriangles, void* work, int64_t work_bytes);

/* ---- reverse mode (gradients with respect to the white noise) ---- */

/* Step (1) of Sec. II C from a given white-noise field: as
 * gridspt_linear_field, with w(x) = noise (N^3 real, device) instead of the
 * Philox draw (lp->seed and lp->stream are unused). */
int gridspt_noise_field(gridspt_ctx* ctx, const gridspt_grid* g, const gridspt_linpk* lp, const void* noise,
                        void* delta1, void* delta1_k, void* work, int64_t work_bytes);

/* Device scratch of gridspt_adjoint: the transform buffers plus
 * 8 (nmax - 1) + 4 real fields. */
int64_t gridspt_adjoint_workspace_bytes(const gridspt_grid* g, int32_t nmax);

/* Reverse mode of noise -> delta_1 .. delta_nmax, i.e. gridspt_noise_field
 * followed by gridspt_orders(nmax, lp->n2max, n2max2): for a scalar objective
 * J of the delta_n alone, given gdelta[n-1] = dJ/d delta_n(x) (host array of
 * nmax device N^3 real fields), writes gnoise = dJ/dw(x) (N^3 real).  Every
 * step of the recursion is a spectral multiply, whose adjoint multiplies by
 * the complex-conjugate multiplier, or a pointwise product, whose adjoint is
 * the transposed product; the order-n step (Eq. 10) uses the transposed
 * matrix [[n + 1/2, 3/2], [1, n]].
 * Checkpoints: delta_k[m], theta_k[m] for m < nmax - 1 are the cube-layout
 * spectra of delta_(m+1), theta_(m+1) as gridspt_orders stored them in the
 * forward run (theta_k[0] is unused: theta_1 = delta_1; theta_k may be NULL
 * when nmax <= 2); delta_m and u_m are regenerated from them.  Inputs are
 * not modified. */
int gridspt_adjoint(gridspt_ctx* ctx, const gridspt_grid* g, const gridspt_linpk* lp, int32_t nmax, int64_t n2max2,
                    const void* const* delta_k, const void* const* theta_k, const void* const* gdelta, void* gnoise,
                    void* work, int64_t work_bytes);

/* ---- batched realisations in one captured graph ----
 * Many independent realisations, of several grid sizes, computed by one HIP
 * graph: every pass of a size class is one launch over all its realisations
 * (realisation r of a class uses the buffers of realisation 0 shifted by a
 * fixed byte stride), and the size classes are independent branches of the
 * graph.  Each realisation runs the linear field (step 1 of Sec. II C, Philox
 * stream lin.stream + r), orders 1..nmax, the cross spectra of its delta_n and,
 * optionally, bispectra; the graph ends with the realisation mean and sample
 * standard deviation of every spectrum bin and bispectrum term (the
 * realisation averages of Sec. IV). */
typedef struct {
    gridspt_grid grid;       /* size class; grid.kc must hold both masks; grid.flags is ignored */
    int32_t nreal;           /* realisations >= 1 */
    int32_t nmax;            /* orders 1..nmax, nmax in [1, 5] */
    int64_t n2max2;          /* W2 of orders n >= 2 (W1 is lin.n2max) */
    gridspt_linpk lin;       /* spectrum, growth, W1, seed; realisation r uses stream lin.stream + r */
    int32_t npairs;          /* cross spectra P_ab of delta_(a+1), delta_(b+1); 1..64 */
    const int32_t* pairs;    /* host, 2 * npairs indices in [0, nmax) */
    int32_t nbins;           /* spectrum bins, 1..256 */
    const int64_t* edge_n2;  /* host, nbins + 1, as for gridspt_power */
    int32_t ntri;            /* bispectrum triangles, 0 for none */
    const int32_t* tri_bins; /* host, 3 * ntri bins of edge_n2 (closure rule of gridspt_bispectrum) */
    int32_t nterms;          /* bispectrum terms */
    const int32_t* terms;    /* host, 4 * nterms (fa, fb, fc, tri), fields in [0, nmax) */
} gridspt_batch_group;

/* Device outputs of one group (NULL entries are skipped). */
typedef struct {
    double* pk_mean;    /* [npairs][nbins] realisation mean of P_ab */
    double* pk_std;     /* [npairs][nbins] sample standard deviation */
    double* kmean;      /* [nbins] */
    double* nmodes;     /* [nbins] */
    double* bk_mean;    /* [nterms] */
    double* bk_std;     /* [nterms] */
    double* ntriangles; /* [ntri] */
} gridspt_batch_out;

typedef struct gridspt_batch gridspt_batch;

enum {
    GRIDSPT_BATCH_TUNE = 1, /* autotune the launch variant of every pass kind per group */
    GRIDSPT_BATCH_EAGER = 2 /* no graph: gridspt_batch_run enqueues the launches directly */
};

/* Device scratch of a batch (all realisations' fields, spectra and scratch). */
int64_t gridspt_batch_workspace_bytes(int32_t ngroups, const gridspt_batch_group* groups);
/* Validate the groups, lay out `work`, run the autotuner if asked (it
 * enqueues and waits for complete trial runs, overwriting `work`), and
 * capture the graph.  Host arrays of the groups are copied; `outs` (host
 * array of ngroups) and `work` must stay valid for the batch's life. */
int gridspt_batch_create(gridspt_ctx* ctx, int32_t ngroups, const gridspt_batch_group* groups,
                         const gridspt_batch_out* outs, void* work, int64_t work_bytes, uint32_t flags,
                         gridspt_batch** out);
/* Launch the whole batch (one graph launch) on the context's stream. */
int gridspt_batch_run(gridspt_batch* b);
void gridspt_batch_destroy(gridspt_batch* b);

enum {
    GRIDSPT_BATCH_DELTA = 0,   /* delta_n(x) of a realisation, N^3 real; index = n - 1 */
    GRIDSPT_BATCH_THETA = 1,   /* theta_n(x), index = n - 1 (n = 1 gives delta_1) */
    GRIDSPT_BATCH_DELTA_K = 2, /* cube-layout spectrum of delta_n, index = n - 1 */
    GRIDSPT_BATCH_PK = 3,      /* the realisation's P_ab, [npairs][nbins] doubles; index 0 */
    GRIDSPT_BATCH_BK = 4       /* the realisation's bispectrum terms, [nterms] doubles; index 0 */
};
/* Device address, inside `work`, of one realisation's buffer `what`. */
int gridspt_batch_buffer(const gridspt_batch* b, int32_t group, int32_t real, int32_t what, int32_t index,
                         void** ptr);
/* The launch variant chosen per pass kind for a group (0 without tuning),
 * with the tuner's time for it: up to max kinds; names as for
 * gridspt_profile_read; ms may be NULL.  Returns the number of kinds. */
int gridspt_batch_tuning(const gridspt_batch* b, int32_t group, int32_t max, char* names, int32_t* variant,
                         double* ms);

/* ---- kernel timing ----
 * With profiling on, every kernel the context enqueues is bracketed by HIP
 * events on its stream.  gridspt_profile_read waits for the stream, then
 * reports per kernel kind (up to max entries): name (host, 32 bytes each,
 * NUL-terminated), launches, total milliseconds and the algorithmic bytes the
 * launches move (inputs read once, outputs written once, in the layouts
 * above).  Returns the number of kinds reported; reading resets the record. */
int gridspt_set_profiling(gridspt_ctx* ctx, int32_t enable);
int gridspt_profile_read(gridspt_ctx* ctx, int32_t max, char* names, int64_t* launches, double* ms, double* bytes);
/* The same launches grouped by the order of the recursion they belong to, as
 * of the last gridspt_profile_read: ms[i] and bytes[i] (host, max entries) for
 * order i, where order 1 includes the linear field of gridspt_orders_linear,
 * the product pass of order n >= 2 (which also finishes the z inverse of
 * order n - 1) counts for order n, and index 0 collects launches of no order
 * (estimators, sums).  Returns the highest order with launches. */
int gridspt_profile_orders(const gridspt_ctx* ctx, int32_t max, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* GRIDSPT_H */

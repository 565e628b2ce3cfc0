// The five pass kernels of one GridSPT order (Sec. II C, steps 2-6) and the
// linear-field variants of step 1, specialised per precision T and grid size N.
//
// Every pass reads whole rows along the axis it transforms (contiguous in
// HBM) and, except the last, writes its result transposed so that the next
// pass again reads contiguous rows.  The transposition goes through LDS: a
// block holds RPB rows, and writes RPB consecutive elements of each output row.
//
// Pruning: every field after a forward transform is masked to |n|^2 <= n2max
// with n2max < (N/2)^2, so only the cube |n_i| <= Kc (Kc = floor(sqrt(n2max)))
// is ever non-zero.  Forward passes store only that range, inverse passes read
// only that range.  Spectral layouts (complex, "fftfreq" order for signed
// indices: i' <= Kc is +i', i' > Kc is i' - (2Kc+1)):
//   S1 [kz][x][y]    Kz x N  x N      after the z pass        (Kz = Kc + 1)
//   S2 [kz][ky][x]   Kz x Ky x N      after the y pass        (Ky = 2Kc + 1)
//   S3 [kz][x][ky]   Kz x N  x Ky     after the fused x pass
//   S4 [x][y][kz]    N  x N  x Kz     after the inverse y pass
//   cube [kz][ky][kx] Kz x Ky x Kx    the spectra handed to the caller
// Real fields are [x][y][z], z contiguous.
#pragma once
#include "fft_engine.hpp"

namespace gridspt {

template <typename T, int N>
struct Rows {
    // rows per block: about 64 KB of LDS, at most 32 rows, at most N rows
    static constexpr int bytes = 65536 / (N * (int)sizeof(cpx<T>));
    static constexpr int RPB0 = bytes < 1 ? 1 : (bytes > 32 ? 32 : bytes);
    static constexpr int RPB = RPB0 > N ? N : RPB0;
    static constexpr int P = N / 16;
    static constexpr int THREADS = RPB * P;
    static constexpr int ROWE = lds_row_elems(N);
};

// signed mode index of FFT position p on an N grid
__device__ __forceinline__ int signed_pos(int p, int n) { return p < n / 2 ? p : p - n; }
// position (0..N-1) of compact fftfreq index i' of a (2Kc+1)-long axis
__device__ __forceinline__ int compact_to_pos(int ic, int Kc, int n) { return ic <= Kc ? ic : n - (2 * Kc + 1) + ic; }
// compact index of position p, or -1 if |n| > Kc
__device__ __forceinline__ int pos_to_compact(int p, int Kc, int n) {
    if (p <= Kc) return p;
    if (p >= n - Kc) return p - n + 2 * Kc + 1;
    return -1;
}

// --------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and Box-Muller: unit Gaussian of a cell.
// counter = (cell, stream, 0, 0), key = (seed, 0); two 53-bit uniforms in (0,1).
// --------------------------------------------------------------------------
__device__ __forceinline__ double cell_gaussian(uint64_t seed, uint64_t stream, uint64_t cell) {
    uint64_t c0 = cell, c1 = stream, c2 = 0, c3 = 0;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const uint64_t lo0 = 0xD2E7470EE14C6C93ull * c0, hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
        const uint64_t lo1 = 0xCA5A826395121157ull * c2, hi1 = __umul64hi(0xCA5A826395121157ull, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    const double u1 = ((double)(c0 >> 11) + 0.5) * 0x1p-53;
    const double u2 = ((double)(c1 >> 11) + 0.5) * 0x1p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.28318530717958647692528676655900577 * u2);
}

// Linear amplitude sqrt(P0(k) N^3 / L^3) D, P0 = A k^ns T(k / Gamma)^2 with the
// BBKS transfer function (Bardeen, Bond, Kaiser & Szalay 1986, Eq. G3).
struct LinParams {
    double amp, ns, gamma, growth, vol;  // vol = N^3 / L^3
};
__device__ __forceinline__ double lin_amplitude(double k, const LinParams& p) {
    const double q = k / p.gamma;
    const double a = 2.34 * q;
    const double t = log1p(a) / a *
                     pow(1.0 + 3.89 * q + (16.1 * q) * (16.1 * q) + (5.46 * q) * (5.46 * q) * (5.46 * q) +
                             (6.71 * q) * (6.71 * q) * (6.71 * q) * (6.71 * q),
                         -0.25);
    const double p0 = p.amp * pow(k, p.ns) * t * t;
    return sqrt(p0 * p.vol) * p.growth;
}

// --------------------------------------------------------------------------
// shared pieces
// --------------------------------------------------------------------------

// canonical registers of one row -> this row's LDS buffer in natural order
template <int N, typename T>
__device__ __forceinline__ void stage_row(const cpx<T> (&v)[16], cpx<T>* row, int l) {
    constexpr int P = N / 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) row[lds_pad(l + P * e)] = v[e];
}

// --------------------------------------------------------------------------
// P1: z pass, forward.  Block = RPB consecutive y at one x.
// SRC 0: one real field; SRC 1: Gaussian noise generated in place;
// SRC 2: the products of order n (V = sum delta_m u_{n-m}, W = sum u_m.u_{n-m}).
// Output S1 fields.
// --------------------------------------------------------------------------
template <typename T>
struct ProductInputs {
    const T* d[4];     // delta_1 .. delta_{n-1}
    const T* u[4][3];  // u_1 .. u_{n-1}
};

// SRC 2, order NORD: every input field is read once per cell; V and W are
// formed in registers and packed as a = V_x + i V_y, b = V_z + i W.
template <typename T, int NORD>
__device__ __forceinline__ void load_products(const ProductInputs<T>& pin, size_t c, cpx<T>& a, cpx<T>& b) {
    T d[NORD], u[NORD][3];
#pragma unroll
    for (int m = 1; m < NORD; ++m) {
        d[m] = pin.d[m - 1][c];
#pragma unroll
        for (int j = 0; j < 3; ++j) u[m][j] = pin.u[m - 1][j][c];
    }
    T vx = 0, vy = 0, vz = 0, w = 0;
#pragma unroll
    for (int m = 1; m < NORD; ++m) {
        vx += d[m] * u[NORD - m][0];
        vy += d[m] * u[NORD - m][1];
        vz += d[m] * u[NORD - m][2];
        w += u[m][0] * u[NORD - m][0] + u[m][1] * u[NORD - m][1] + u[m][2] * u[NORD - m][2];
    }
    a = {vx, vy};
    b = {vz, w};
}

template <typename T, int N, int SRC, int NORD>
__global__ __launch_bounds__((Rows<T, N>::THREADS)) void k_zfwd(const T* __restrict__ f, ProductInputs<T> pin,
                                                               uint64_t seed, uint64_t stream, cpx<T>* __restrict__ s1,
                                                               size_t s1_field, const cpx<T>* __restrict__ tw, int Kz) {
    using RW = Rows<T, N>;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE;
    __shared__ cpx<T> lds[RPB * ROWE];
    const uint32_t groups = N / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, N * groups);
    const int x = blk / groups, y0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const size_t rowbase = ((size_t)x * N + (y0 + r)) * N;
    cpx<T>* row = lds + r * ROWE;

    cpx<T> a[16], b[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const size_t c = rowbase + l + P * e;
        if constexpr (SRC == 0) {
            a[e] = {f[c], (T)0};
        } else if constexpr (SRC == 1) {
            a[e] = {(T)cell_gaussian(seed, stream, c), (T)0};
        } else {
            load_products<T, NORD>(pin, c, a[e], b[e]);
        }
    }

    constexpr int NPACK = (SRC == 2) ? 2 : 1;
    static_for<NPACK>([&](auto pkc) {
        constexpr int pk = decltype(pkc)::value;
        cpx<T> v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = pk == 0 ? a[e] : b[e];
        if constexpr (pk > 0) __syncthreads();  // previous read-out has finished with LDS
        fft_row<N, -1, T>(v, row, tw, l);
        stage_row<N, T>(v, row, l);
        __syncthreads();
        // read-out: element (kz, y0 + rr) of every row
        for (int idx = threadIdx.x; idx < Kz * RPB; idx += RW::THREADS) {
            const int kz = idx / RPB, rr = idx % RPB;
            const cpx<T> c = lds[rr * ROWE + lds_pad(kz)];
            const size_t o = ((size_t)kz * N + x) * N + y0 + rr;
            if constexpr (SRC == 2) {
                // two real fields packed as c = A + iB:
                // A(k) = (C(k) + C(-k)^*) / 2,  B(k) = (C(k) - C(-k)^*) / 2i
                const cpx<T> m = lds[rr * ROWE + lds_pad((N - kz) & (N - 1))];
                const cpx<T> A = {(T)0.5 * (c.x + m.x), (T)0.5 * (c.y - m.y)};
                const cpx<T> B = {(T)0.5 * (c.y + m.y), (T)0.5 * (m.x - c.x)};
                s1[(size_t)(2 * pk) * s1_field + o] = A;
                s1[(size_t)(2 * pk + 1) * s1_field + o] = B;
            } else {
                s1[o] = c;
            }
        }
    });
}

// --------------------------------------------------------------------------
// P2: y pass, forward.  Rows (kz, x) of S1; block = RPB consecutive x at one
// kz; grid.y = field.  Keeps |ky| <= Kc and writes S2 [kz][ky'][x].
// --------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__((Rows<T, N>::THREADS)) void k_yfwd(const cpx<T>* __restrict__ s1, size_t s1_field,
                                                               cpx<T>* __restrict__ s2, size_t s2_field,
                                                               const cpx<T>* __restrict__ tw, CubeDims cd) {
    using RW = Rows<T, N>;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE;
    __shared__ cpx<T> lds[RPB * ROWE];
    const uint32_t groups = N / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, x0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const cpx<T>* in = s1 + (size_t)blockIdx.y * s1_field + ((size_t)kz * N + x0 + r) * N;
    cpx<T>* out = s2 + (size_t)blockIdx.y * s2_field;
    cpx<T>* row = lds + r * ROWE;
    cpx<T> v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = in[l + P * e];
    fft_row<N, -1, T>(v, row, tw, l);
    stage_row<N, T>(v, row, l);
    __syncthreads();
    for (int idx = threadIdx.x; idx < cd.Ky * RPB; idx += RW::THREADS) {
        const int ky = idx / RPB, rr = idx % RPB;
        out[((size_t)kz * cd.Ky + ky) * N + x0 + rr] = lds[rr * ROWE + lds_pad(compact_to_pos(ky, cd.Kc, N))];
    }
}

// --------------------------------------------------------------------------
// P3: x pass, fused.  Rows (kz, ky') of S2; block = RPB consecutive ky' at one
// kz.  Forward x transform, the k-space step, optional cube stores, then the
// inverse x transform of every output field, written transposed to S3.
// --------------------------------------------------------------------------
enum XMode { XM_ORDER = 0, XM_ORDER1 = 1, XM_LINEAR = 2, XM_FORWARD = 3 };

template <typename T>
struct XArgs {
    const cpx<T>* s2;
    size_t s2_field;
    cpx<T>* s3;
    size_t s3_field;
    cpx<T>* cube_d;  // may be null
    cpx<T>* cube_t;  // may be null
    int n, nout;     // order; number of output fields (written as S3 fields 0..nout-1)
    int64_t n2max;   // mask of this order
    double kF, invN3;
    LinParams lin;
};

template <typename T, int N, int MODE>
__global__ __launch_bounds__((Rows<T, N>::THREADS)) void k_xfused(XArgs<T> a, const cpx<T>* __restrict__ tw,
                                                                 CubeDims cd) {
    using RW = Rows<T, N>;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE;
    __shared__ cpx<T> lds[RPB * ROWE];
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    cpx<T>* row = lds + r * ROWE;
    const size_t rowoff = ((size_t)kz * cd.Ky + (active ? kyc : 0)) * N;

    // k-space step: sd holds delta_n(k), st holds theta_n(k) afterwards
    cpx<T> sd[16], st[16];
    const int nin = (MODE == XM_ORDER) ? 4 : 1;
#pragma unroll
    for (int e = 0; e < 16; ++e) sd[e] = st[e] = {(T)0, (T)0};
    for (int f = 0; f < nin; ++f) {
        cpx<T> v[16];
        const cpx<T>* in = a.s2 + (size_t)f * a.s2_field + rowoff;
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = active ? in[l + P * e] : cpx<T>{(T)0, (T)0};
        fft_row<N, -1, T>(v, row, tw, l);
        if constexpr (MODE == XM_ORDER) {
            if (f < 3) {
                // S_delta += i k_f V_f(k)  (kF and N^-3 applied below)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int kx = signed_pos(l + P * e, N);
                    const T kf = (T)(f == 0 ? kx : (f == 1 ? ky : kz));
                    sd[e] = cadd(sd[e], cscale(cmul_i(v[e]), kf));
                }
            } else {
#pragma unroll
                for (int e = 0; e < 16; ++e) st[e] = v[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) sd[e] = v[e];
        }
    }

    const T kF = (T)a.kF, invN3 = (T)a.invN3;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int kx = signed_pos(l + P * e, N);
        const int64_t n2 = (int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz;
        const bool keep = active && n2 > 0 && n2 <= a.n2max;
        if constexpr (MODE == XM_ORDER) {
            // S_delta = i k.V(k) N^-3, S_theta = -(k^2/2) W(k) N^-3 (divergence form of Eq. 10)
            const cpx<T> sdel = cscale(sd[e], kF * invN3);
            const cpx<T> sthe = cscale(st[e], (T)(-0.5) * kF * kF * (T)n2 * invN3);
            const T cn = (T)(2.0 / ((2.0 * a.n + 3.0) * (a.n - 1.0)));
            const T m00 = cn * (T)(a.n + 0.5), m01 = cn, m10 = cn * (T)1.5, m11 = cn * (T)a.n;
            const cpx<T> dn = {m00 * sdel.x + m01 * sthe.x, m00 * sdel.y + m01 * sthe.y};
            const cpx<T> tn = {m10 * sdel.x + m11 * sthe.x, m10 * sdel.y + m11 * sthe.y};
            sd[e] = keep ? dn : cpx<T>{(T)0, (T)0};
            st[e] = keep ? tn : cpx<T>{(T)0, (T)0};
        } else if constexpr (MODE == XM_LINEAR) {
            T s = (T)0;
            if (keep) s = (T)(lin_amplitude(a.kF * sqrt((double)n2), a.lin) * a.invN3);
            sd[e] = cscale(sd[e], s);
            st[e] = sd[e];
        } else {
            sd[e] = keep ? cscale(sd[e], invN3) : cpx<T>{(T)0, (T)0};
            st[e] = sd[e];
        }
    }

    // cube stores (masked spectra), kept kx only
    if (active && (a.cube_d || a.cube_t)) {
        const size_t cbase = ((size_t)kz * cd.Ky + kyc) * cd.Ky;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int ic = pos_to_compact(l + P * e, cd.Kc, N);
            if (ic >= 0) {
                if (a.cube_d) a.cube_d[cbase + ic] = sd[e];
                if (a.cube_t) a.cube_t[cbase + ic] = st[e];
            }
        }
    }
    if constexpr (MODE == XM_FORWARD) return;

    // outputs: 0 delta, 1 theta (or u_x for order 1), then u components
    for (int o = 0; o < a.nout; ++o) {
        cpx<T> v[16];
        // field o: ORDER: {delta, theta, ux, uy, uz}; ORDER1: {delta, ux, uy, uz}; LINEAR: {delta}
        const int comp = (MODE == XM_ORDER) ? o - 2 : o - 1;  // velocity component, < 0 for delta/theta
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if (comp < 0) {
                v[e] = (MODE == XM_ORDER && o == 1) ? st[e] : sd[e];
            } else {
                // u_j(k) = (-i k_j / k^2) theta(k)
                const int kx = signed_pos(l + P * e, N);
                const int64_t n2 = (int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz;
                const int kj = comp == 0 ? kx : (comp == 1 ? ky : kz);
                const T s = n2 > 0 ? (T)((double)kj / (a.kF * (double)n2)) : (T)0;
                const cpx<T> t = st[e];
                v[e] = {t.y * s, -t.x * s};
            }
        }
        __syncthreads();  // previous field's read-out is done with LDS
        fft_row<N, +1, T>(v, row, tw, l);
        stage_row<N, T>(v, row, l);
        __syncthreads();
        cpx<T>* out = a.s3 + (size_t)o * a.s3_field;
        const int nrows = min(RPB, cd.Ky - ky0);
        for (int idx = threadIdx.x; idx < N * RPB; idx += RW::THREADS) {
            const int x = idx / RPB, rr = idx % RPB;
            if (rr < nrows) out[((size_t)kz * N + x) * cd.Ky + ky0 + rr] = lds[rr * ROWE + lds_pad(x)];
        }
    }
}

// --------------------------------------------------------------------------
// P3 for shell-filtered fields (bispectrum): rows (kz, ky') of a cube, kept
// when lo <= n^2 < hi; the field pointer may be null for the indicator 1_b.
// Inverse x transform, written transposed to S3.  grid.y = slot.
// --------------------------------------------------------------------------
template <typename T>
struct ShellSlots {
    const cpx<T>* cube[8];
    int64_t lo[8], hi[8];
    cpx<T>* s3;
    size_t s3_field;
};

template <typename T, int N>
__global__ __launch_bounds__((Rows<T, N>::THREADS)) void k_xshell(ShellSlots<T> a, const cpx<T>* __restrict__ tw,
                                                                 CubeDims cd) {
    using RW = Rows<T, N>;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE;
    __shared__ cpx<T> lds[RPB * ROWE];
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    const int slot = blockIdx.y;
    const cpx<T>* cube = a.cube[slot];
    const size_t cbase = ((size_t)kz * cd.Ky + (active ? kyc : 0)) * cd.Ky;
    cpx<T>* row = lds + r * ROWE;
    cpx<T> v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int p = l + P * e;
        const int ic = pos_to_compact(p, cd.Kc, N);
        const int kx = signed_pos(p, N);
        const int64_t n2 = (int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz;
        const bool in = active && ic >= 0 && n2 >= a.lo[slot] && n2 < a.hi[slot];
        cpx<T> c = {(T)0, (T)0};
        if (in) c = cube ? cube[cbase + ic] : cpx<T>{(T)1, (T)0};
        v[e] = c;
    }
    fft_row<N, +1, T>(v, row, tw, l);
    stage_row<N, T>(v, row, l);
    __syncthreads();
    cpx<T>* out = a.s3 + (size_t)slot * a.s3_field;
    const int nrows = min(RPB, cd.Ky - ky0);
    for (int idx = threadIdx.x; idx < N * RPB; idx += RW::THREADS) {
        const int x = idx / RPB, rr = idx % RPB;
        if (rr < nrows) out[((size_t)kz * N + x) * cd.Ky + ky0 + rr] = lds[rr * ROWE + lds_pad(x)];
    }
}

// --------------------------------------------------------------------------
// P4: y pass, inverse.  Rows (kz, x) of S3 (Ky values, zero-extended to N);
// block = RPB consecutive kz at one x; grid.y = field.  Writes S4 [x][y][kz].
// --------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__((Rows<T, N>::THREADS)) void k_yinv(const cpx<T>* __restrict__ s3, size_t s3_field,
                                                               cpx<T>* __restrict__ s4, size_t s4_field,
                                                               const cpx<T>* __restrict__ tw, CubeDims cd) {
    using RW = Rows<T, N>;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE;
    __shared__ cpx<T> lds[RPB * ROWE];
    const uint32_t groups = (cd.Kz + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, N * groups);
    const int x = blk / groups, kz0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const bool active = kz0 + r < cd.Kz;
    const cpx<T>* in = s3 + (size_t)blockIdx.y * s3_field + ((size_t)(active ? kz0 + r : 0) * N + x) * cd.Ky;
    cpx<T>* row = lds + r * ROWE;
    cpx<T> v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int ic = pos_to_compact(l + P * e, cd.Kc, N);
        v[e] = (active && ic >= 0) ? in[ic] : cpx<T>{(T)0, (T)0};
    }
    fft_row<N, +1, T>(v, row, tw, l);
    stage_row<N, T>(v, row, l);
    __syncthreads();
    cpx<T>* out = s4 + (size_t)blockIdx.y * s4_field;
    const int nrows = min(RPB, cd.Kz - kz0);
    for (int idx = threadIdx.x; idx < N * RPB; idx += RW::THREADS) {
        const int y = idx / RPB, rr = idx % RPB;
        if (rr < nrows) out[((size_t)x * N + y) * cd.Kz + kz0 + rr] = lds[rr * ROWE + lds_pad(y)];
    }
}

// --------------------------------------------------------------------------
// P5: z pass, inverse to real.  Rows (x, y) of S4 (Kz values).  Two real
// outputs per complex transform: C(k) = A(k) + i B(k) for k in [0, Kz),
// C(-k) = A(k)^* + i B(k)^*; then a(z) = Re c(z), b(z) = Im c(z).
// grid.y = pair; block = RPB consecutive rows.
// --------------------------------------------------------------------------
template <typename T>
struct ZPairs {
    int fa[3], fb[3];  // S4 field indices (fb < 0: none)
    T* outa[3];
    T* outb[3];
};

template <typename T, int N>
__global__ __launch_bounds__((Rows<T, N>::THREADS)) void k_zinv(const cpx<T>* __restrict__ s4, size_t s4_field,
                                                               ZPairs<T> zp, const cpx<T>* __restrict__ tw,
                                                               CubeDims cd) {
    using RW = Rows<T, N>;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE;
    __shared__ cpx<T> lds[RPB * ROWE];
    const int pair = blockIdx.y;
    const uint32_t nblk = (uint32_t)((size_t)N * N / RPB);
    const uint32_t blk = xcd_block(blockIdx.x, nblk);
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const size_t q = (size_t)blk * RPB + r;  // row index x N + y
    const cpx<T>* A = s4 + (size_t)zp.fa[pair] * s4_field + q * cd.Kz;
    const bool hasb = zp.fb[pair] >= 0;
    const cpx<T>* B = s4 + (size_t)(hasb ? zp.fb[pair] : 0) * s4_field + q * cd.Kz;
    cpx<T>* row = lds + r * ROWE;
    cpx<T> v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int p = l + P * e;
        cpx<T> c = {(T)0, (T)0};
        if (p < cd.Kz) {
            const cpx<T> av = A[p];
            const cpx<T> bv = hasb ? B[p] : cpx<T>{(T)0, (T)0};
            c = {av.x - bv.y, av.y + bv.x};
        } else if (p > N - cd.Kz) {
            const cpx<T> av = A[N - p];
            const cpx<T> bv = hasb ? B[N - p] : cpx<T>{(T)0, (T)0};
            c = {av.x + bv.y, bv.x - av.y};
        }
        v[e] = c;
    }
    fft_row<N, +1, T>(v, row, tw, l);
    T* oa = zp.outa[pair] + q * N;
#pragma unroll
    for (int e = 0; e < 16; ++e) oa[l + P * e] = v[e].x;
    if (hasb) {
        T* ob = zp.outb[pair] + q * N;
#pragma unroll
        for (int e = 0; e < 16; ++e) ob[l + P * e] = v[e].y;
    }
}

}  // namespace gridspt

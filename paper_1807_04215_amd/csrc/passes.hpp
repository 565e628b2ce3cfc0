// The five pass kernels of one GridSPT order (Sec. II C, steps 2-6) and the
// linear-field variants of step 1, specialised per precision T and grid size N.
//
// Every pass writes the rows it transforms contiguously (each lane stores its
// points straight from registers), and every pass after the first reads its
// rows transposed: a block holds RPB rows that are RPB consecutive elements of
// the previous layout, loads those short runs for every position along the
// axis and regroups them into rows through LDS.  Scattered short stores cost
// about twice what scattered short loads cost on this memory system, so the
// transposition sits on the load side.
//
// Pruning: every field after a forward transform is masked to |n|^2 <= n2max
// with n2max < (N/2)^2, so only the cube |n_i| <= Kc (Kc = floor(sqrt(n2max)))
// is ever non-zero.  Forward passes store only that range, inverse passes read
// only that range.  Spectral layouts (complex, "fftfreq" order for signed
// indices: i' <= Kc is +i', i' > Kc is i' - (2Kc+1)):
//   S1 [x][kz/TZ][y][kz%TZ]           after the z pass        (Kz = Kc + 1)
//                    N  x Kz x N, in tiles of TZ kz (the last tile narrower)
//   S2 [kz][x][ky]   Kz x N  x Ky     after the y pass        (Ky = 2Kc + 1)
//                    rows s2_row apart (Ky rounded up to a multiple of 16)
//   S3 [kz][ky][x]   Kz x Ky x N      after the fused x pass
//   S4 [x][kz][y]    N  x Kz x N      after the inverse y pass
//   cube [kz][ky][kx] Kz x Ky x Kx    the spectra handed to the caller
// Real fields are [x][y][z], z contiguous.  S1 is tiled because the z pass
// (rows (x, y)) and the y pass (rows (x, kz)) both hold one x per block: a z
// pass block stores a whole block of y for every tile, and a y pass block
// reads one whole tile.
//
// Real data along z is transformed two rows (or two fields) per complex FFT:
// c = a + i b gives A(k) = (C(k) + C(-k)^*) / 2 and B(k) = (C(k) - C(-k)^*) / 2i,
// and in reverse C(k) = A(k) + i B(k), C(-k) = A(k)^* + i B(k)^*.
//
// Addressing: the rows a block touches start at a block-uniform base pointer;
// the bulk loads and stores add a 32-bit per-lane offset to it, so they use
// the scalar base + vector offset form and need no 64-bit address registers.
#pragma once
#include "fft_engine.hpp"

namespace gridspt {

constexpr int pow2_floor(int v) {
    int p = 1;
    while (2 * p <= v) p *= 2;
    return p;
}

// Row stride (elements of `dw` dwords) at least `minimum` whose dword offset
// between consecutive rows is 64 / RPB modulo 64: a transposed scatter, in
// which consecutive lanes write the same position of consecutive rows, then
// writes 64 distinct banks per 256 bytes.  `minimum` where that is impossible.
constexpr int spread_stride(int minimum, int rpb, int dw) {
    const int m = 64 / dw;  // elements per 64 dwords
    if (rpb > 64 / dw || (64 / rpb) % dw != 0) return minimum;
    const int want = 64 / rpb / dw;
    return minimum + ((want - minimum % m) % m + m) % m;
}
static_assert(spread_stride(512, 8, 2) == 516 && spread_stride(512, 4, 2) == 520, "FP32 staging rows, N = 1024");
static_assert(spread_stride(1089, 8, 2) == 1092 && spread_stride(1089, 4, 4) == 1092, "complex rows, N = 1024");
static_assert(spread_stride(9, 64, 2) == 9, "no spread for more rows than 64-dword slots");

// Block shape of a pass kernel.  Variant V (a launch-time choice of the
// autotuner): bits 0-1 divide the rows per block by 2^(V & 3), bit 2 caps the
// later FFT radices at 4.  Rows per block: about 64 KB of LDS, at most 32,
// a power of two dividing N/2 (so blocks of 2 RPB rows tile an axis).
template <typename T, int N, int V = 0>
struct Rows {
    using PL = Plan<N, (V >> 2) & 1>;
    static constexpr int bytes = 65536 / (N * (int)sizeof(cpx<T>));
    static constexpr int RPB0 = pow2_floor(bytes < 1 ? 1 : (bytes > 32 ? 32 : bytes)) >> (V & 3);
    static constexpr int HALF = (N / 2) & -(N / 2);  // largest power of two dividing N/2
    static constexpr int RPB1 = RPB0 < 1 ? 1 : RPB0;
    static constexpr int RPB = RPB1 > HALF ? HALF : RPB1;
    static constexpr int P = PL::P, E = PL::E;
    static constexpr int THREADS = RPB * P;
    static constexpr int ROWE = lds_row_elems(N);
    // Row stride of the x pass's complex rows, into which it scatters transposed runs:
    // spread over the banks where one wavefront holds one row (P = 64), so no exchange
    // sees another row; else ROWE.
    static constexpr int CPX_ROWE = P == 64 ? spread_stride(ROWE, RPB, 2 * (int)sizeof(T) / 4) : ROWE;
    // Complex staging rows of the z inverse (two fields in the chained pass): at
    // least N / 2 elements, at most ROWE / 2 (the LDS of RPB real rows).
    static constexpr int SROW0 = spread_stride(N / 2, RPB, 2 * (int)sizeof(T) / 4);
    static constexpr int SROW = SROW0 <= ROWE / 2 ? SROW0 : ROWE / 2;
    static_assert(THREADS <= 1024, "block too large");
};

// Width of the kz tiles of S1: the rows of a y pass block in variant 0.
template <typename T, int N>
constexpr int kTileZ = Rows<T, N, 0>::RPB;

// element at a 32-bit element offset from a block-uniform base
template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void sto(T* base, uint32_t idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(T)) = v;
}

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

// Full 128-bit product a m, high and low halves, from the four 32 x 32 -> 64-bit
// partial products (a = a1 2^32 + a0, m likewise); the low half is assembled from
// the same partials rather than multiplied out again.
__device__ __forceinline__ void mul_hilo64(uint64_t a, uint64_t m, uint64_t& lo, uint64_t& hi) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
    const uint64_t p00 = (uint64_t)a0 * m0;
    const uint64_t t = (uint64_t)a0 * m1 + (p00 >> 32);  // < 2^64: (2^32 - 1)^2 + 2^32 - 1
    const uint64_t u = (uint64_t)a1 * m0 + (uint32_t)t;
    const uint64_t v = (uint64_t)a1 * m1 + (t >> 32);
    hi = v + (u >> 32);
    lo = (u << 32) | (uint32_t)p00;
}

// a ^ b ^ c in one three-input bitwise operation per 32-bit half (truth table 0x96)
__device__ __forceinline__ uint64_t xor3_64(uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi =
        __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0x96);
    return ((uint64_t)hi << 32) | lo;
}

// --------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and Box-Muller: unit Gaussians of the
// four cells 4q .. 4q+3.  counter = (q, stream, 0, 0), key = (seed, 0); word
// pairs (w0, w1), (w2, w3) give 53-bit uniforms in (0, 1); cell 4q + r takes
// pair r / 2 and the cosine (r even) or sine (r odd) branch.  The transform
// runs in the precision T of the field (an FP32 field needs no FP64 logarithm).
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void group_gaussians(uint64_t seed, uint64_t stream, uint64_t q, T (&g)[4]) {
    uint64_t c0 = q, c1 = stream, c2 = 0, c3 = 0;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        uint64_t lo0, hi0, lo1, hi1;
        mul_hilo64(c0, 0xD2E7470EE14C6C93ull, lo0, hi0);
        mul_hilo64(c2, 0xCA5A826395121157ull, lo1, hi1);
        const uint64_t n0 = xor3_64(hi1, c1, k0), n2 = xor3_64(hi0, c3, k1);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    const uint64_t w[4] = {c0, c1, c2, c3};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        // the 53-bit uniforms are formed in FP64 (exact), then rounded once to T
        const T u1 = (T)(((double)(w[2 * p] >> 11) + 0.5) * 0x1p-53);
        const T u2 = (T)(((double)(w[2 * p + 1] >> 11) + 0.5) * 0x1p-53);
        const T rad = sqrt((T)-2 * log(u1));
        T sn, cs;  // the angle 2 pi u2, without a general range reduction
        if constexpr (sizeof(T) == 4) sincospif((T)2 * u2, &sn, &cs);
        else sincospi((T)2 * u2, &sn, &cs);
        g[2 * p] = rad * cs;
        g[2 * p + 1] = rad * sn;
    }
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

// Radial table of the linear amplitude times N^-3 at every integer |n|^2:
// tab[n2] = lin_amplitude(kF sqrt(n2)) N^-3 for 0 < n2 <= n2max, tab[0] = 0.
static __global__ void k_amp_table(double* tab, int64_t n2max, double kF, double invN3, LinParams p) {
    const int64_t n2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n2 > n2max) return;
    tab[n2] = n2 == 0 ? 0.0 : lin_amplitude(kF * sqrt((double)n2), p) * invN3;
}

// canonical registers of one row -> this row's LDS buffer in natural order
template <typename PL, typename T>
__device__ __forceinline__ void stage_row(const cpx<T> (&v)[PL::E], cpx<T>* row, int l) {
#pragma unroll
    for (int e = 0; e < PL::E; ++e) row[lds_pad(l + PL::P * e)] = v[e];
}

// Transposed load, gather half: item it of this thread is idx = threadIdx.x +
// THREADS it, i.e. (q, rr) = (idx / RPB, idx % RPB): position q of block row
// rr, read from in[q * stride + rr].  Every lane loads (items past `count`
// read item count - 1, rows past `nrows` read row 0; both are dropped later),
// so all loads are in flight together and can be issued before other work.
// tid: the thread's index within its team of THREADS (default: the block).
template <typename T, int N, int V, int ITEMS>
__device__ __forceinline__ void gather_runs(cpx<T> (&g)[ITEMS], const cpx<T>* in, uint32_t stride, int count,
                                           int nrows, int tid = -1) {
    using RW = Rows<T, N, V>;
    constexpr int RPB = RW::RPB;
    const int t = tid < 0 ? (int)threadIdx.x : tid;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int idx = min(t + RW::THREADS * it, count * RPB - 1);
        const int q = idx / RPB, rr = idx % RPB;
        g[it] = ldo(in, (uint32_t)q * stride + (uint32_t)(rr < nrows ? rr : 0));
    }
}

// Transposed load, scatter half, through real-valued LDS rows (split
// exchange): the gathered items go to position pos(q) of LDS row rr, real
// parts first; afterwards v[e] holds position l + P e of this wave's row, or
// zero where has(l + P e) is false.  Starts with a block barrier (the rows may
// still be in use) and leaves every row free for this wave's own exchanges.
// lds: the team's rows; tid as for gather_runs.
template <typename T, int N, int V, int ITEMS, typename PosF, typename HasF, int E>
__device__ __forceinline__ void scatter_runs_split(const cpx<T> (&g)[ITEMS], T* lds, const T* row, int l, int count,
                                                   PosF pos, HasF has, cpx<T> (&v)[E], int tid = -1) {
    using RW = Rows<T, N, V>;
    constexpr int RPB = RW::RPB, ROWE = RW::ROWE, P = RW::P;
    static_assert(E == RW::E, "register count of the row");
    const int t = tid < 0 ? (int)threadIdx.x : tid;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int idx = t + RW::THREADS * it;
            if (idx < count * RPB) lds[(idx % RPB) * ROWE + lds_pad(pos(idx / RPB))] = part ? g[it].y : g[it].x;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T t = row[lds_pad(l + P * e)];
            const T z = has(l + P * e) ? t : (T)0;
            if (part) v[e].y = z;
            else v[e].x = z;
        }
    }
}

// unpack the transform C of c = a + i b at mode k (m = C(-k)):
// which = 0 gives A(k), which = 1 gives B(k)
template <typename T>
__device__ __forceinline__ cpx<T> unpack_real_pair(cpx<T> c, cpx<T> m, int which) {
    if (which == 0) return {(T)0.5 * (c.x + m.x), (T)0.5 * (c.y - m.y)};
    return {(T)0.5 * (c.y + m.y), (T)0.5 * (m.x - c.x)};
}

// --------------------------------------------------------------------------
// P1: z pass, forward, into S1.
// SRC 0: one real field, SRC 1: Gaussian noise generated in place.  A block
//   covers 2 RPB consecutive y at one x; team r transforms rows y0 + r (real
//   part) and y0 + RPB + r (imaginary part) together.
// SRC 3: four real fields pin.d[0..3] (the reverse mode's g delta, g u),
//   packed as d0 + i d1 and d2 + i d3; a block covers RPB consecutive y.
// SRC 4: two real fields pin.d[0..1] (the printed sources S_delta, S_theta),
//   packed as d0 + i d1; a block covers RPB consecutive y.
// The products of an order, the remaining source of P1, are formed in
// k_zchain below.
// --------------------------------------------------------------------------
// base[idx] where ok, zero elsewhere, with no branch around the load: the caller passes
// an index that names a valid element also where ok is false, so every lane loads and
// all loads of a row are in flight together (a branch per element would wait for each).
template <typename T>
__device__ __forceinline__ cpx<T> load_or_zero(const cpx<T>* base, size_t idx, bool ok) {
    const cpx<T> t = base[idx];
    return ok ? t : cpx<T>{(T)0, (T)0};
}

template <typename T>
struct ProductInputs {
    const T* d[4];     // delta_1 .. delta_{n-1}
    const T* u[4][3];  // u_1 .. u_{n-1}
};

// The 4 (NORD - 1) raw inputs of one cell: delta_m, u_m for m = 1 .. NORD - 1.
template <typename T, int NORD>
__device__ __forceinline__ void load_raw(const ProductInputs<T>& pin, size_t blockbase, uint32_t off,
                                         T (&raw)[4 * (NORD - 1)]) {
#pragma unroll
    for (int m = 1; m < NORD; ++m) {
        raw[4 * (m - 1)] = ldo(pin.d[m - 1] + blockbase, off);
#pragma unroll
        for (int j = 0; j < 3; ++j) raw[4 * (m - 1) + 1 + j] = ldo(pin.u[m - 1][j] + blockbase, off);
    }
}

template <typename T, int NORD>
__device__ __forceinline__ void combine_products(const T (&raw)[4 * (NORD - 1)], cpx<T>& a, cpx<T>& b) {
    T d[NORD], u[NORD][3];
#pragma unroll
    for (int m = 1; m < NORD; ++m) {
        d[m] = raw[4 * (m - 1)];
#pragma unroll
        for (int j = 0; j < 3; ++j) u[m][j] = raw[4 * (m - 1) + 1 + j];
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

// Forward z transforms of a block's packed rows and the read-out of their kept
// kz into S1 tiles.  NPACK transforms per row (a, then b).  PACK4: every row
// packs two fields, the block covers RPB rows of y, and transform pk goes to
// S1 fields 2 pk and 2 pk + 1; otherwise team r packs rows y0 + r and
// y0 + RPB + r of one field (2 RPB rows of y).
template <typename T, int N, int V, int NPACK, bool PACK4, typename TWS>
__device__ __forceinline__ void zfwd_readout(const cpx<T> (&a)[Rows<T, N, V>::E], const cpx<T> (&b)[Rows<T, N, V>::E],
                                             cpx<T>* lds, TWS tws, cpx<T>* s1, size_t s1_field, int x, int y0,
                                             int Kz) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    constexpr int YB = PACK4 ? RPB : 2 * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    cpx<T>* row = lds + r * ROWE;
    static_for<NPACK>([&](auto pkc) {
        constexpr int pk = decltype(pkc)::value;
        cpx<T> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = pk == 0 ? a[e] : b[e];
        if constexpr (pk > 0) __syncthreads();  // previous read-out has finished with LDS
        fft_row<PL, -1, T>(v, row, tws, l);
        stage_row<PL, T>(v, row, l);
        __syncthreads();
        // read-out: the kept kz of rows y0 + rr in S1 tile order, tile by tile (tb = first
        // kz of the tile, w its width); consecutive items are consecutive addresses
        constexpr int TZ = kTileZ<T, N>;
        cpx<T>* out = s1 + (size_t)x * N * Kz;
        for (int idx = threadIdx.x; idx < Kz * YB; idx += RW::THREADS) {
            const int tb = idx / (YB * TZ) * TZ, w = min(TZ, Kz - tb);
            const int j = idx - tb * YB, rr = j / w, kz = tb + j % w;
            const uint32_t o = (uint32_t)(tb * N + (y0 + rr) * w + (kz - tb));
            const int team = PACK4 ? rr : rr % RPB;
            const cpx<T> c = lds[team * ROWE + lds_pad(kz)];
            const cpx<T> m = lds[team * ROWE + lds_pad(kz == 0 ? 0 : N - kz)];
            if constexpr (PACK4) {
                sto(out + (size_t)(2 * pk) * s1_field, o, unpack_real_pair(c, m, 0));
                sto(out + (size_t)(2 * pk + 1) * s1_field, o, unpack_real_pair(c, m, 1));
            } else {
                sto(out, o, unpack_real_pair(c, m, rr / RPB));
            }
        }
    });
}

template <typename T, int N, int V, int SRC>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_zfwd(const T* __restrict__ f, ProductInputs<T> pin,
                                                                    uint64_t seed, uint64_t stream,
                                                                    cpx<T>* __restrict__ s1, size_t s1_field,
                                                                    const cpx<T>* __restrict__ tw, int Kz, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    static_assert(SRC >= 0 && SRC <= 4 && SRC != 2, "sources 0, 1, 3, 4");
    constexpr bool PACK4 = SRC == 3 || SRC == 4;  // field pairs packed per row
    constexpr int YB = PACK4 ? RPB : 2 * RPB;  // rows of y per block
    __shared__ cpx<T> lds[RPB * ROWE];
    // twiddles in LDS for FP32 (this pass's LDS traffic is light), else from the cache
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    f = zptr(f, zs);
    s1 = zptr(s1, zs);
    if constexpr (SRC == 3 || SRC == 4) {
#pragma unroll
        for (int m = 0; m < (SRC == 3 ? 4 : 2); ++m) pin.d[m] = zptr(pin.d[m], zs);
    }
    stream += blockIdx.z;  // realisation r of a batch draws Philox stream `stream + r`
    constexpr uint32_t groups = N / YB;
    const uint32_t blk = xcd_block(blockIdx.x, N * groups);
    const int x = blk / groups, y0 = (blk % groups) * YB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const size_t blockbase = ((size_t)x * N + y0) * N;  // first cell of the block
    cpx<T>* row = lds + r * ROWE;

    cpx<T> a[E], b[E];
    if constexpr (SRC == 1) {
        // 2 RPB N consecutive cells: each thread draws E / 2 groups of 4 cells
        // straight into the LDS rows (row y0 + rr goes to team rr % RPB, real
        // part for rr < RPB, imaginary part otherwise)
        T* words = reinterpret_cast<T*>(lds);
#pragma unroll
        for (int i = 0; i < E / 2; ++i) {
            const int grp = threadIdx.x + RW::THREADS * i;  // < 2 RPB N / 4
            T gs[4];
            group_gaussians<T>(seed, stream, (blockbase >> 2) + grp, gs);
            const int rr = (4 * grp) / N, pos = (4 * grp) % N;
            const int team = rr % RPB, part = rr / RPB;
#pragma unroll
            for (int k = 0; k < 4; ++k) words[2 * (team * ROWE + lds_pad(pos + k)) + part] = (T)gs[k];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) a[e] = row[lds_pad(l + P * e)];
        wave_sync();
    } else if constexpr (SRC == 0) {
        const T* f0 = f + blockbase;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t o = (uint32_t)(r * N + l + P * e);
            a[e] = {ldo(f0, o), ldo(f0, o + (uint32_t)(RPB * N))};
        }
    } else if constexpr (SRC == 3 || SRC == 4) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t o = (uint32_t)(r * N + l + P * e);
            a[e] = {ldo(pin.d[0] + blockbase, o), ldo(pin.d[1] + blockbase, o)};
            if constexpr (SRC == 3) b[e] = {ldo(pin.d[2] + blockbase, o), ldo(pin.d[3] + blockbase, o)};
        }
    }

    constexpr int NPACK = SRC == 3 ? 2 : 1;
    zfwd_readout<T, N, V, NPACK, PACK4>(a, b, lds, tws, s1, s1_field, x, y0, Kz);
}

// --------------------------------------------------------------------------
// P5 of order NORD - 1 chained into P1 of order NORD.  The products of order
// NORD are V = sum_m delta_m u_{n-m} and W = sum_m u_m . u_{n-m} (the
// divergence form of the sources of Eq. 10), packed as V_x + i V_y and
// V_z + i W.  They read delta_m, u_m of the lower orders as real rows.  The
// latest order's four fields (delta, u_x, u_y, u_z) come straight from their
// S4 spectra (u_z as phi, times kz here): the z inverse of delta + i u_x and
// of u_y + i u_z (the two-fields-per-transform packing of the header) runs here, its real rows
// are stored where an output is set (a field no later pass reads is not) and
// go into the products without a round trip through HBM.  A block covers RPB
// consecutive y at one x, the layout of SRC 3 of k_zfwd.
// --------------------------------------------------------------------------
template <typename T>
struct ChainArgs {
    const cpx<T>* s4;
    size_t s4_field;
    int f[4];   // S4 fields of delta, u_x, u_y and phi (u_z = kz phi) of order NORD - 1
    T* out[4];  // their real rows, or null
    T* dup;     // a second copy of delta, or null
};

template <typename T, int N, int V, int NORD>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS))
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_zchain(ProductInputs<T> pin, ChainArgs<T> ch,
                                                                      cpx<T>* __restrict__ s1, size_t s1_field,
                                                                      const cpx<T>* __restrict__ tw, int Kz,
                                                                      size_t zs) {
    static_assert(NORD >= 2 && NORD <= 5, "orders 2 .. 5");
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    __shared__ cpx<T> lds[RPB * ROWE];
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    s1 = zptr(s1, zs);
    ch.s4 = zptr(ch.s4, zs);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (ch.out[i]) ch.out[i] = zptr(ch.out[i], zs);
    if (ch.dup) ch.dup = zptr(ch.dup, zs);
#pragma unroll
    for (int m = 0; m < NORD - 2; ++m) {
        pin.d[m] = zptr(pin.d[m], zs);
#pragma unroll
        for (int j = 0; j < 3; ++j) pin.u[m][j] = zptr(pin.u[m][j], zs);
    }
    constexpr uint32_t groups = N / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, N * groups);
    const int x = blk / groups, y0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const size_t blockbase = ((size_t)x * N + y0) * N;  // first cell of the block

    // z inverse of the latest order: pair q packs fields f[2q] + i f[2q+1].  The
    // staged runs of the two fields sit side by side in LDS (rows of SROW >= Kz
    // complex elements); position p of the Hermitian row takes kz = p or N - p.
    constexpr int IT = E / 2, SROW = RW::SROW;
    static_assert(SROW >= N / 2 && 2 * SROW <= ROWE, "a staged row holds every kept kz");
    cpx<T>* stage = lds;
    cpx<T>* crow = lds + r * ROWE;  // this row's complex exchange row
    auto src = [&](int p) { return p < Kz ? p : (p > N - Kz ? N - p : 0); };
    const cpx<T>* s4x = ch.s4 + (size_t)x * Kz * N + y0;
    cpx<T> cur[2][E];
    static_for<2>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        cpx<T> ga[IT], gb[IT];
        gather_runs<T, N, V>(ga, s4x + (size_t)ch.f[2 * q] * ch.s4_field, (uint32_t)N, Kz, RPB);
        gather_runs<T, N, V>(gb, s4x + (size_t)ch.f[2 * q + 1] * ch.s4_field, (uint32_t)N, Kz, RPB);
        __syncthreads();  // the previous transform's exchanges are done with the LDS
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = (int)threadIdx.x + RW::THREADS * it;
            if (idx < Kz * RPB) {
                // the second pair's B field is phi: u_z = kz phi at the stored kz = idx / RPB
                const cpx<T> b = q == 1 ? cscale(gb[it], (T)(idx / RPB)) : gb[it];
                stage[(idx % RPB) * SROW + idx / RPB] = ga[it];
                stage[(RPB + idx % RPB) * SROW + idx / RPB] = b;
            }
        }
        __syncthreads();
        cpx<T> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = l + P * e;
            const cpx<T> av = stage[r * SROW + src(p)], bv = stage[(RPB + r) * SROW + src(p)];
            const cpx<T> lo = {av.x - bv.y, av.y + bv.x};
            const cpx<T> hi = {av.x + bv.y, bv.x - av.y};
            const cpx<T> zero = {(T)0, (T)0};
            v[e] = p < Kz ? lo : (p > N - Kz ? hi : zero);
        }
        __syncthreads();  // every wave has read the staged runs before the exchanges reuse the LDS
        fft_row<PL, +1, T>(v, crow, tws, l);
        T* o0 = ch.out[2 * q];
        T* o1 = ch.out[2 * q + 1];
        if (o0) {
#pragma unroll
            for (int e = 0; e < E; ++e) sto(o0 + blockbase, (uint32_t)(r * N + l + P * e), v[e].x);
        }
        if (q == 0 && ch.dup) {
#pragma unroll
            for (int e = 0; e < E; ++e) sto(ch.dup + blockbase, (uint32_t)(r * N + l + P * e), v[e].x);
        }
        if (o1) {
#pragma unroll
            for (int e = 0; e < E; ++e) sto(o1 + blockbase, (uint32_t)(r * N + l + P * e), v[e].y);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) cur[q][e] = v[e];
    });

    // products, with the latest order's values from registers.  The packed products
    // are formed before the forward transforms, so the raw inputs are dead when they
    // start.  The lower orders' raw loads run DEPTH elements ahead of the products
    // (about 48 values in flight per lane), so a wave waits for memory once per DEPTH
    // elements rather than once per element.
    constexpr int NL = 4 * (NORD - 2), NR = 4 * (NORD - 1);
    cpx<T> a[E], b[E];
    auto combine = [&](const T* lower, int e) {
        T raw[NR];
#pragma unroll
        for (int i = 0; i < NL; ++i) raw[i] = lower[i];
        raw[NL] = cur[0][e].x;
        raw[NL + 1] = cur[0][e].y;
        raw[NL + 2] = cur[1][e].x;
        raw[NL + 3] = cur[1][e].y;
        combine_products<T, NORD>(raw, a[e], b[e]);
    };
    if constexpr (NORD == 2) {
#pragma unroll
        for (int e = 0; e < E; ++e) combine(nullptr, e);
    } else {
        constexpr int DEPTH = (48 / NL) < 2 ? 2 : ((48 / NL) > 4 ? 4 : (48 / NL));
        T raw[DEPTH][NL];
#pragma unroll
        for (int e = 0; e < DEPTH - 1; ++e)
            load_raw<T, NORD - 1>(pin, blockbase, (uint32_t)(r * N + l + P * e), raw[e]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e + DEPTH - 1 < E)
                load_raw<T, NORD - 1>(pin, blockbase, (uint32_t)(r * N + l + P * (e + DEPTH - 1)),
                                      raw[(e + DEPTH - 1) % DEPTH]);
            combine(raw[e % DEPTH], e);
            keep_here(a[e]);
            keep_here(b[e]);
        }
    }
    __syncthreads();  // the inverse transforms' exchanges are done with the LDS
    zfwd_readout<T, N, V, 2, true>(a, b, lds, tws, s1, s1_field, x, y0, Kz);
}

// --------------------------------------------------------------------------
// P2: y pass, forward.  Rows (x, kz) along y of S1; block = RPB consecutive
// kz at one x (one S1 tile); grid.y = j takes input field j in_step to output
// field j out_step.  Keeps |ky| <= Kc and writes S2 rows (kz, x) of Ky values
// (s2_row apart).
// COMB (the products of an order, one launch with grid.y = 1; the steps are
// unused): output field 1 is D = i (ky V_y + kz V_z) from inputs V_y, V_z (fields 1, 2).
// i k.V is linear, so its y and z terms are summed here and the x pass needs one
// field fewer; V_x and W go through a plain launch.
// --------------------------------------------------------------------------
template <typename T, int N, int V, bool COMB = false>
__global__ __launch_bounds__(((COMB ? 2 : 1) * Rows<T, N, V>::THREADS)) void k_yfwd(
    const cpx<T>* __restrict__ s1, size_t s1_field, cpx<T>* __restrict__ s2, size_t s2_field,
    const cpx<T>* __restrict__ tw, CubeDims cd, size_t zs, int in_step, int out_step, int s2_row) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    // COMB: two teams of THREADS, team 0 transforms V_y and team 1 V_z of the same rows
    constexpr int TEAMS = COMB ? 2 : 1;
    static_assert(TEAMS * RW::THREADS <= 1024, "block too large");
    __shared__ T lds[TEAMS * RPB * ROWE];  // real-valued rows (split exchange), per team
    // twiddles in LDS for FP32 (this pass's LDS traffic is light), else from the cache
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    s1 = zptr(s1, zs);
    s2 = zptr(s2, zs);
    // block = RPB consecutive kz at one x: the rows (x, kz) along y
    const uint32_t groups = (cd.Kz + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, N * groups);
    const int x = blk / groups, kz0 = (blk % groups) * RPB;
    const int nrows = min(RPB, cd.Kz - kz0);
    const int team = COMB ? (int)threadIdx.x / RW::THREADS : 0;
    const int tid = (int)threadIdx.x - team * RW::THREADS;
    const int r = tid / P, l = tid % P;
    T* tl = lds + team * RPB * ROWE;
    T* row = tl + r * ROWE;
    // the S1 tile holding kz0 .. kz0 + nrows - 1 (RPB divides the tile width TZ)
    constexpr int TZ = kTileZ<T, N>;
    const int tb = kz0 / TZ * TZ, w = min(TZ, cd.Kz - tb);
    auto transform = [&](int f, cpx<T>(&v)[E]) {
        cpx<T> g[E];
        gather_runs<T, N, V>(g, s1 + (size_t)f * s1_field + (size_t)x * N * cd.Kz + (size_t)tb * N + (kz0 - tb),
                             (uint32_t)w, N, nrows, tid);
        scatter_runs_split<T, N, V>(g, tl, row, l, N, [](int q) { return q; }, [](int) { return true; }, v, tid);
        fft_row_split<PL, -1, T>(v, row, tws, l);
    };
    cpx<T> v[E];
    const int fout = COMB ? 1 : (int)blockIdx.y * out_step;
    if constexpr (!COMB) {
        transform((int)blockIdx.y * in_step, v);
    } else {
        // D = i ky V_y + i kz V_z (inputs 1 and 2), the y and z terms of i k.V (integer
        // ky, kz; the x pass adds i kx V_x and applies kF).  Team 1 hands its V_z rows to
        // team 0 through LDS, as complex rows.
        transform(1 + team, v);
        __syncthreads();  // both teams are done with their exchange rows
        cpx<T>* xrow = reinterpret_cast<cpx<T>*>(lds) + r * ROWE;
        if (team == 1) {
#pragma unroll
            for (int e = 0; e < E; ++e) xrow[lds_pad(l + P * e)] = v[e];
        }
        __syncthreads();
        if (team == 1) return;
        const T kz = (T)(kz0 + r);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cpx<T> vz = xrow[lds_pad(l + P * e)];
            const T ky = (T)signed_pos(l + P * e, N);
            v[e] = cmul_i(cpx<T>{ky * v[e].x + kz * vz.x, ky * v[e].y + kz * vz.y});
        }
    }
    // S2 row (kz0 + r, x): the kept ky in compact order, rows s2_row >= Ky apart
    if (r < nrows) {
        cpx<T>* out = s2 + (size_t)fout * s2_field + ((size_t)kz0 * N + x) * s2_row;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ic = pos_to_compact(l + P * e, cd.Kc, N);
            if (ic >= 0) sto(out, (uint32_t)(r * N * s2_row + ic), v[e]);
        }
    }
}

// --------------------------------------------------------------------------
// P3: x pass, fused.  Rows (kz, ky') along x of S2; block = RPB consecutive
// ky' at one kz (runs of RPB elements of S2).  Forward x transform, the
// k-space step, optional cube stores, then the inverse x transform of every
// output field, stored as S3 rows (kz, ky').
// --------------------------------------------------------------------------
// LIN_ORDER1: the linear field from noise (as LINEAR) with the outputs of
// order 1 (as ORDER1): delta_1 and u_1 without a round trip through real space
enum XMode {
    XM_ORDER = 0,
    XM_ORDER1 = 1,
    XM_LINEAR = 2,
    XM_FORWARD = 3,
    XM_ADJ = 4,
    XM_ADJ1 = 5,
    XM_PFORM = 6,
    XM_LIN_ORDER1 = 7
};

template <typename T>
struct XArgs {
    const cpx<T>* s2;
    size_t s2_field;
    int s2_row;  // S2 row stride (complex elements, >= Ky)
    cpx<T>* s3;
    size_t s3_field;
    cpx<T>* cube_d;  // may be null
    cpx<T>* cube_t;  // may be null
    int n, nout;     // order; number of output fields (written as S3 fields 0..nout-1)
    int nin;         // reverse modes: input fields (1: g delta only, 4: g delta, g u)
    int64_t n2max;   // mask of this order
    double kF, invN3;
    LinParams lin;
    const double* amp;  // LINEAR, LIN_ORDER1, ADJ1: the radial amplitude table (k_amp_table)
};

// inverse x transform of this wave's output row and its store as S3 row r of
// the block (out = the block's first row; rows are N apart).  The row is
// contiguous in S3, so every lane stores its points from registers, and the
// transform only uses this wave's LDS row: no block barrier.
template <typename T, int N, int V, typename TW, int E>
__device__ __forceinline__ void x_inverse_store(cpx<T> (&v)[E], cpx<T>* row, TW tw, int l, cpx<T>* out, int r,
                                                bool active) {
    using PL = typename Rows<T, N, V>::PL;
    static_assert(E == PL::E, "register count of the row");
    fft_row<PL, +1, T>(v, row, tw, l);
    if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) sto(out, (uint32_t)(r * N + l + PL::P * e), v[e]);
    }
}

// The orders' step in FP32 at N = 1024 with blocks of at most four waves asks
// for three waves per SIMD: it then fits 168 VGPRs with a few spills and runs
// faster than at two waves.  Blocks of eight waves would still fit only one per
// CU, and at smaller N the same request spills more.
template <typename T, int N, int V, int MODE>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS))
__attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 && N == 1024 && Rows<T, N, V>::THREADS <= 256 && MODE == XM_ORDER ? 3 : 1))) void k_xfused(
    XArgs<T> a, const cpx<T>* __restrict__ tw, CubeDims cd, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, E = RW::E;
    constexpr int CS = RW::CPX_ROWE;
    __shared__ cpx<T> lds[RPB * CS];
    // FP32 twiddles in LDS: a global-table read at every pass would leave its latency
    // exposed at this pass's low occupancy
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    a.s2 = zptr(a.s2, zs);
    a.s3 = zptr(a.s3, zs);
    a.cube_d = zptr(a.cube_d, zs);
    a.cube_t = zptr(a.cube_t, zs);
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    const int nrows = min(RPB, cd.Ky - ky0);
    cpx<T>* row = lds + r * CS;

    // k-space step: sd holds delta_n(k), st holds theta_n(k) afterwards
    cpx<T> sd[E], st[E];
    constexpr bool ADJ = MODE == XM_ADJ || MODE == XM_ADJ1;
    constexpr int NIN = MODE == XM_ORDER ? 3 : (ADJ ? 4 : (MODE == XM_PFORM ? 2 : 1));
#pragma unroll
    for (int e = 0; e < E; ++e) sd[e] = st[e] = {(T)0, (T)0};
    // |n|^2 <= 3 (N/2)^2 and every mask lies below (N/2)^2: 32-bit integers are exact here
    const T kF = (T)a.kF, invN3 = (T)a.invN3;
    const int n2lim = (int)(a.n2max < INT32_MAX ? a.n2max : INT32_MAX);
    // the radial amplitudes are gathered before the transform, so their latency hides behind it
    constexpr bool AMP = MODE == XM_LINEAR || MODE == XM_LIN_ORDER1 || MODE == XM_ADJ1;
    T ampv[AMP ? E : 1];
    if constexpr (AMP) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int kx = signed_pos(l + P * e, N);
            const int n2 = kx * kx + ky * ky + kz * kz;
            const T t = (T)a.amp[n2 <= n2lim ? n2 : 0];  // unconditional: no branch around the load
            ampv[e] = n2 <= n2lim ? t : (T)0;
        }
    }
    // Input rows: runs of RPB ky' for every x, regrouped through LDS (rows past the cube
    // read row 0 of the block and are never stored).  The runs of field f + 1 are
    // loaded before field f is transformed, so their latency hides behind it (not in
    // the reverse mode, whose k-space accumulation leaves no registers for them).
    auto gather_field = [&](int f, cpx<T>(&gf)[E]) {
        gather_runs<T, N, V>(gf, a.s2 + (size_t)f * a.s2_field + (size_t)kz * N * a.s2_row + ky0, (uint32_t)a.s2_row, N,
                             nrows);
    };
    cpx<T> g[E];
    gather_field(0, g);
    static_for<NIN>([&](auto fc) {
        constexpr int f = decltype(fc)::value;
        if (ADJ && f >= a.nin) return;
        if constexpr (ADJ && f > 0) gather_field(f, g);
        __syncthreads();  // every wave is done with its row
#pragma unroll
        for (int it = 0; it < E; ++it) {
            const int idx = (int)threadIdx.x + RW::THREADS * it;
            lds[(idx % RPB) * CS + lds_pad(idx / RPB)] = g[it];
        }
        __syncthreads();
        cpx<T> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = row[lds_pad(l + P * e)];
        if constexpr (!ADJ && f + 1 < NIN) gather_field(f + 1, g);
        fft_row<PL, -1, T>(v, row, tws, l);
        if constexpr (MODE == XM_ORDER) {
            // inputs V_x, D = i (ky V_y + kz V_z) (formed by the y pass), W
            if constexpr (f == 0) {
                // S_delta = i kx V_x + D  (kF and N^-3 applied below)
#pragma unroll
                for (int e = 0; e < E; ++e) sd[e] = cscale(cmul_i(v[e]), (T)signed_pos(l + P * e, N));
            } else if constexpr (f == 1) {
#pragma unroll
                for (int e = 0; e < E; ++e) sd[e] = cadd(sd[e], v[e]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) st[e] = v[e];
            }
            // pin only what has been assigned: a pinned all-zero row would hold 32 VGPRs
#pragma unroll
            for (int e = 0; e < E; ++e) {
                keep_here(sd[e]);
                if constexpr (f == 2) keep_here(st[e]);
            }
        } else if constexpr (MODE == XM_PFORM) {
            // the printed sources of Eq. 10, transformed as they are
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if constexpr (f == 0) sd[e] = v[e];
                else st[e] = v[e];
                keep_here(sd[e]);
                if constexpr (f > 0) keep_here(st[e]);
            }
        } else if constexpr (ADJ) {
            if constexpr (f == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) sd[e] = v[e];  // G_delta (unnormalised)
            } else {
                // G_theta += (+i k_f / k^2) F[g u_f]: the adjoint of u = (-i k / k^2) theta
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int kx = signed_pos(l + P * e, N);
                    const int n2 = kx * kx + ky * ky + kz * kz;
                    const int kf = f == 1 ? kx : (f == 2 ? ky : kz);
                    const T s = n2 > 0 ? (T)((double)kf / (a.kF * (double)n2)) : (T)0;
                    st[e] = cadd(st[e], cpx<T>{-v[e].y * s, v[e].x * s});
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                keep_here(sd[e]);
                if constexpr (f > 0) keep_here(st[e]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) sd[e] = v[e];
        }
    });

#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int kx = signed_pos(l + P * e, N);
        const int n2 = kx * kx + ky * ky + kz * kz;
        const bool keep = active && n2 > 0 && n2 <= n2lim;
        if constexpr (MODE == XM_ORDER || MODE == XM_PFORM) {
            // D-form: S_delta = i k.V(k) N^-3, S_theta = -(k^2/2) W(k) N^-3 (divergence form of
            // Eq. 10); P-form: the transforms of the printed sources, times N^-3
            const cpx<T> sdel = MODE == XM_ORDER ? cscale(sd[e], kF * invN3) : cscale(sd[e], invN3);
            const cpx<T> sthe =
                MODE == XM_ORDER ? cscale(st[e], (T)(-0.5) * kF * kF * (T)n2 * invN3) : cscale(st[e], invN3);
            const T cn = (T)(2.0 / ((2.0 * a.n + 3.0) * (a.n - 1.0)));
            const T m00 = cn * (T)(a.n + 0.5), m01 = cn, m10 = cn * (T)1.5, m11 = cn * (T)a.n;
            const cpx<T> dn = {m00 * sdel.x + m01 * sthe.x, m00 * sdel.y + m01 * sthe.y};
            const cpx<T> tn = {m10 * sdel.x + m11 * sthe.x, m10 * sdel.y + m11 * sthe.y};
            sd[e] = keep ? dn : cpx<T>{(T)0, (T)0};
            st[e] = keep ? tn : cpx<T>{(T)0, (T)0};
        } else if constexpr (MODE == XM_LINEAR || MODE == XM_LIN_ORDER1) {
            sd[e] = cscale(sd[e], keep ? ampv[e] : (T)0);
        } else if constexpr (MODE == XM_ADJ) {
            // (a, b) = W2 c_n M^T (G_delta, G_theta), M = [[n + 1/2, 1], [3/2, n]]
            const T cn = (T)(2.0 / ((2.0 * a.n + 3.0) * (a.n - 1.0)));
            const cpx<T> gd = cscale(sd[e], invN3), gt = cscale(st[e], invN3);
            const T m00 = cn * (T)(a.n + 0.5), m10 = cn * (T)1.5, m01 = cn, m11 = cn * (T)a.n;
            const cpx<T> av = {m00 * gd.x + m10 * gt.x, m00 * gd.y + m10 * gt.y};
            const cpx<T> bv = {m01 * gd.x + m11 * gt.x, m01 * gd.y + m11 * gt.y};
            sd[e] = keep ? av : cpx<T>{(T)0, (T)0};
            st[e] = keep ? bv : cpx<T>{(T)0, (T)0};
        } else if constexpr (MODE == XM_ADJ1) {
            // g w(k) = W1 A(k) (G_delta + G_theta): the transpose of the linear field
            sd[e] = cscale(cadd(sd[e], st[e]), keep ? ampv[e] : (T)0);
        } else {
            sd[e] = keep ? cscale(sd[e], invN3) : cpx<T>{(T)0, (T)0};
        }
    }
    // theta_1 = delta_1 below order 2
    if constexpr (MODE != XM_ORDER && MODE != XM_PFORM && !ADJ) {
#pragma unroll
        for (int e = 0; e < E; ++e) st[e] = sd[e];
    }

    // cube stores (masked spectra), kept kx only
    if (active && (a.cube_d || a.cube_t)) {
        const size_t cbase = ((size_t)kz * cd.Ky + kyc) * cd.Ky;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ic = pos_to_compact(l + P * e, cd.Kc, N);
            if (ic >= 0) {
                if (a.cube_d) a.cube_d[cbase + ic] = sd[e];
                if (a.cube_t) a.cube_t[cbase + ic] = st[e];
            }
        }
    }
    if constexpr (MODE != XM_FORWARD) {
        // outputs.  ORDER: delta, theta, u_x, phi;  ORDER1: delta, u_x, phi;  LINEAR: delta;
        // ADJ: g V_x, g V_y, g V_z, g W;  ADJ1: g w
        // PFORM: delta, theta
        // phi = (-i / k^2) theta: along this row ky and kz are constant, so u_y = ky phi and
        // u_z = kz phi share one transform here; the inverse y pass (k_yinv<..., true>)
        // applies ky, the inverse z pass (k_zchain) kz.
        constexpr int NOUT_MAX =
            (MODE == XM_ORDER || MODE == XM_ADJ)
                ? 4
                : ((MODE == XM_ORDER1 || MODE == XM_LIN_ORDER1) ? 3 : (MODE == XM_PFORM ? 2 : 1));
        constexpr int FIRST_U = (MODE == XM_ORDER || MODE == XM_PFORM) ? 2 : 1;
        const size_t outbase = ((size_t)kz * cd.Ky + ky0) * N;
        static_for<NOUT_MAX>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            if (o < a.nout) {
                cpx<T> v[E];
                if constexpr (MODE == XM_ADJ) {
                    // g V_j = F^-1[-i k_j a],  g W = F^-1[-(k^2/2) b]
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int kx = signed_pos(l + P * e, N);
                        if constexpr (o < 3) {
                            const T kj = (T)(a.kF * (double)(o == 0 ? kx : (o == 1 ? ky : kz)));
                            v[e] = {sd[e].y * kj, -sd[e].x * kj};
                        } else {
                            const int n2 = kx * kx + ky * ky + kz * kz;
                            v[e] = cscale(st[e], (T)(-0.5 * a.kF * a.kF * (double)n2));
                        }
                    }
                } else if constexpr (MODE == XM_ADJ1) {
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = sd[e];
                } else if constexpr (o < FIRST_U) {
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = (o == 0) ? sd[e] : st[e];
                } else {
                    // u_x(k) = (-i kx / k^2) theta(k), then phi; the factors kx / (kF n^2) and
                    // 1 / (kF n^2) are formed in FP64 and rounded once (u feeds every later
                    // order's products)
                    constexpr int comp = o - FIRST_U;
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int kx = signed_pos(l + P * e, N);
                        const int n2 = kx * kx + ky * ky + kz * kz;
                        const double num = comp == 0 ? (double)kx : 1.0;
                        const T s = n2 > 0 ? (T)(num / (a.kF * (double)n2)) : (T)0;
                        v[e] = {st[e].y * s, -st[e].x * s};
                    }
                }
                x_inverse_store<T, N, V>(v, row, tws, l, a.s3 + (size_t)o * a.s3_field + outbase, r, active);
            }
        });
    }
}

// --------------------------------------------------------------------------
// P3 for shell-filtered fields (bispectrum): rows (kz, ky') of a cube, kept
// when lo <= n^2 < hi; the field pointer may be null for the indicator 1_b.
// Inverse x transform, stored as S3 rows.  grid.y = slot.
// --------------------------------------------------------------------------
template <typename T>
struct ShellSlots {
    const cpx<T>* cube[8];
    int64_t lo[8], hi[8];
    cpx<T>* s3;
    size_t s3_field;
    CubeDims src;  // layout of the cubes (the launch's CubeDims may be a smaller cube
                   // holding every shell of the launch)
};

template <typename T, int N, int V>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_xshell(ShellSlots<T> a, const cpx<T>* __restrict__ tw,
                                                                      CubeDims cd, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    __shared__ cpx<T> lds[RPB * ROWE];
    // FP32 twiddles in LDS: a global-table read at every pass would leave its latency
    // exposed at this pass's low occupancy
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    const int slot = blockIdx.y;
    const cpx<T>* cube = zptr(a.cube[slot], zs);
    // this row in the source cube: the same signed (ky, kz), source compact indices
    const int kys = ky >= 0 ? ky : ky + a.src.Ky;
    const size_t cbase = ((size_t)kz * a.src.Ky + kys) * a.src.Ky;
    cpx<T>* row = lds + r * ROWE;
    cpx<T> v[E];
    bool in[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = l + P * e;
        const int kx = signed_pos(p, N);
        const int64_t n2 = (int64_t)(kx * kx + ky * ky + kz * kz);
        in[e] = active && pos_to_compact(p, cd.Kc, N) >= 0 && n2 >= a.lo[slot] && n2 < a.hi[slot];
    }
    if (cube) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int kx = signed_pos(l + P * e, N);
            v[e] = load_or_zero(cube, in[e] ? cbase + (kx >= 0 ? kx : kx + a.src.Ky) : 0, in[e]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = in[e] ? cpx<T>{(T)1, (T)0} : cpx<T>{(T)0, (T)0};
    }
    x_inverse_store<T, N, V>(v, row, tws, l,
                             zptr(a.s3, zs) + (size_t)slot * a.s3_field + ((size_t)kz * cd.Ky + ky0) * N, r, active);
}

// --------------------------------------------------------------------------
// P3 from stored spectra (reverse mode): rows (kz, ky') of the cubes of
// delta_m and theta_m; inverse x transforms of delta_m and
// u_m = (-i k / k^2) theta_m, stored as rows of S3 fields 0..3.
// --------------------------------------------------------------------------
template <typename T>
struct RegenArgs {
    const cpx<T>* cube_d;
    const cpx<T>* cube_t;
    cpx<T>* s3;
    size_t s3_field;
    double kF;
};

template <typename T, int N, int V>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_xregen(RegenArgs<T> a, const cpx<T>* __restrict__ tw,
                                                                      CubeDims cd, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    __shared__ cpx<T> lds[RPB * ROWE];
    constexpr bool LT = kLdsTwiddles<T>;  // FP32 twiddles in LDS (see k_xfused)
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    const size_t cbase = ((size_t)kz * cd.Ky + kyc) * cd.Ky;
    const cpx<T>* cdl = zptr(a.cube_d, zs);
    const cpx<T>* ctl = zptr(a.cube_t, zs);
    cpx<T>* s3 = zptr(a.s3, zs);
    cpx<T>* row = lds + r * ROWE;
    const size_t outbase = ((size_t)kz * cd.Ky + ky0) * N;
    static_for<4>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        cpx<T> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = l + P * e;
            const int ic = pos_to_compact(p, cd.Kc, N);
            const bool ok = active && ic >= 0;
            const cpx<T> t = load_or_zero(o == 0 ? cdl : ctl, ok ? cbase + ic : 0, ok);
            if constexpr (o == 0) {
                v[e] = t;
            } else {
                const int kx = signed_pos(p, N);
                const int n2 = kx * kx + ky * ky + kz * kz;
                const int kj = o == 1 ? kx : (o == 2 ? ky : kz);
                const T sc = n2 > 0 ? (T)((double)kj / (a.kF * (double)n2)) : (T)0;
                v[e] = {t.y * sc, -t.x * sc};
            }
        }
        x_inverse_store<T, N, V>(v, row, tws, l, s3 + (size_t)o * a.s3_field + outbase, r, active);
    });
}

// --------------------------------------------------------------------------
// P3 for the printed (P-form) sources: the derived real fields of one order
// (Eq. 15, 16) from its stored spectra, five per launch (chunk 0, 1, 2):
//   0-2  grad delta = F^-1[i k delta],      3-5  grad theta = F^-1[i k theta],
//   6-8  u = F^-1[(-i k / k^2) theta],       9-14 d_i u_j = F^-1[(k_i k_j / k^2) theta]
//        for (i, j) = (x,x), (y,y), (z,z), (x,y), (x,z), (y,z) (symmetric: u is a gradient)
// stored as rows of S3 fields 0..4.
// --------------------------------------------------------------------------
template <typename T, int N, int V, int CHUNK>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_xderived(RegenArgs<T> a, const cpx<T>* __restrict__ tw,
                                                                        CubeDims cd, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    __shared__ cpx<T> lds[RPB * ROWE];
    constexpr bool LT = kLdsTwiddles<T>;  // FP32 twiddles in LDS (see k_xfused)
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    const size_t cbase = ((size_t)kz * cd.Ky + kyc) * cd.Ky;
    const cpx<T>* cdl = zptr(a.cube_d, zs);
    const cpx<T>* ctl = zptr(a.cube_t, zs);
    cpx<T>* s3 = zptr(a.s3, zs);
    cpx<T>* row = lds + r * ROWE;
    const size_t outbase = ((size_t)kz * cd.Ky + ky0) * N;
    // the row of each source spectrum, loaded once for the chunk's five outputs
    // (delta for fields 0-2, theta for the rest)
    constexpr int NSRC = CHUNK == 0 ? 2 : 1;
    cpx<T> srcv[NSRC][E];
#pragma unroll
    for (int k = 0; k < NSRC; ++k)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ic = pos_to_compact(l + P * e, cd.Kc, N);
            const bool ok = active && ic >= 0;
            srcv[k][e] = load_or_zero((CHUNK == 0 && k == 0) ? cdl : ctl, ok ? cbase + ic : 0, ok);
        }
    static_for<5>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        constexpr int fld = 5 * CHUNK + o;
        cpx<T> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = l + P * e;
            const cpx<T> src = srcv[(CHUNK == 0 && fld >= 3) ? 1 : 0][e];
            const int kx = signed_pos(p, N);
            auto kc = [&](int axis) { return axis == 0 ? kx : (axis == 1 ? ky : kz); };
            const int n2 = kx * kx + ky * ky + kz * kz;
            if constexpr (fld < 6) {  // i k_j F
                const T kj = (T)(a.kF * (double)kc(fld % 3));
                v[e] = {-src.y * kj, src.x * kj};
            } else if constexpr (fld < 9) {  // (-i k_j / k^2) F
                const T sc = n2 > 0 ? (T)((double)kc(fld - 6) / (a.kF * (double)n2)) : (T)0;
                v[e] = {src.y * sc, -src.x * sc};
            } else {  // (k_i k_j / k^2) F
                constexpr int q = fld - 9;
                constexpr int i = q < 3 ? q : (q < 5 ? 0 : 1);
                constexpr int j = q < 3 ? q : (q == 3 ? 1 : 2);
                const T sc = n2 > 0 ? (T)((double)kc(i) * (double)kc(j) / (double)n2) : (T)0;
                v[e] = cscale(src, sc);
            }
        }
        x_inverse_store<T, N, V>(v, row, tws, l, s3 + (size_t)o * a.s3_field + outbase, r, active);
    });
}

// --------------------------------------------------------------------------
// P3 for smoothed fields (Sec. III A-B): rows (kz, ky') of up to five cubes;
// output o is the inverse x transform of exp(-k^2 R^2 / 2) S_o(k) with
// S_o = sum_{i <= o} coef_i F_i (cumulative, the truncated series of Eq. 8)
// or coef_o F_o, stored as rows of S3 field o.
// --------------------------------------------------------------------------
template <typename T>
struct SmoothArgs {
    const cpx<T>* cube[5];
    double coef[5];
    int nin, cumulative;
    double kF, radius;
    cpx<T>* s3;
    size_t s3_field;
};

template <typename T, int N, int V>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_xsmooth(SmoothArgs<T> a, const cpx<T>* __restrict__ tw,
                                                                       CubeDims cd, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    __shared__ cpx<T> lds[RPB * ROWE];
    constexpr bool LT = kLdsTwiddles<T>;  // FP32 twiddles in LDS (see k_xfused)
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    const uint32_t groups = (cd.Ky + RPB - 1) / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, ky0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int kyc = ky0 + r;
    const bool active = kyc < cd.Ky;
    const int ky = active ? (kyc <= cd.Kc ? kyc : kyc - cd.Ky) : 0;
    const size_t cbase = ((size_t)kz * cd.Ky + kyc) * cd.Ky;
    cpx<T>* s3 = zptr(a.s3, zs);
    cpx<T>* row = lds + r * ROWE;
    const size_t outbase = ((size_t)kz * cd.Ky + ky0) * N;
    const double g = -0.5 * a.kF * a.kF * a.radius * a.radius;
    // the window of each kept element, once for all outputs
    T w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = l + P * e;
        const int kx = signed_pos(p, N);
        const double n2 = (double)((int64_t)kx * kx + (int64_t)ky * ky + (int64_t)kz * kz);
        w[e] = (active && pos_to_compact(p, cd.Kc, N) >= 0) ? (T)exp(g * n2) : (T)0;
    }
    // cumulative: the running sum sum_{i <= o} coef_i F_i, each spectrum read once
    // (the same additions in the same order as summing each output afresh)
    cpx<T> acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = {(T)0, (T)0};
    static_for<5>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        if (o >= a.nin) return;
        if (!a.cumulative) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = {(T)0, (T)0};
        }
        // uniform branch on the mode; the loads inside are unconditional (w = 0 off the cube)
        const cpx<T>* cb = zptr(a.cube[o], zs);
        const T co = (T)a.coef[o];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int ic = pos_to_compact(l + P * e, cd.Kc, N);
            const bool ok = active && ic >= 0;
            acc[e] = cadd(acc[e], cscale(load_or_zero(cb, ok ? cbase + ic : 0, ok), co));
        }
        cpx<T> v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cscale(acc[e], w[e]);
        x_inverse_store<T, N, V>(v, row, tws, l, s3 + (size_t)o * a.s3_field + outbase, r, active);
    });
}

// --------------------------------------------------------------------------
// P4: y pass, inverse.  Rows (kz, x) along ky' of S3 (Ky values, zero-extended
// to N); block = RPB consecutive x at one kz (runs of RPB elements of S3);
// grid.y = field.  Writes S4 rows (x, kz) of N values.
// YZ (grid.y = 1): the input is phi of the x pass; output field 0 is the
// transform of ky phi (u_y), output field 1 that of phi itself, which the
// inverse z pass turns into u_z = kz phi.
// --------------------------------------------------------------------------
template <typename T, int N, int V, bool YZ = false>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_yinv(const cpx<T>* __restrict__ s3, size_t s3_field,
                                                                    cpx<T>* __restrict__ s4, size_t s4_field,
                                                                    const cpx<T>* __restrict__ tw, CubeDims cd,
                                                                    size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    __shared__ T lds[RPB * ROWE];  // real-valued rows (split exchange)
    // FP32 twiddles in LDS: a global-table read at every pass would leave its latency
    // exposed at this pass's low occupancy
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    s3 = zptr(s3, zs);
    s4 = zptr(s4, zs);
    constexpr uint32_t groups = N / RPB;
    const uint32_t blk = xcd_block(blockIdx.x, cd.Kz * groups);
    const int kz = blk / groups, x0 = (blk % groups) * RPB;
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    T* row = lds + r * ROWE;
    cpx<T> g[E];
    gather_runs<T, N, V>(g, s3 + (size_t)blockIdx.y * s3_field + (size_t)kz * cd.Ky * N + x0, (uint32_t)N, cd.Ky,
                         RPB);
    cpx<T> v[E];
    scatter_runs_split<T, N, V>(
        g, lds, row, l, cd.Ky, [&](int q) { return compact_to_pos(q, cd.Kc, N); },
        [&](int p) { return pos_to_compact(p, cd.Kc, N) >= 0; }, v);
    // S4 row (x0 + r, kz)
    cpx<T>* out = s4 + (size_t)blockIdx.y * s4_field + ((size_t)x0 * cd.Kz + kz) * N;
    if constexpr (YZ) {
        cpx<T> w[E];
#pragma unroll
        for (int e = 0; e < E; ++e) w[e] = cscale(v[e], (T)signed_pos(l + P * e, N));
        fft_row_split<PL, +1, T>(w, row, tws, l);
#pragma unroll
        for (int e = 0; e < E; ++e) sto(out, (uint32_t)(r * cd.Kz * N + l + P * e), w[e]);
        out += s4_field;
        wave_sync();  // every lane of this row's team is done with its exchanges
    }
    fft_row_split<PL, +1, T>(v, row, tws, l);
#pragma unroll
    for (int e = 0; e < E; ++e) sto(out, (uint32_t)(r * cd.Kz * N + l + P * e), v[e]);
}

// --------------------------------------------------------------------------
// P5: z pass, inverse to real.  Rows (x, y) along kz of S4 (Kz values).  Job
// j (grid.y) is S4 field f[j] into the real field out[j]; a block holds 2 RPB
// consecutive y at one x, and each complex transform carries rows y and
// y + RPB as its real and imaginary parts, so the block loads runs of 2 RPB
// consecutive y (whole cache lines).  grid.x = N^2 / (2 RPB).
// --------------------------------------------------------------------------
template <typename T>
struct ZJobs {
    int f[8];  // S4 field indices
    T* out[8];
    T* dup[8];  // a second output of the same field, or null
};

template <typename T, int N, int V>
__global__ __launch_bounds__((Rows<T, N, V>::THREADS)) void k_zinv(const cpx<T>* __restrict__ s4, size_t s4_field,
                                                                    ZJobs<T> zj, const cpx<T>* __restrict__ tw,
                                                                    CubeDims cd, size_t zs) {
    using RW = Rows<T, N, V>;
    using PL = typename RW::PL;
    constexpr int P = RW::P, RPB = RW::RPB, ROWE = RW::ROWE, E = RW::E;
    // real-valued exchange rows (split exchange); before the transform the same
    // LDS holds the staged runs as complex rows of SROW >= Kz elements
    __shared__ __align__(16) T lds[RPB * ROWE];
    constexpr int SROW = RW::SROW;
    static_assert(SROW >= N / 2 && 2 * SROW <= ROWE, "a staged row holds every kept kz");
    const int job = blockIdx.y;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const size_t q0 = (size_t)blk * 2 * RPB;  // first row (x N + y) of the block
    // twiddles in LDS for FP32 (this pass's LDS traffic is light), else from the cache
    constexpr bool LT = kLdsTwiddles<T> && true;
    __shared__ cpx<T> twl[LT ? PL::TW_ALLOC : 1];
    if constexpr (LT) load_twiddles<PL, T>(twl, tw);
    __syncthreads();
    const Twiddles<T, PL, LT> tws{LT ? twl : tw};
    s4 = zptr(s4, zs);
    const int r = threadIdx.x / P, l = threadIdx.x % P;
    const int x = (int)(q0 / N), y0 = (int)(q0 % N);
    const cpx<T>* A = s4 + (size_t)zj.f[job] * s4_field + (size_t)x * cd.Kz * N + y0;  // rows y0 + r
    const cpx<T>* B = A + RPB;                                                          // rows y0 + RPB + r
    T* row = lds + r * ROWE;
    // runs of RPB y for every kz, twice (Kz <= N / 2, so E / 2 items per thread), all loads first
    constexpr int IT = E / 2;
    cpx<T> ga[IT], gb[IT];
    gather_runs<T, N, V>(ga, A, (uint32_t)N, cd.Kz, RPB);
    gather_runs<T, N, V>(gb, B, (uint32_t)N, cd.Kz, RPB);
    cpx<T>* stage = reinterpret_cast<cpx<T>*>(lds);
    auto scatter = [&](const cpx<T>(&gg)[IT]) {
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = (int)threadIdx.x + RW::THREADS * it;
            if (idx < cd.Kz * RPB) stage[(idx % RPB) * SROW + idx / RPB] = gg[it];
        }
        __syncthreads();
    };
    // position p of the Hermitian row takes kz = p (p < Kz) or the mirror N - p
    auto src = [&](int p) { return p < cd.Kz ? p : (p > N - cd.Kz ? N - p : 0); };
    scatter(ga);
    cpx<T> av[E];
#pragma unroll
    for (int e = 0; e < E; ++e) av[e] = stage[r * SROW + src(l + P * e)];
    scatter(gb);
    cpx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = l + P * e;
        const cpx<T> bv = stage[r * SROW + src(p)];
        const cpx<T> lo = {av[e].x - bv.y, av[e].y + bv.x};
        const cpx<T> hi = {av[e].x + bv.y, bv.x - av[e].y};
        const cpx<T> zero = {(T)0, (T)0};
        v[e] = p < cd.Kz ? lo : (p > N - cd.Kz ? hi : zero);
    }
    __syncthreads();  // every wave has read the staged runs before the exchanges reuse the LDS
    fft_row_split<PL, +1, T>(v, row, tws, l);
    auto store = [&](T* base) {
        T* out = zptr(base, zs) + q0 * N;
#pragma unroll
        for (int e = 0; e < E; ++e) sto(out, (uint32_t)(r * N + l + P * e), v[e].x);
#pragma unroll
        for (int e = 0; e < E; ++e) sto(out, (uint32_t)((r + RPB) * N + l + P * e), v[e].y);
    };
    store(zj.out[job]);
    if (zj.dup[job]) store(zj.dup[job]);
}

}  // namespace gridspt

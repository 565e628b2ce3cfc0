// Estimator kernels: shell-binned cross spectra (Eq. 19-21), the FFT
// bispectrum estimator's triple-product sums (Eq. 22-23), the weighted sum of
// orders, and the twiddle table.  All sums accumulate in FP64 in a fixed order
// (no floating-point atomics), so results are bitwise reproducible.
#pragma once
#include "fft_engine.hpp"

namespace gridspt {

constexpr int kMaxBins = 256;
constexpr int kMaxFields = 16;
constexpr int kMaxPairs = 64;

// tw[m] = exp(-2 pi i m / N), evaluated in FP64 and rounded once.
template <typename T>
__global__ void k_twiddles(cpx<T>* tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) {
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        tw[m] = {(T)c, (T)(-s)};
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Cross spectra (Eq. 19-21).  Along a half-row of the cube (fixed ky and kz;
// kx >= 0, or kx < 0) |n|^2 = kx^2 + ky^2 + kz^2 grows with a = |kx|, so the
// modes of the half-row inside the bins form one stretch a0 <= a < a1, and
// bin b holds the part [lo_b, hi_b) of it given by integer square roots of
// the bin's edges.  The four half-rows (+ky and -ky; kx >= 0 and kx < 0) of
// one (|ky|, kz) share ky^2 + kz^2 and the weight w, hence every stretch:
// they form one work unit (two half-rows when ky = 0).  A wavefront takes one
// unit at a time:
//  1. lane j takes the j-th bin the unit meets: its stretch of a >= 1 and its
//     number of pieces P_j = ceil(L_j / s), s the least piece length for
//     which the pieces fit the 64 lanes (when fewer than 64 bins are met);
//  2. lane p takes piece p, piece i of bin j: the modes a = lo_j + i + k P_j
//     (k = 0, 1, ...) inside the stretch, in each half-row of the unit, so
//     that the lanes of one bin read consecutive modes of a row.  It sums
//     the per-mode quantities in FP64 registers with no bin test per mode:
//     the products Re[F_a F_b^*], the mode count and sum |k|;
//  3. the pieces' sums go to LDS, and lane j adds those of its bin, in piece
//     order and times w, to the wavefront's own accumulator [bin][q] in LDS;
//     then the kx = 0 modes of the unit's rows, when they lie in the bins.
// Modes outside the bins (k = 0, the corners of the cube past the last edge)
// are never read.  The block partials [block][bin][q] are reduced in a fixed
// order by k_power_reduce: every sum has a fixed order, so the result is
// bitwise reproducible.  Every kernel here takes a realisation stride zs
// (see zptr): gridDim.z realisations in one launch.
// ---------------------------------------------------------------------------
constexpr int kPowerPairsPerLaunch = 16;
constexpr int kPowerWaves = 2;
// Modes of a half-row's stretch staged in LDS at once (six per lane): the
// staged form serves FP32 fields with all pairs of up to five fields
// (TRI > 0) when a stretch fits; others load each mode directly.
constexpr int kPowerStageModes = 384;

template <typename T>
struct PowerArgs {
    const cpx<T>* f[kMaxFields];  // distinct fields used by this launch
    int pa[kPowerPairsPerLaunch], pb[kPowerPairsPerLaunch];  // indices into f
    int nf, npairs, nbins;
    double kF;
    double* partial;  // [gridDim.x][nbins][npairs + 2]
};

// Bin b holds the integer |n|^2 with e[b] <= |n|^2 < e[b + 1].
struct BinEdges {
    int64_t e[kMaxBins + 1];
    int nbins;
};

// LDS of k_power_partial per wavefront, beyond the block's static edge
// table: the accumulators [nbins][nq] (FP64), one region holding either the
// piece sums [64][nq] or a staged stretch (stage_bytes), and the piece table
// (64 x 16 bytes); each part 16-byte aligned.
__host__ __device__ constexpr size_t power_align16(size_t b) { return (b + 15) / 16 * 16; }
__host__ __device__ constexpr size_t power_acc_bytes(int nbins, int nq) {
    return power_align16((size_t)nbins * nq * sizeof(double));
}
__host__ __device__ constexpr size_t power_region_bytes(int nq, size_t stage_bytes) {
    return power_align16((size_t)64 * nq * sizeof(double) > stage_bytes ? (size_t)64 * nq * sizeof(double)
                                                                        : stage_bytes);
}
__host__ __device__ constexpr size_t power_wave_bytes(int nbins, int nq, size_t stage_bytes) {
    return power_acc_bytes(nbins, nq) + power_region_bytes(nq, stage_bytes) + 64 * 4 * sizeof(int);
}
template <typename T, int TRI>
__host__ __device__ constexpr size_t power_stage_bytes() {
    return TRI > 0 && sizeof(T) == 4 ? (size_t)TRI * kPowerStageModes * sizeof(cpx<T>) : 0;
}

// DPP lane moves (VALU, no LDS traffic): row shift right by S within rows of
// 16 lanes, lane 15 of a row to the next row, lane 31 to the upper half.
// Lanes without a source, or in rows outside the row mask, get `old`.
constexpr int kDppRowShr = 0x110, kDppBcast15 = 0x142, kDppBcast31 = 0x143;

// Inclusive prefix sum of v over the 64 lanes: shifts 1, 2, 4, 8 within rows
// of 16, then lane 15 into rows 1 and 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 2, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 4, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 8, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppBcast15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppBcast31, 0xc, 0xf, false);
    return v;
}

// Inclusive running maximum of v over the 64 lanes (lanes without a DPP
// source take INT_MIN, which changes no maximum).
__device__ __forceinline__ int wave_incl_max(int v) {
    constexpr int lo = -0x7fffffff - 1;
    v = max(v, __builtin_amdgcn_update_dpp(lo, v, kDppRowShr + 1, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(lo, v, kDppRowShr + 2, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(lo, v, kDppRowShr + 4, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(lo, v, kDppRowShr + 8, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(lo, v, kDppBcast15, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(lo, v, kDppBcast31, 0xc, 0xf, false));
    return v;
}

// sqrt(n) for an integer 1 <= n < 2^31: the hardware reciprocal square root y,
// then one Goldschmidt step on (x y, y / 2) and one Newton step on the root;
// within about an ulp of the correctly rounded root.
__device__ __forceinline__ double root_of_int(int n) {
    const double x = (double)n, y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = fma(-h, s, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    return fma(fma(-s, s, x), h, s);
}

// The least a >= 0 with a^2 >= x, capped at kc1 (x >= kc1^2 gives kc1, kc1 < 46341):
// the truncated root corrected to the exact floor, then rounded up.
__device__ __forceinline__ int ceil_sqrt(int64_t x, int kc1) {
    if (x <= 0) return 0;
    if (x >= (int64_t)kc1 * kc1) return kc1;
    const int n = (int)x;
    int r = (int)root_of_int(n);
    if (r * r > n) --r;
    if ((r + 1) * (r + 1) <= n) ++r;
    return r * r < n ? r + 1 : r;
}

// ceil(len / s) for 0 <= len, 1 <= s < 2^11, with rs = 1 / s in FP32: the float
// quotient of len + s - 1 is off by at most one and is corrected.
__device__ __forceinline__ int ceil_div_small(int len, int s, float rs) {
    const int x = len + s - 1;
    int q = (int)((float)x * rs);
    if (q * s > x) --q;
    if ((q + 1) * s <= x) ++q;
    return q;
}

// v & m: the AND is written as an instruction so that it stays one VALU
// operation on the loaded word (a select on the converted FP64 value would
// take two)
__device__ __forceinline__ float and_bits(float v, unsigned m) {
    float r;
    asm("v_and_b32 %0, %1, %2" : "=v"(r) : "v"(v), "v"(m));
    return r;
}
__device__ __forceinline__ double and_bits(double v, unsigned m) {
    return __hiloint2double(__float_as_int(and_bits(__int_as_float(__double2hiint(v)), m)),
                            __float_as_int(and_bits(__int_as_float(__double2loint(v)), m)));
}

// Row-major index of the pair (i, j), i <= j, among all pairs of TRI fields.
__host__ __device__ constexpr int tri_index(int i, int j, int tri) { return i * tri - i * (i - 1) / 2 + (j - i); }

// TRI = 0: the npairs requested pairs (pa[q], pb[q]).  TRI = 1..5: every pair
// i <= j of the TRI fields (a.npairs = TRI (TRI + 1) / 2), each field loaded
// once per mode; the requested pairs are picked out by k_power_final.
template <typename T, int TRI>
__global__ __launch_bounds__(64 * kPowerWaves) void k_power_partial(PowerArgs<T> a, BinEdges be, CubeDims cd,
                                                                     size_t zs) {
    constexpr int QP = kPowerPairsPerLaunch;
    constexpr int NP = TRI > 0 ? TRI * (TRI + 1) / 2 : QP;  // pair sums held per lane
    constexpr int NQ = NP + 2;                               // then the mode count and sum |k|
    constexpr int NF = TRI > 0 ? TRI : 2 * QP;               // values loaded per mode
    constexpr int H = TRI == 0 ? 1 : (sizeof(T) == 4 ? 4 : 2);  // direct form: half-rows loaded together
    constexpr bool STAGED = power_stage_bytes<T, TRI>() > 0;
    constexpr int W = kPowerStageModes, WL = W / 64;
    extern __shared__ double smem[];
    __shared__ int64_t edge[kMaxBins + 1];
    // pair sums per mode (TRI > 0: all NP of them), quantities per bin
    const int npairs = TRI > 0 ? NP : a.npairs, Q = npairs + 2, nb = be.nbins;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64), lane = threadIdx.x % 64;
    const size_t wave_bytes = power_wave_bytes(nb, Q, power_stage_bytes<T, TRI>());
    auto acc_of = [&](int wv) { return reinterpret_cast<double*>(reinterpret_cast<char*>(smem) + wv * wave_bytes); };
    for (int i = threadIdx.x; i < kPowerWaves * nb * Q; i += blockDim.x) acc_of(i / (nb * Q))[i % (nb * Q)] = 0.0;
    for (int i = threadIdx.x; i <= nb; i += blockDim.x) edge[i] = be.e[i];
    __syncthreads();
    double* acc = acc_of(wave);  // [nbins][Q]
    char* region = reinterpret_cast<char*>(acc) + power_acc_bytes(nb, Q);
    double* stage = reinterpret_cast<double*>(region);  // [64][Q] piece sums
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(region);    // [NF][W] a staged stretch
    int4* piece = reinterpret_cast<int4*>(region + power_region_bytes(Q, power_stage_bytes<T, TRI>()));
    // the launch's field of load slot i (TRI > 0: field i; else pair i / 2, side i % 2)
    auto field = [&](int i) -> const cpx<T>* {
        if constexpr (TRI > 0) return zptr(a.f[i], zs);
        else return zptr(a.f[(i & 1) ? a.pb[i >> 1] : a.pa[i >> 1]], zs);
    };
    // the unweighted products of one mode (values x) added to v; MASK: x & m
    auto add_mode = [&](auto mask_tag, const cpx<T>(&x)[NF], unsigned m, double(&v)[NQ]) {
        constexpr bool MASK = decltype(mask_tag)::value;
        auto cv = [&](T t) -> double { return (double)(MASK ? and_bits(t, m) : t); };
        if constexpr (TRI > 0) {
            double re[TRI], im[TRI];
#pragma unroll
            for (int i = 0; i < TRI; ++i) {
                re[i] = cv(x[i].x);
                im[i] = cv(x[i].y);
            }
#pragma unroll
            for (int i = 0; i < TRI; ++i)
#pragma unroll
                for (int i2 = i; i2 < TRI; ++i2) {
                    double& t = v[tri_index(i, i2, TRI)];
                    t = fma(re[i], re[i2], t);
                    t = fma(im[i], im[i2], t);
                }
        } else {
#pragma unroll
            for (int q = 0; q < QP; ++q) {
                if (q < npairs) {
                    v[q] = fma(cv(x[2 * q].x), cv(x[2 * q + 1].x), v[q]);
                    v[q] = fma(cv(x[2 * q].y), cv(x[2 * q + 1].y), v[q]);
                }
            }
        }
    };
    const int Kc = cd.Kc, Kx = cd.Ky, kc1 = cd.Kc + 1;
    const int nunit = kc1 * kc1;  // (|ky|, kz)
    const int gw = blockIdx.x * kPowerWaves + wave, nw = gridDim.x * kPowerWaves;
    for (int uu = gw; uu < nunit; uu += nw) {
        // everything of the unit is uniform over the wavefront
        const int u = __builtin_amdgcn_readfirstlane(uu);
        const int kz = u / kc1, ky = u - kz * kc1;  // ky = |ky|
        const int c2 = ky * ky + kz * kz;
        // the modes in the bins: a0 <= a < a1, a = |kx|
        const int a0 = __builtin_amdgcn_readfirstlane(ceil_sqrt(edge[0] - c2, kc1));
        const int a1 = __builtin_amdgcn_readfirstlane(ceil_sqrt(edge[nb] - c2, kc1));
        if (a0 >= a1) continue;
        const double w = kz == 0 ? 1.0 : 2.0;
        const int nrow = ky > 0 ? 2 : 1, nh = 2 * nrow;  // rows +ky, -ky; their half-rows
        const int rowp = kz * cd.Ky + ky, rowm = kz * cd.Ky + (ky > 0 ? cd.Ky - ky : 0);
        const int s1 = max(1, a0), L = max(0, a1 - s1);  // the pieces cover a >= 1 in every half-row
        // bins of the first and the last mode: the number of upper edges at or below their |n|^2
        const int64_t n2f = (int64_t)a0 * a0 + c2, n2l = (int64_t)(a1 - 1) * (a1 - 1) + c2;
        int bf = 0, bl = 0;
        for (int g = 0; g < nb; g += 64) {
            const int e = g + lane + 1;
            const int64_t up = e <= nb ? edge[e] : (int64_t)0x7fffffffffffffffll;
            bf += __popcll(__ballot(up <= n2f));
            bl += __popcll(__ballot(up <= n2l));
        }
        const int nbr = bl - bf + 1;  // bins the unit meets (some may hold no mode)
        const bool staged = L <= W;   // the stretch fits the LDS window
        for (int g0 = 0; g0 < nbr; g0 += 64) {
            // lane j: bin b = bf + g0 + j, its stretch [lo, hi) of a >= s1
            const int j = g0 + lane, b = bf + j;
            int lo = 0, hi = 0;
            if (j < nbr) {
                lo = max(s1, ceil_sqrt(edge[b] - c2, kc1));
                hi = min(a1, ceil_sqrt(edge[b + 1] - c2, kc1));
            }
            const int len = max(0, hi - lo);
            // piece length s: the least for which the group's pieces fit 64 lanes, searched
            // between an even split of the stretch and a length that fits (or about twice
            // the even split, the most allowed: then the pieces take several rounds)
            const int ng = min(64, nbr - g0);
            const int even = max(1, (L + 63) / 64);
            int slo = even, shi = ng < 64 ? max(even, min((L + 63 - ng) / (64 - ng), 2 * even + 2)) : even;
            while (slo < shi) {
                const int mid = (slo + shi) >> 1;
                const int t = __builtin_amdgcn_readlane(wave_incl_scan(ceil_div_small(len, mid, 1.0f / (float)mid)), 63);
                if (t <= 64) shi = mid;
                else slo = mid + 1;
            }
            const int s = slo;
            const int np = ceil_div_small(len, s, 1.0f / (float)s);
            const int incl = wave_incl_scan(np);
            const int off = incl - np;                            // first piece of bin j
            const int npc = __builtin_amdgcn_readlane(incl, 63);  // pieces of this group of bins
            for (int r0 = 0; r0 < npc; r0 += 64) {
                // bin lanes: the table entry of each of their pieces in this round
                const int t0 = max(off, r0), t1 = min(off + np, r0 + 64);
                for (int t = t0; t < t1; ++t) piece[t - r0] = make_int4(lo + (t - off), np, hi, 0);
                wave_sync();
                // piece lanes: modes d.x + k d.y < d.z; a lane past the last piece has none
                const bool act = r0 + lane < npc;
                const int4 d = act ? piece[lane] : make_int4(s1, 1, s1, 0);
                double v[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) v[q] = 0.0;
                // mode k of every piece lane: MASK when some piece lane has no mode k
                auto trip = [&](auto mask_tag, int k) {
                    constexpr bool MASK = decltype(mask_tag)::value;
                    const int m = d.x + k * d.y;
                    const bool ok = m < d.z;
                    const int am = ok ? m : s1;  // a mode of the stretch: the loads stay in their rows
                    const unsigned mk = ok ? 0xffffffffu : 0u;
                    // the unit's half-rows h = 2 r + half (row r: +ky, -ky), H at a time
                    auto load = [&](int h, cpx<T>(&x)[NF]) {
                        const int row = (h >> 1) && h < nh ? rowm : rowp;  // h >= nh (ky = 0): row +ky again
                        const uint32_t o = (uint32_t)((h & 1) ? Kx - am : am);
#pragma unroll
                        for (int i = 0; i < NF; ++i)
                            if (TRI > 0 || i < 2 * npairs) x[i] = ldo(field(i) + (size_t)row * Kx, o);
                    };
                    if constexpr (H == 1) {
#pragma unroll 1
                        for (int h = 0; h < nh; ++h) {
                            cpx<T> x[NF];
                            load(h, x);
                            add_mode(mask_tag, x, mk, v);
                        }
                    } else {
#pragma unroll
                        for (int hb = 0; hb < 4; hb += H) {
                            if (hb >= nh) break;  // uniform
                            cpx<T> xs[H][NF];
#pragma unroll
                            for (int hh = 0; hh < H; ++hh) load(hb + hh, xs[hh]);
#pragma unroll
                            for (int hh = 0; hh < H; ++hh)
                                if (hb + hh < nh) add_mode(mask_tag, xs[hh], mk, v);
                        }
                    }
                    const double cnt = nh, ks = a.kF * nh;
                    v[NP] += MASK ? and_bits(cnt, mk) : cnt;
                    v[NP + 1] = fma(MASK ? and_bits(ks, mk) : ks, root_of_int(am * am + c2), v[NP + 1]);
                };
                // modes per piece: every piece lane has the first kmin, some have up to kmax
                const int cnt = act ? ceil_div_small(d.z - d.x, d.y, 1.0f / (float)d.y) : 0;
                const int kmax = __builtin_amdgcn_readlane(wave_incl_max(cnt), 63);
                const int kmin = __builtin_amdgcn_readlane(wave_incl_max(act ? -cnt : -kmax), 63) * -1;
                if (STAGED && staged) {
                    // half-row by half-row: its stretch [s1, a1) (positions c0 .. c0 + L - 1 of the
                    // row, ascending) is read with coalesced loads into LDS, the next half-row's
                    // loads in flight while the pieces of this one read theirs from LDS
                    cpx<T> xs[WL][NF];
                    auto issue = [&](int h) {
                        const int row = (h >> 1) ? rowm : rowp;
                        const int c0 = (h & 1) ? Kx - (a1 - 1) : s1;
#pragma unroll
                        for (int t = 0; t < WL; ++t) {
                            if (t * 64 < L) {  // uniform
                                const uint32_t o = (uint32_t)(c0 + min(t * 64 + lane, L - 1));
#pragma unroll
                                for (int i = 0; i < NF; ++i) xs[t][i] = ldo(field(i) + (size_t)row * Kx, o);
                            }
                        }
                    };
                    issue(0);
                    for (int h = 0; h < nh; ++h) {
                        wave_sync();  // the previous half-row's reads of buf are done
#pragma unroll
                        for (int t = 0; t < WL; ++t)
                            if (t * 64 < L)
#pragma unroll
                                for (int i = 0; i < NF; ++i) buf[i * W + t * 64 + lane] = xs[t][i];
                        wave_sync();
                        if (h + 1 < nh) issue(h + 1);
                        // mode a of this half-row sits at LDS index a - s1 (kx >= 0) or a1 - 1 - a
                        const bool neg = h & 1, first = h == 0;
                        auto trip_lds = [&](auto mask_tag, int k) {
                            constexpr bool MASK = decltype(mask_tag)::value;
                            const int m = d.x + k * d.y;
                            const bool ok = m < d.z;
                            const int am = ok ? m : s1;
                            const unsigned mk = ok ? 0xffffffffu : 0u;
                            const int idx = neg ? a1 - 1 - am : am - s1;
                            cpx<T> x[NF];
#pragma unroll
                            for (int i = 0; i < NF; ++i) x[i] = buf[i * W + idx];
                            add_mode(mask_tag, x, mk, v);
                            if (first) {  // the count and sum |k| of all nh half-rows
                                const double cnt = nh, ks = a.kF * nh;
                                v[NP] += MASK ? and_bits(cnt, mk) : cnt;
                                v[NP + 1] = fma(MASK ? and_bits(ks, mk) : ks, root_of_int(am * am + c2), v[NP + 1]);
                            }
                        };
                        int k = 0;
                        for (; k < kmin; ++k) trip_lds(std::false_type{}, k);
                        for (; k < kmax; ++k) trip_lds(std::true_type{}, k);
                    }
                    wave_sync();  // buf is read before the piece sums take its place
                } else {
                    int k = 0;
                    for (; k < kmin; ++k) trip(std::false_type{}, k);
                    for (; k < kmax; ++k) trip(std::true_type{}, k);
                }
                if (act) {
                    double* dst = stage + lane * Q;
#pragma unroll
                    for (int q = 0; q < NP; ++q)
                        if (q < npairs) dst[q] = v[q];
                    dst[npairs] = v[NP];
                    dst[npairs + 1] = v[NP + 1];
                }
                wave_sync();
                // bin lanes: their pieces of this round in order, weighted, into the accumulator
                if (t1 > t0) {
                    double sum[NQ];
#pragma unroll
                    for (int q = 0; q < NQ; ++q) sum[q] = 0.0;
                    for (int t = t0; t < t1; ++t) {
                        const double* src = stage + (t - r0) * Q;
#pragma unroll
                        for (int q = 0; q < NQ; ++q)
                            if (q < Q) sum[q] += src[q];
                    }
                    double* dst = acc + (size_t)b * Q;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (q < Q) dst[q] += w * sum[q];
                }
                wave_sync();
            }
        }
        // the kx = 0 mode of each row (one half-row holds it), in bin bf when a0 = 0
        if (a0 == 0 && lane == 0) {
            double z[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) z[q] = 0.0;
            for (int r = 0; r < nrow; ++r) {
                cpx<T> x[NF];
#pragma unroll
                for (int i = 0; i < NF; ++i)
                    if (TRI > 0 || i < 2 * npairs) x[i] = field(i)[(size_t)(r ? rowm : rowp) * Kx];
                add_mode(std::false_type{}, x, 0u, z);
            }
            z[NP] = (double)nrow;
            z[NP + 1] = a.kF * nrow * root_of_int(c2);
            double* dst = acc + (size_t)bf * Q;
#pragma unroll
            for (int q = 0; q < NP; ++q)
                if (q < npairs) dst[q] += w * z[q];
            dst[npairs] += w * z[NP];
            dst[npairs + 1] += w * z[NP + 1];
        }
        wave_sync();
    }
    __syncthreads();
    double* out = zptr(a.partial, zs) + (size_t)blockIdx.x * nb * Q;
    for (int i = threadIdx.x; i < nb * Q; i += blockDim.x) {
        double sum = 0.0;
        for (int wv = 0; wv < kPowerWaves; ++wv) sum += acc_of(wv)[i];
        out[i] = sum;
    }
}

// One block per item (gridDim.x items, e.g. bin * nq + q): sum the block
// partials [nblocks][items] in a fixed order (strided per thread, then an LDS
// tree) into sums[item].
constexpr int kReduceThreads = 256;
static __global__ __launch_bounds__(kReduceThreads) void k_power_reduce(const double* partial, int nblocks,
                                                                 double* sums, size_t zs) {
    __shared__ double red[kReduceThreads];
    partial = zptr(partial, zs);
    sums = zptr(sums, zs);
    const int item = blockIdx.x;  // bin * nq + q
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kReduceThreads) s += partial[(size_t)i * gridDim.x + item];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[item] = red[0];
}

// P = L^3 S / sum w, kmean = sum w |k| / sum w, nmodes = sum w; output pair p
// is column col[p] of the sums [bin][nq] (the last two columns are sum w and
// sum w |k|).
struct PairCols {
    int col[kPowerPairsPerLaunch];
};
static __global__ void k_power_final(const double* sums, int nbins, int nq, int npairs, PairCols pc, double vol,
                                     double* pk, int pk_stride, double* kmean, double* nmodes, size_t zs) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    sums = zptr(sums, zs);
    pk = zptr(pk, zs);
    kmean = zptr(kmean, zs);
    nmodes = zptr(nmodes, zs);
    if (b >= nbins) return;
    const double cnt = sums[(size_t)b * nq + nq - 2], ks = sums[(size_t)b * nq + nq - 1];
    if (nmodes) nmodes[b] = cnt;
    if (kmean) kmean[b] = cnt > 0.0 ? ks / cnt : 0.0;
    for (int p = 0; p < npairs; ++p)
        pk[(size_t)p * pk_stride + b] = cnt > 0.0 ? vol * sums[(size_t)b * nq + pc.col[p]] / cnt : 0.0;
}

// ---------------------------------------------------------------------------
// Triple products sum_x I_a(x) I_b(x) I_c(x) for up to 8 terms per launch,
// FP64 per thread, fixed-order block tree, partials [block][term].
// ---------------------------------------------------------------------------
template <typename T>
struct TripleArgs {
    const T* a[8];
    const T* b[8];
    const T* c[8];
    int nterms;
    size_t ncell;
    double* partial;  // [gridDim.x][8]
};

constexpr int kTripleThreads = 256;

// NT terms (the launch's nterms).  A thread takes 16 bytes of consecutive cells
// of every factor per step, all 3 NT loads before the first product, so the
// loads of a step are in flight together; the factors are 16-byte aligned and
// ncell is a multiple of the vector width (checked by the caller).
template <typename T, int NT>
__global__ __launch_bounds__(kTripleThreads) void k_triple_partial(TripleArgs<T> t, size_t zs) {
    __shared__ double red[kTripleThreads];
    constexpr int VW = 16 / (int)sizeof(T);
    using Vec = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const Vec* pa[NT];
    const Vec* pb[NT];
    const Vec* pc[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        pa[u] = reinterpret_cast<const Vec*>(zptr(t.a[u], zs));
        pb[u] = reinterpret_cast<const Vec*>(zptr(t.b[u], zs));
        pc[u] = reinterpret_cast<const Vec*>(zptr(t.c[u], zs));
    }
    double* partial = zptr(t.partial, zs);
    double s[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) s[u] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x, nvec = t.ncell / VW;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) {
        Vec va[NT], vb[NT], vc[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            va[u] = pa[u][i];
            vb[u] = pb[u][i];
            vc[u] = pc[u][i];
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const T* x = reinterpret_cast<const T*>(&va[u]);
            const T* y = reinterpret_cast<const T*>(&vb[u]);
            const T* z = reinterpret_cast<const T*>(&vc[u]);
#pragma unroll
            for (int k = 0; k < VW; ++k) s[u] += (double)x[k] * (double)y[k] * (double)z[k];
        }
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        red[threadIdx.x] = s[u];
        __syncthreads();
        for (int h = kTripleThreads / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * 8 + u] = red[0];
        __syncthreads();
    }
}

// sums of the block partials, item u to out[dst.idx[u]]: per item a strided
// sum per thread, then a fixed-order LDS tree (one block of kReduceThreads)
struct TripleDst {
    int idx[8];
};
static __global__ __launch_bounds__(kReduceThreads) void k_triple_final(const double* partial, int nblocks,
                                                                        int nterms, TripleDst dst, double* out,
                                                                        size_t zs) {
    __shared__ double red[kReduceThreads];
    partial = zptr(partial, zs);
    out = zptr(out, zs);
    for (int u = 0; u < nterms; ++u) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblocks; i += kReduceThreads) s += partial[(size_t)i * 8 + u];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[dst.idx[u]] = red[0];
        __syncthreads();
    }
}

// ntriangles = N^-3 J rounded to the nearest integer (J comes from FP64
// indicator transforms, so N^-3 J lies within far less than 1/2 of the count
// of closed triangles) for triangles u0 .. u0+nt-1, and bk = L^6 N^-3 T /
// ntriangles for terms u0 .. u0+nu-1.
struct TriMap {
    int tri[64];  // triangle of term u0 + i
    int rep[64];  // the term whose sum term u0 + i takes
};
// jzs: realisation stride of jsum (0 when the triangle counts are shared)
static __global__ void k_bisp_final(const double* tsum, const double* jsum, TriMap m, int u0, int nu, int nt,
                                    double vol2, double invN3, double* bk, double* ntriangles, size_t zs,
                                    size_t jzs) {
    const int i = threadIdx.x;
    tsum = zptr(tsum, zs);
    jsum = zptr(jsum, jzs);
    bk = zptr(bk, zs);
    ntriangles = zptr(ntriangles, zs);
    if (i < nu) {
        const double cnt = rint(jsum[m.tri[i]] * invN3);
        bk[u0 + i] = cnt != 0.0 ? vol2 * (tsum[m.rep[i]] * invN3) / cnt : 0.0;
    }
    if (i < nt) ntriangles[u0 + i] = rint(jsum[u0 + i] * invN3);
}

// out(x) = sum_n coef_n delta_n(x) in FP64
template <typename T>
struct SumArgs {
    const T* d[8];
    double coef[8];
    int nmax;
    size_t ncell;
    double* out;
};

template <typename T, int NMAX>
__global__ void k_sum_orders(SumArgs<T> s) {
    // four consecutive cells per thread and iteration (ncell is a multiple of 4); the
    // loads of every order go out before the sums, which add the orders in turn
    static_assert(NMAX >= 1 && NMAX <= 8, "orders per sum");
    using V4 = HIP_vector_type<T, 4>;
    const size_t n4 = s.ncell / 4;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        V4 v[NMAX];
#pragma unroll
        for (int n = 0; n < NMAX; ++n) v[n] = reinterpret_cast<const V4*>(s.d[n])[i];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int n = 0; n < NMAX; ++n) {
            acc[0] += s.coef[n] * (double)v[n].x;
            acc[1] += s.coef[n] * (double)v[n].y;
            acc[2] += s.coef[n] * (double)v[n].z;
            acc[3] += s.coef[n] * (double)v[n].w;
        }
        double2* o = reinterpret_cast<double2*>(s.out + 4 * i);
        o[0] = make_double2(acc[0], acc[1]);
        o[1] = make_double2(acc[2], acc[3]);
    }
}

// ---------------------------------------------------------------------------
// Input check (GRIDSPT_CHECK_FINITE): *flag = 1 if any of the n values of f is
// a NaN or an infinity.  Every writer stores the same value, so the unordered
// stores need no atomic.  n is a multiple of 4 and f 16-byte aligned.
// ---------------------------------------------------------------------------
static __global__ void k_clear_word(uint32_t* w) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *w = 0u;
}

template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite(const T* __restrict__ f, size_t n, uint32_t* flag) {
    using Vec = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int VW = 16 / (int)sizeof(T);
    const Vec* fv = reinterpret_cast<const Vec*>(f);
    const size_t nv = n / VW, stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const Vec v = fv[i];
        const T* x = reinterpret_cast<const T*>(&v);
#pragma unroll
        for (int k = 0; k < VW; ++k) bad = bad || !isfinite(x[k]);
    }
    if (__any(bad) && (threadIdx.x % 64) == 0) *flag = 1u;
}

// ---------------------------------------------------------------------------
// A cube-layout spectrum in the half layout [ix][iy][iz] (N x N x (N/2 + 1)
// complex, zero outside the cube): one output element per thread and step,
// consecutive threads on consecutive outputs.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_spectrum_half(const cpx<T>* __restrict__ cube, cpx<T>* __restrict__ half,
                                                       int n, CubeDims cd) {
    const int h = n / 2 + 1;
    const size_t total = (size_t)n * n * h, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int iz = (int)(i % h);
        const size_t r = i / h;
        const int iy = (int)(r % n), ix = (int)(r / n);
        const int ky = iy < n / 2 ? iy : iy - n, kx = ix < n / 2 ? ix : ix - n;
        const bool in = iz <= cd.Kc && abs(ky) <= cd.Kc && abs(kx) <= cd.Kc;
        const int cy = ky >= 0 ? ky : ky + cd.Ky, cx = kx >= 0 ? kx : kx + cd.Ky;
        const size_t at = in ? ((size_t)iz * cd.Ky + cy) * cd.Ky + cx : 0;
        const cpx<T> v = cube[at];  // unconditional: no branch around the load
        half[i] = in ? v : cpx<T>{(T)0, (T)0};
    }
}

// copy a real field (theta_1 = delta_1)
template <typename T>
__global__ void k_copy(const T* __restrict__ src, T* __restrict__ dst, size_t n, size_t zs) {
    src = zptr(src, zs);
    dst = zptr(dst, zs);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Reverse mode of the products of order NORD (V = sum_m delta_m u_{n-m},
// W = sum_m u_m . u_{n-m}): with g V, g W the gradients of the sources, for
// every i < n
//   g delta_i += g V . u_{n-i},   g u_i += g V delta_{n-i} + 2 g W u_{n-i}.
// first: the accumulators start from g delta_in (the objective's gradient)
// and zero instead of their stored values.
template <typename T>
struct AdjProducts {
    const T* gv[4];     // g V_x, g V_y, g V_z, g W
    const T* d[4];      // delta_1 .. delta_{n-1}
    const T* u[4][3];   // u_1 .. u_{n-1}
    const T* gd_in[4];  // objective gradients of delta_1 .. delta_{n-1}
    T* gd[4];           // accumulators
    T* gu[4][3];
    size_t ncell;
};

template <typename T, int NORD>
__global__ __launch_bounds__(256) void k_adj_products(AdjProducts<T> a, int first) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell; c += stride) {
        const T gx = a.gv[0][c], gy = a.gv[1][c], gz = a.gv[2][c], gw = a.gv[3][c];
#pragma unroll
        for (int i = 1; i < NORD; ++i) {
            const int j = NORD - i;  // partner order
            const T dj = a.d[j - 1][c];
            const T ux = a.u[j - 1][0][c], uy = a.u[j - 1][1][c], uz = a.u[j - 1][2][c];
            T gdi = gx * ux + gy * uy + gz * uz;
            T g0 = gx * dj + (T)2 * gw * ux, g1 = gy * dj + (T)2 * gw * uy, g2 = gz * dj + (T)2 * gw * uz;
            if (first) {
                gdi += a.gd_in[i - 1][c];
            } else {
                gdi += a.gd[i - 1][c];
                g0 += a.gu[i - 1][0][c];
                g1 += a.gu[i - 1][1][c];
                g2 += a.gu[i - 1][2][c];
            }
            a.gd[i - 1][c] = gdi;
            a.gu[i - 1][0][c] = g0;
            a.gu[i - 1][1][c] = g1;
            a.gu[i - 1][2][c] = g2;
        }
    }
}

// The printed sources of Eq. 10 for order NORD from the derived fields of the
// earlier orders (17 per order: delta, theta, grad delta (3), grad theta (3),
// u (3), d_i u_j (6: xx, yy, zz, xy, xz, yz)):
//   S_delta = sum_m (grad delta_m) . u_{n-m} + delta_m theta_{n-m}
//   S_theta = sum_m [d_j u_{m,k}][d_k u_{n-m,j}] + u_m . grad theta_{n-m}
template <typename T>
struct PFormProducts {
    const T* f[4][17];  // orders 1 .. n-1: delta, theta, gd x3, gt x3, u x3, du x6
    T* sd;
    T* st;
    size_t ncell;
};

template <typename T, int NORD>
__global__ __launch_bounds__(256) void k_pform_products(PFormProducts<T> a) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell; c += stride) {
        T v[NORD][17];
#pragma unroll
        for (int m = 1; m < NORD; ++m)
#pragma unroll
            for (int q = 0; q < 17; ++q) v[m][q] = a.f[m - 1][q][c];
        T sdel = 0, sthe = 0;
#pragma unroll
        for (int m = 1; m < NORD; ++m) {
            const T* A = v[m];
            const T* B = v[NORD - m];
            sdel += A[2] * B[8] + A[3] * B[9] + A[4] * B[10] + A[0] * B[1];
            // symmetric d_i u_j: diagonal once, off-diagonal twice
            sthe += A[11] * B[11] + A[12] * B[12] + A[13] * B[13] +
                    (T)2 * (A[14] * B[14] + A[15] * B[15] + A[16] * B[16]);
            sthe += A[8] * B[5] + A[9] * B[6] + A[10] * B[7];
        }
        a.sd[c] = sdel;
        a.st[c] = sthe;
    }
}

// ---------------------------------------------------------------------------
// One-point statistics of real fields (Sec. III A-B): FP64 sums of x, x^2, x^3,
// x^4 per field and x_a x_b per pair (fixed-order block trees, then the
// fixed-order reduction of k_power_reduce), and histograms: per-block counts
// in LDS (integer LDS atomics; the count does not depend on their order), then
// an integer sum over blocks.  Bin b = floor((x - lo) * scale) in FP64,
// values outside [0, nbins) dropped.
// ---------------------------------------------------------------------------
constexpr int kStatsMaxFields = 8;
constexpr int kStatsQ = 4 * kStatsMaxFields + kStatsMaxFields * (kStatsMaxFields - 1) / 2;  // 60
constexpr int kStatsThreads = 256;

template <typename T>
struct MomentArgs {
    const T* f[kStatsMaxFields];
    int nf;
    size_t ncell;
    double* partial;  // [gridDim.x][kStatsQ]
    // one-point histograms (k_moments_partial<T, NF, true>): nbins bins of width
    // 1 / scale from lo, per-block counts [nf][gridDim.x][nbins]; hcopies LDS
    // copies (one per wavefront, or one per block when those would not fit)
    uint32_t* hpart;
    int nbins, hcopies;
    double lo, scale;
};

__host__ __device__ constexpr int pair_index(int i, int j) {  // i < j < 8
    return i * kStatsMaxFields - i * (i + 1) / 2 + (j - i - 1);
}

template <typename T>
__device__ __forceinline__ int bin_of(T x, double lo, double scale, int nbins) {
    const double fb = floor(((double)x - lo) * scale);
    return (fb >= 0.0 && fb < (double)nbins) ? (int)fb : -1;
}

// NF = a.nf fields, a template argument so that every load of a cell is
// unconditional and all of them are in flight together.  HIST: the same pass
// also counts every field's one-point histogram, each wavefront into its own
// LDS copy (fewer lanes collide on one bin's atomic; counts are integers, so
// the order does not matter), so the fields are read once for both.
template <typename T, int NF, bool HIST>
__global__ __launch_bounds__(kStatsThreads) void k_moments_partial(MomentArgs<T> a) {
    __shared__ double red[kStatsQ * (kStatsThreads / 64)];
    extern __shared__ uint32_t hl[];  // HIST: [hcopies][NF][nbins]
    const int hsize = NF * a.nbins;
    if constexpr (HIST) {
        for (int i = threadIdx.x; i < a.hcopies * hsize; i += blockDim.x) hl[i] = 0u;
        __syncthreads();
    }
    uint32_t* hw = hl + (int)(threadIdx.x / 64) % (a.hcopies > 0 ? a.hcopies : 1) * hsize;
    double s[kStatsMaxFields][4], x[kStatsQ - 4 * kStatsMaxFields];
#pragma unroll
    for (int i = 0; i < kStatsMaxFields; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) s[i][q] = 0.0;
#pragma unroll
    for (int i = 0; i < kStatsQ - 4 * kStatsMaxFields; ++i) x[i] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell; c += stride) {
        double v[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) v[i] = (double)a.f[i][c];
        if constexpr (HIST) {
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const int b = bin_of(v[i], a.lo, a.scale, a.nbins);
                if (b >= 0) atomicAdd(&hw[i * a.nbins + b], 1u);
            }
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const double p2 = v[i] * v[i];
            s[i][0] += v[i];
            s[i][1] += p2;
            s[i][2] += p2 * v[i];
            s[i][3] += p2 * p2;
#pragma unroll
            for (int j = i + 1; j < NF; ++j) x[pair_index(i, j)] += v[i] * v[j];
        }
    }
    // per item: butterfly sum within each wavefront (fixed order), then the
    // wavefront totals in wave order
    constexpr int NW = kStatsThreads / 64;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    double* out = a.partial + (size_t)blockIdx.x * kStatsQ;
#pragma unroll
    for (int q = 0; q < kStatsQ; ++q) {
        const double t = wave_sum(q < 4 * kStatsMaxFields ? s[q / 4][q % 4] : x[q - 4 * kStatsMaxFields]);
        if (lane == 0) red[q * NW + wave] = t;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kStatsQ; q += blockDim.x) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += red[q * NW + w];
        out[q] = t;
    }
    if constexpr (HIST) {
        // the waves' counts of this block (the barrier above ordered every atomic)
        for (int i = threadIdx.x; i < hsize; i += blockDim.x) {
            uint32_t t = 0u;
            for (int w = 0; w < a.hcopies; ++w) t += hl[w * hsize + i];
            const int f = i / a.nbins, b = i % a.nbins;
            a.hpart[((size_t)f * gridDim.x + blockIdx.x) * a.nbins + b] = t;
        }
    }
}

// moments [nf][4]: mean, variance, skewness, excess kurtosis; corr [nf][nf]: Pearson r
static __global__ void k_moments_final(const double* sums, int nf, double ncell, double* moments, double* corr) {
    const int t = threadIdx.x;
    auto mean_var = [&](int i, double& m, double& v) {
        m = sums[4 * i] / ncell;
        v = sums[4 * i + 1] / ncell - m * m;
    };
    if (t < nf && moments) {
        double m, v;
        mean_var(t, m, v);
        const double e3 = sums[4 * t + 2] / ncell, e2 = sums[4 * t + 1] / ncell, e4 = sums[4 * t + 3] / ncell;
        const double c3 = e3 - 3.0 * m * e2 + 2.0 * m * m * m;
        const double c4 = e4 - 4.0 * m * e3 + 6.0 * m * m * e2 - 3.0 * m * m * m * m;
        moments[4 * t] = m;
        moments[4 * t + 1] = v;
        moments[4 * t + 2] = v > 0.0 ? c3 / (v * sqrt(v)) : 0.0;
        moments[4 * t + 3] = v > 0.0 ? c4 / (v * v) - 3.0 : 0.0;
    }
    if (t < nf * nf && corr) {
        const int i = t / nf, j = t % nf;
        double mi, vi, mj, vj;
        mean_var(i, mi, vi);
        mean_var(j, mj, vj);
        double cov;
        if (i == j) cov = vi;
        else {
            const int a = i < j ? i : j, b = i < j ? j : i;
            cov = sums[4 * kStatsMaxFields + pair_index(a, b)] / ncell - mi * mj;
        }
        corr[t] = (vi > 0.0 && vj > 0.0) ? cov / sqrt(vi * vj) : 0.0;
    }
}

template <typename T>
struct HistArgs {
    const T* f[kStatsMaxFields];
    int nbins;  // per axis
    double lo, scale;
    size_t ncell;
    uint32_t* partial;  // [gridDim.y][gridDim.x][nbins^2]
};

// Joint histogram of field 0 and field 1 + blockIdx.y.  Each wavefront counts
// into its own LDS histogram (fewer lanes collide on one bin's atomic), the
// block adds its wavefronts' counts at the end; counts are integers, so the
// order does not matter.  A thread takes 16 bytes of consecutive cells of
// each field per step (the tail, if any, one cell at a time).
template <typename T>
__global__ __launch_bounds__(kStatsThreads) void k_joint_partial(HistArgs<T> a) {
    extern __shared__ uint32_t h[];  // [waves][nbins^2]
    constexpr int NW = kStatsThreads / 64;
    const int nb = a.nbins * a.nbins;
    for (int i = threadIdx.x; i < NW * nb; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    uint32_t* hw = h + (threadIdx.x / 64) * nb;
    const T* x = a.f[0];
    const T* y = a.f[1 + blockIdx.y];
    auto count = [&](T xv, T yv) {
        const int b = bin_of(xv, a.lo, a.scale, a.nbins);
        const int b2 = bin_of(yv, a.lo, a.scale, a.nbins);
        if (b >= 0 && b2 >= 0) atomicAdd(&hw[b * a.nbins + b2], 1u);
    };
    // U vectors per thread per step, all loaded before the first is counted
    constexpr int VW = 16 / (int)sizeof(T), U = 4;
    using Vec = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const size_t stride = (size_t)gridDim.x * blockDim.x, nv = a.ncell / VW, nstep = nv / (U * stride);
    const Vec* xv = reinterpret_cast<const Vec*>(x);
    const Vec* yv = reinterpret_cast<const Vec*>(y);
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t s = 0; s < nstep; ++s) {
        Vec vx[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vx[u] = xv[(s * U + u) * stride + t0];
            vy[u] = yv[(s * U + u) * stride + t0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T* px = reinterpret_cast<const T*>(&vx[u]);
            const T* py = reinterpret_cast<const T*>(&vy[u]);
#pragma unroll
            for (int k = 0; k < VW; ++k) count(px[k], py[k]);
        }
    }
    // the remaining vectors one at a time, then the cells past the last whole vector
    for (size_t c = nstep * U * stride + t0; c < nv; c += stride) {
        const Vec vx = xv[c], vy = yv[c];
        const T* px = reinterpret_cast<const T*>(&vx);
        const T* py = reinterpret_cast<const T*>(&vy);
#pragma unroll
        for (int k = 0; k < VW; ++k) count(px[k], py[k]);
    }
    for (size_t c = nv * VW + t0; c < a.ncell; c += stride) count(x[c], y[c]);
    __syncthreads();
    uint32_t* out = a.partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * nb;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        uint32_t t = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += h[w * nb + i];
        out[i] = t;
    }
}

// counts[y][bin] = sum over blocks (exact integers), as doubles.  Block
// (kHistRedBins, kHistRedSlices): lane x owns one bin of this block's run of
// kHistRedBins bins (coalesced reads along the partial rows), row w sums the
// partial blocks w, w + kHistRedSlices, ...; the slices meet in LDS.
constexpr int kHistRedBins = 64, kHistRedSlices = 16;
static __global__ __launch_bounds__(kHistRedBins* kHistRedSlices) void k_hist_reduce(const uint32_t* partial,
                                                                                     int nblocks, int nb,
                                                                                     double* counts) {
    __shared__ uint64_t part[kHistRedSlices][kHistRedBins];
    const int b = blockIdx.x * kHistRedBins + threadIdx.x, y = blockIdx.y, w = threadIdx.y;
    const int bc = b < nb ? b : nb - 1;
    const uint32_t* p = partial + (size_t)y * nblocks * nb + bc;
    uint64_t s = 0;
    int i = w;
    for (; i + 3 * kHistRedSlices < nblocks; i += 4 * kHistRedSlices) {
        const uint32_t v0 = p[(size_t)i * nb], v1 = p[(size_t)(i + kHistRedSlices) * nb];
        const uint32_t v2 = p[(size_t)(i + 2 * kHistRedSlices) * nb], v3 = p[(size_t)(i + 3 * kHistRedSlices) * nb];
        s += (uint64_t)v0 + v1 + v2 + v3;
    }
    for (; i < nblocks; i += kHistRedSlices) s += p[(size_t)i * nb];
    part[w][threadIdx.x] = s;
    __syncthreads();
    if (w == 0 && b < nb) {
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < kHistRedSlices; ++j) t += part[j][threadIdx.x];
        counts[(size_t)y * nb + b] = (double)t;
    }
}

// Mean and sample standard deviation over nreal realisations of `count`
// doubles at byte stride zs: a fixed-order two-pass sum per item.
static __global__ void k_batch_stats(const double* x, int nreal, int count, size_t zs, double* mean, double* sdev) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    auto at = [&](int r) { return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(x + i) + (size_t)r * zs); };
    double s = 0.0;
    for (int r = 0; r < nreal; ++r) s += at(r);
    const double m = s / nreal;
    double q = 0.0;
    for (int r = 0; r < nreal; ++r) q += (at(r) - m) * (at(r) - m);
    if (mean) mean[i] = m;
    if (sdev) sdev[i] = nreal > 1 ? sqrt(q / (nreal - 1)) : 0.0;
}

}  // namespace gridspt

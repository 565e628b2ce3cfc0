// Row FFT engine for gfx950: one row of N complex points is held by a team of
// P lanes of one 64-wide wavefront, E points per lane (E = 16 for N = 2^a,
// E = 12 for N = 3 * 2^a), and transformed by Stockham autosort passes (first
// radix E in registers, later passes exchanging through a per-row LDS
// buffer).  A row never spans two wavefronts, so the exchanges only need
// wavefront-scope synchronisation.
//
// Register layout ("canonical"): lane l of the team, register e holds point
// l + P*e of the row, both before and after a transform.  This is also the
// order in which a team reads a contiguous row from HBM (consecutive lanes,
// consecutive addresses), so loads feed the first pass directly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace gridspt {

// Spectral cube extents: Kc half-width, Kz = Kc + 1, Ky = Kx = 2Kc + 1.
struct CubeDims {
    int Kc, Kz, Ky;
};

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by +i
template <typename T>
__device__ __forceinline__ cpx<T> cmul_i(cpx<T> a) { return {-a.y, a.x}; }

// Force a value to be materialised in registers at this point: an empty asm
// with a read-write register operand (emits no instruction), which stops the
// compiler from sinking the computation of v past later code.
template <typename T>
__device__ __forceinline__ void keep_here(cpx<T>& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y));
}

// Compile-time loop.
template <typename F, int... Ks>
__host__ __device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Ks...>) {
    (f(std::integral_constant<int, Ks>{}), ...);
}
template <int Count, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, Count>{});
}

// cos of 2 pi m / 16, m = 0..15 (exact values of the eighth-circle constants
// cos(pi/8), cos(pi/4), cos(3pi/8)), and of 2 pi m / 12 (sqrt(3)/2 and 1/2).
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kCos12[12] = {1.0, 0.86602540378443864676, 0.5, 0.0, -0.5, -0.86602540378443864676,
                                          -1.0, -0.86602540378443864676, -0.5, 0.0, 0.5, 0.86602540378443864676};

// a * exp(DIR * 2 pi i K / R) for a compile-time root of unity of order
// R | 16 or R | 12, with the multiples of pi/2 done by swaps and sign flips.
template <int R, int K, int DIR, typename T>
__device__ __forceinline__ cpx<T> twiddle_const(cpx<T> a) {
    static_assert(16 % R == 0 || 12 % R == 0, "root order must divide 16 or 12");
    constexpr int C = (16 % R == 0) ? 16 : 12;  // circle the root lives on
    constexpr int k = ((K % R) + R) % R;
    constexpr int m = k * (C / R);  // position on the C-point circle
    if constexpr (m == 0) {
        return a;
    } else if constexpr (2 * m == C) {
        return {-a.x, -a.y};
    } else if constexpr (4 * m == C) {  // exp(DIR i pi/2) = DIR i
        if constexpr (DIR > 0) return {-a.y, a.x};
        else return {a.y, -a.x};
    } else if constexpr (4 * m == 3 * C) {  // exp(DIR i 3pi/2) = -DIR i
        if constexpr (DIR > 0) return {a.y, -a.x};
        else return {-a.y, a.x};
    } else {
        // sin(2 pi m / C) = cos(2 pi (m - C/4) / C)
        constexpr double c = C == 16 ? kCos16[m] : kCos12[m];
        constexpr double s0 = C == 16 ? kCos16[(m + 12) % 16] : kCos12[(m + 9) % 12];
        constexpr double s = (DIR > 0 ? 1.0 : -1.0) * s0;
        const T cc = (T)c, ss = (T)s;
        return {a.x * cc - a.y * ss, a.x * ss + a.y * cc};
    }
}

// In-place DFT of R points in natural order: X[k] = sum_j x[j] exp(DIR 2 pi i jk/R),
// for R a power of two (radix-2 decimation in time), R = 3, or R = 12
// (four-point DFTs of the three residue classes j mod 3, twiddles w_12^(j2 k1),
// then three-point DFTs); all twiddles are compile-time constants.
template <int R, int DIR, typename T>
struct Dft {
    static __device__ __forceinline__ void run(cpx<T>* x) {
        static_assert((R & (R - 1)) == 0, "power-of-two radix expected");
        cpx<T> ev[R / 2], od[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            ev[i] = x[2 * i];
            od[i] = x[2 * i + 1];
        }
        Dft<R / 2, DIR, T>::run(ev);
        Dft<R / 2, DIR, T>::run(od);
        static_for<R / 2>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            const cpx<T> t = twiddle_const<R, k, DIR>(od[k]);
            x[k] = cadd(ev[k], t);
            x[k + R / 2] = csub(ev[k], t);
        });
    }
};
template <int DIR, typename T>
struct Dft<1, DIR, T> {
    static __device__ __forceinline__ void run(cpx<T>*) {}
};
template <int DIR, typename T>
struct Dft<3, DIR, T> {
    // w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2
    static __device__ __forceinline__ void run(cpx<T>* x) {
        const cpx<T> s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
        const cpx<T> t = {x[0].x - (T)0.5 * s.x, x[0].y - (T)0.5 * s.y};
        const T h = (T)(DIR > 0 ? 0.86602540378443864676 : -0.86602540378443864676);
        const cpx<T> r = {-h * d.y, h * d.x};  // DIR i sqrt(3)/2 (x1 - x2)
        x[0] = cadd(x[0], s);
        x[1] = cadd(t, r);
        x[2] = csub(t, r);
    }
};
template <int DIR, typename T>
struct Dft<12, DIR, T> {
    static __device__ __forceinline__ void run(cpx<T>* x) {
        cpx<T> y[3][4];
#pragma unroll
        for (int j2 = 0; j2 < 3; ++j2) {
#pragma unroll
            for (int j1 = 0; j1 < 4; ++j1) y[j2][j1] = x[3 * j1 + j2];
            Dft<4, DIR, T>::run(y[j2]);
        }
        static_for<4>([&](auto kc) {
            constexpr int k1 = decltype(kc)::value;
            cpx<T> z[3] = {y[0][k1], twiddle_const<12, k1, DIR>(y[1][k1]), twiddle_const<12, 2 * k1, DIR>(y[2][k1])};
            Dft<3, DIR, T>::run(z);
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) x[k1 + 4 * k2] = z[k2];
        });
    }
};

// Wavefront-scope barrier: orders LDS traffic of all lanes of this wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS row buffer: element `pos` of a row lives at pad(pos); one extra slot
// every 16 breaks the power-of-two strides of the Stockham exchanges.
__host__ __device__ constexpr int lds_pad(int pos) { return pos + (pos >> 4); }
__host__ __device__ constexpr int lds_row_elems(int n) { return n + (n >> 4) + 1; }

// Radix plan of an N-point row.  A row is held by P lanes with E points each
// (E = 16 when N is a power of two, E = 12 when N = 3 * 2^a), so P = N / E is
// a power of two <= 64 and a team never straddles a wavefront.  Pass 0 is a
// radix-E DFT in registers; passes q = 1..NP have radices R_q dividing E
// (at most 16, or at most 4 when E = 12 or SPLIT is set) and exchange through
// LDS.  Pass q has Stockham stride S_q = E R_1 ... R_(q-1).
template <int N_, int SPLIT = 0>
struct Plan {
    static constexpr int N = N_;
    static constexpr int E = (N % 3 == 0) ? 12 : 16;
    static constexpr int P = N / E;
    static constexpr int CAP = (E == 12 || SPLIT != 0) ? 4 : 16;
    static constexpr int take(int rem) { return rem <= 1 ? 1 : (rem >= CAP ? CAP : rem); }
    static constexpr int R1 = take(P);
    static constexpr int R2 = take(P / R1);
    static constexpr int R3 = take(P / (R1 * R2));
    static constexpr int NP = (R1 > 1) + (R2 > 1) + (R3 > 1);
    static constexpr int radix(int q) { return q == 0 ? E : (q == 1 ? R1 : (q == 2 ? R2 : R3)); }
    static constexpr int stride(int q) { return q == 0 ? 1 : (q == 1 ? E : (q == 2 ? E * R1 : E * R1 * R2)); }
    // per-pass twiddle tables [j - 1][k], j < R_q, k < S_q, back to back
    static constexpr int tw_off(int q) {
        int o = 0;
        for (int i = 1; i < q; ++i) o += (radix(i) - 1) * stride(i);
        return o;
    }
    static constexpr int TW_SIZE = tw_off(NP + 1);
    static constexpr int TW_ALLOC = TW_SIZE > 0 ? TW_SIZE : 1;
    static_assert(E * P == N && P >= 1 && P <= 64 && (P & (P - 1)) == 0, "N must be 2^a (16..1024) or 3 2^a (12..768)");
    static_assert(R1 * R2 * R3 == P, "radix plan does not cover N");
    static_assert(E % R1 == 0 && E % R2 == 0 && E % R3 == 0, "later radices must divide E");
};

// Twiddles of the passes after the first: pass q multiplies input j of
// butterfly b by w_{S R}^{j k}, k = b mod S, with w_M = exp(-2 pi i / M).
//   LDS form: the per-pass tables of Plan, so the lanes of a wavefront
//     (consecutive k) read consecutive words.
//   global form: the full table w_N^m, m < N, read through the cache.
template <typename T, typename PL, bool LDS>
struct Twiddles {
    const cpx<T>* t;
    template <int Q>
    __device__ __forceinline__ cpx<T> get(int j, int k) const {
        constexpr int R = PL::radix(Q), S = PL::stride(Q);
        if constexpr (LDS) {
            return t[PL::tw_off(Q) + (j - 1) * S + k];
        } else {
            return t[j * k * (PL::N / (S * R))];
        }
    }
};

// Only FP32 may keep the per-pass tables in LDS: FP64 tables would cost a
// block per CU of LDS, so FP64 always reads the global table.  Each pass
// kernel further decides whether its own LDS traffic leaves room for them.
template <typename T>
constexpr bool kLdsTwiddles = sizeof(T) == 4;

// Fill the LDS tables from the global full table w_N^m; the caller
// synchronises the block before the first transform.
template <typename PL, typename T>
__device__ __forceinline__ void load_twiddles(cpx<T>* lds_tw, const cpx<T>* __restrict__ tw) {
    for (int i = threadIdx.x; i < PL::TW_SIZE; i += blockDim.x) {
        int q = 1;
        if (PL::NP >= 2 && i >= PL::tw_off(2)) q = 2;
        if (PL::NP >= 3 && i >= PL::tw_off(3)) q = 3;
        const int S = PL::stride(q), R = PL::radix(q), o = i - PL::tw_off(q);
        const int j = o / S + 1, k = o % S;
        lds_tw[i] = tw[j * k * (PL::N / (S * R))];
    }
}

// Row positions in the Stockham schedule, lane l, register i of the pass:
//   in_pos<Q>:  inputs of pass Q (butterfly b = l + P (i / R) reads b + (i mod R) N / R)
//   out_pos<Q>: outputs of pass Q (to (b - k) R + k + (i mod R) S, k = b mod S)
template <typename PL, int Q>
__device__ __forceinline__ int in_pos(int l, int i) {
    constexpr int R = PL::radix(Q);
    return l + PL::P * (i / R) + (i % R) * (PL::N / R);
}
template <typename PL, int Q>
__device__ __forceinline__ int out_pos(int l, int i) {
    constexpr int R = PL::radix(Q), S = PL::stride(Q);
    const int b = l + PL::P * (i / R), k = b % S;
    return (b - k) * R + k + (i % R) * S;
}

// Pass Q >= 1 on values gathered into y (y[t R + j] = input j of butterfly t).
template <typename PL, int Q, int DIR, typename T, bool LT>
__device__ __forceinline__ void stockham_compute(cpx<T> (&y)[PL::E], Twiddles<T, PL, LT> tw, int l) {
    constexpr int R = PL::radix(Q), S = PL::stride(Q), NB = PL::E / R;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int k = (l + PL::P * t) % S;
#pragma unroll
        for (int j = 1; j < R; ++j) {
            cpx<T> w = tw.template get<Q>(j, k);
            if (DIR > 0) w.y = -w.y;
            y[t * R + j] = cmul(y[t * R + j], w);
        }
        Dft<R, DIR, T>::run(&y[t * R]);
    }
}

// After the last pass: butterfly t output j is point l + P (t + j NB), so the
// canonical register order is a compile-time permutation.
template <typename PL, typename T>
__device__ __forceinline__ void to_canonical(const cpx<T> (&y)[PL::E], cpx<T> (&x)[PL::E]) {
    constexpr int R = PL::radix(PL::NP), NB = PL::E / R;
#pragma unroll
    for (int t = 0; t < NB; ++t)
#pragma unroll
        for (int j = 0; j < R; ++j) x[t + j * NB] = y[t * R + j];
}

// Transform one row held in canonical registers, in place (unnormalised).
// `row` is this row's LDS buffer (lds_row_elems(N) complex elements), `tw`
// the twiddle source (see Twiddles), and l the lane in the team.
template <typename PL, int DIR, typename T, bool LT>
__device__ __forceinline__ void fft_row(cpx<T> (&x)[PL::E], cpx<T>* row, Twiddles<T, PL, LT> tw, int l) {
    constexpr int E = PL::E;
    Dft<E, DIR, T>::run(x);  // pass 0: butterfly b = l over points l + P j, no twiddles
    cpx<T> y[E];
    static_for<PL::NP>([&](auto qc) {
        constexpr int Q = decltype(qc)::value + 1;
        // outputs of pass Q - 1 out to the row, inputs of pass Q back
#pragma unroll
        for (int i = 0; i < E; ++i) row[lds_pad(out_pos<PL, Q - 1>(l, i))] = (Q == 1) ? x[i] : y[i];
        wave_sync();
#pragma unroll
        for (int i = 0; i < E; ++i) y[i] = row[lds_pad(in_pos<PL, Q>(l, i))];
        wave_sync();  // every lane has read before the row is written again
        stockham_compute<PL, Q, DIR, T, LT>(y, tw, l);
    });
    if constexpr (PL::NP > 0) to_canonical<PL, T>(y, x);
}

// ---------------------------------------------------------------------------
// Split-exchange variant: the same passes, but every exchange moves the real
// parts and then the imaginary parts through a real-valued row buffer
// (lds_row_elems(N) elements of T), halving the LDS a row needs.
// ---------------------------------------------------------------------------

// Move values from register array `a` (a[i] at row position pa(i)) to
// register array `b` (b[i] from row position pb(i)), two rounds through `row`.
template <int NA, int NB, typename T, typename FA, typename FB>
__device__ __forceinline__ void exchange_split(const cpx<T> (&a)[NA], cpx<T> (&b)[NB], T* row, FA pa, FB pb) {
#pragma unroll
    for (int i = 0; i < NA; ++i) row[lds_pad(pa(i))] = a[i].x;
    wave_sync();
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i].x = row[lds_pad(pb(i))];
    wave_sync();
#pragma unroll
    for (int i = 0; i < NA; ++i) row[lds_pad(pa(i))] = a[i].y;
    wave_sync();
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i].y = row[lds_pad(pb(i))];
    wave_sync();
}

template <typename PL, int DIR, typename T, bool LT>
__device__ __forceinline__ void fft_row_split(cpx<T> (&x)[PL::E], T* row, Twiddles<T, PL, LT> tw, int l) {
    constexpr int E = PL::E;
    Dft<E, DIR, T>::run(x);
    cpx<T> y[E];
    static_for<PL::NP>([&](auto qc) {
        constexpr int Q = decltype(qc)::value + 1;
        if constexpr (Q == 1) {
            exchange_split<E, E, T>(x, y, row, [&](int i) { return out_pos<PL, 0>(l, i); },
                                    [&](int i) { return in_pos<PL, 1>(l, i); });
        } else {
            cpx<T> z[E];
#pragma unroll
            for (int i = 0; i < E; ++i) z[i] = y[i];
            exchange_split<E, E, T>(z, y, row, [&](int i) { return out_pos<PL, Q - 1>(l, i); },
                                    [&](int i) { return in_pos<PL, Q>(l, i); });
        }
        stockham_compute<PL, Q, DIR, T, LT>(y, tw, l);
    });
    if constexpr (PL::NP > 0) to_canonical<PL, T>(y, x);
}

// Realisation batching: a launch with gridDim.z = B processes B realisations
// whose buffers all sit at a fixed byte stride zs from realisation 0's (the
// twiddle table is shared).  zptr moves a pointer to realisation blockIdx.z.
template <typename P>
__device__ __forceinline__ P* zptr(P* p, size_t zs) {
    using B = std::conditional_t<std::is_const_v<P>, const char, char>;
    return p ? reinterpret_cast<P*>(reinterpret_cast<B*>(p) + (size_t)blockIdx.z * zs) : p;
}

// Block-index remap so that consecutive logical blocks (which write adjacent
// pieces of the same cache lines) run on the same XCD: the hardware deals
// blocks round-robin over 8 XCDs, so XCD x runs the physical blocks x, x + 8,
// ...; it gets the contiguous logical range starting at x q + min(x, r)
// (q = total / 8, r = total % 8; the first r XCDs take q + 1 blocks).  A
// bijection on [0, total) for any total = gridDim.x.
__device__ __forceinline__ uint32_t xcd_block(uint32_t phys, uint32_t total) {
    const uint32_t x = phys % 8u, k = phys / 8u, q = total / 8u, r = total % 8u;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace gridspt

// Row FFT engine for gfx950: one row of N complex points is held by a team of
// P = N/16 lanes of one 64-wide wavefront, 16 points per lane, and transformed
// by Stockham autosort passes (first radix 16 in registers, later passes
// exchanging through a per-row LDS buffer).  Rows of N <= 1024 fit in one
// wavefront, so the exchanges only need wavefront-scope synchronisation.
//
// Register layout ("canonical"): lane l of the team, register e holds point
// l + P*e of the row, both before and after a transform.  This is also the
// order in which a team reads a contiguous row from HBM (consecutive lanes,
// consecutive addresses), so loads feed the first radix-16 pass directly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
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
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Ks...>) {
    (f(std::integral_constant<int, Ks>{}), ...);
}
template <int Count, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, Count>{});
}

// cos and sin of 2 pi m / 16, m = 0..15 (exact values of the eighth-circle
// constants cos(pi/8), cos(pi/4), cos(3pi/8)).
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};

// a * exp(DIR * 2 pi i K / R) for a compile-time root of unity of order R | 16,
// with the trivial multiples of pi/2 done by swaps and sign flips.
template <int R, int K, int DIR, typename T>
__device__ __forceinline__ cpx<T> twiddle_const(cpx<T> a) {
    constexpr int k = ((K % R) + R) % R;
    constexpr int m = k * (16 / R);  // position on the 16-point circle
    if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 8) {
        return {-a.x, -a.y};
    } else if constexpr (m == 4) {  // exp(DIR i pi/2) = DIR i
        if constexpr (DIR > 0) return {-a.y, a.x};
        else return {a.y, -a.x};
    } else if constexpr (m == 12) {  // exp(DIR i 3pi/2) = -DIR i
        if constexpr (DIR > 0) return {a.y, -a.x};
        else return {-a.y, a.x};
    } else {
        constexpr double c = kCos16[m];
        constexpr double s = (DIR > 0 ? 1.0 : -1.0) * kCos16[(m + 12) % 16];  // sin = cos(. - pi/2)
        const T cc = (T)c, ss = (T)s;
        return {a.x * cc - a.y * ss, a.x * ss + a.y * cc};
    }
}

// In-place DFT of R points in natural order: X[k] = sum_j x[j] exp(DIR 2 pi i jk/R).
// Radix-2 decimation in time, all twiddles compile-time constants.
template <int R, int DIR, typename T>
struct Dft {
    static __device__ __forceinline__ void run(cpx<T>* x) {
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

// Radix plan: the first pass is radix 16; the remaining factor of N is split
// into at most two more passes of radix <= 16.
template <int N>
struct Plan {
    static constexpr int P = N / 16;  // lanes per row
    static constexpr int R2 = (N <= 16) ? 1 : (N / 16 >= 16 ? 16 : N / 16);
    static constexpr int R3 = (N <= 256) ? 1 : N / 256;
    static_assert(N >= 16 && N <= 1024 && (N & (N - 1)) == 0, "N must be a power of two in [16, 1024]");
};

// Twiddles of the Stockham passes after the first: pass (R, p) multiplies
// input j of butterfly b by w_{pR}^{j k}, k = b mod p, with w_M = exp(-2 pi i / M).
//   LDS form (FP32): one table per pass laid out [j - 1][k], so the lanes of a
//     wavefront (consecutive k) read consecutive words; about N entries.
//   global form (FP64): the full table w_N^m, m < N, read through the cache.
template <int N>
struct TwLayout {
    static constexpr int R2 = Plan<N>::R2, R3 = Plan<N>::R3;
    static constexpr int PASS3 = R2 > 1 ? (R2 - 1) * 16 : 0;  // start of the third pass's table
    static constexpr int SIZE = PASS3 + (R3 > 1 ? (R3 - 1) * 16 * R2 : 0);
    static constexpr int ALLOC = SIZE > 0 ? SIZE : 1;
};

template <typename T, int N, bool LDS>
struct Twiddles {
    const cpx<T>* t;
    template <int R, int PSTRIDE>
    __device__ __forceinline__ cpx<T> get(int j, int k) const {
        if constexpr (LDS) {
            constexpr int base = PSTRIDE == 16 ? 0 : TwLayout<N>::PASS3;
            return t[base + (j - 1) * PSTRIDE + k];
        } else {
            return t[j * k * (N / (PSTRIDE * R))];
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
template <int N, typename T>
__device__ __forceinline__ void load_twiddles(cpx<T>* lds_tw, const cpx<T>* __restrict__ tw) {
    using TL = TwLayout<N>;
    {
        for (int i = threadIdx.x; i < TL::SIZE; i += blockDim.x) {
            int m;
            if (i < TL::PASS3) {
                const int j = i / 16 + 1, k = i % 16;             // pass 2: p = 16, R = R2
                m = j * k * (N / (16 * TL::R2));
            } else {
                const int q = i - TL::PASS3, j = q / (16 * TL::R2) + 1, k = q % (16 * TL::R2);
                m = j * k * (N / (16 * TL::R2 * TL::R3));      // pass 3: p = 16 R2, R = R3
            }
            lds_tw[i] = tw[m];
        }
    }
}

// Stockham pass of radix R over a row held in LDS (not the first pass).
// Lane l handles butterflies b = l + P t, t < 16/R; butterfly b reads points
// b + j N/R, twiddles input j by w_{pR}^{j (b mod p)}, and writes its outputs
// to (b - k) R + k + j p, or, on the last pass, keeps them in registers in
// canonical order (register t + j 16/R holds point l + P (t + j 16/R)).
template <int N, int R, int PSTRIDE, bool LAST, int DIR, typename T, bool LT>
__device__ __forceinline__ void stockham_pass(cpx<T> (&x)[16], cpx<T>* row, Twiddles<T, N, LT> tw, int l) {
    constexpr int P = N / 16;
    constexpr int NB = 16 / R;
    cpx<T> y[16];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int b = l + P * t;
#pragma unroll
        for (int j = 0; j < R; ++j) y[t * R + j] = row[lds_pad(b + j * (N / R))];
    }
    wave_sync();  // every lane has read before anyone overwrites
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int b = l + P * t;
        const int k = b & (PSTRIDE - 1);
        // w_{pR}^{jk} = w_N^{jk N/(pR)} from the forward table; conjugate for DIR > 0
#pragma unroll
        for (int j = 1; j < R; ++j) {
            cpx<T> w = tw.template get<R, PSTRIDE>(j, k);
            if (DIR > 0) w.y = -w.y;
            y[t * R + j] = cmul(y[t * R + j], w);
        }
        Dft<R, DIR, T>::run(&y[t * R]);
    }
    if constexpr (LAST) {
#pragma unroll
        for (int t = 0; t < NB; ++t)
#pragma unroll
            for (int j = 0; j < R; ++j) x[t + j * NB] = y[t * R + j];
    } else {
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int b = l + P * t;
            const int k = b & (PSTRIDE - 1);
#pragma unroll
            for (int j = 0; j < R; ++j) row[lds_pad((b - k) * R + k + j * PSTRIDE)] = y[t * R + j];
        }
        wave_sync();
    }
}

// Transform one row held in canonical registers, in place (unnormalised).
// `row` is this row's LDS buffer (lds_row_elems(N) elements), `tw` the
// twiddle source (see Twiddles), and l the lane in the team.
template <int N, int DIR, typename T, bool LT>
__device__ __forceinline__ void fft_row(cpx<T> (&x)[16], cpx<T>* row, Twiddles<T, N, LT> tw, int l) {
    using PL = Plan<N>;
    Dft<16, DIR, T>::run(x);  // pass 1: butterfly b = l over points l + P j, no twiddles
    if constexpr (N == 16) {
        return;
    } else {
        // pass-1 outputs go to points 16 l + j
#pragma unroll
        for (int j = 0; j < 16; ++j) row[lds_pad(16 * l + j)] = x[j];
        wave_sync();
        if constexpr (PL::R3 == 1) {
            stockham_pass<N, PL::R2, 16, true, DIR, T, LT>(x, row, tw, l);
        } else {
            stockham_pass<N, PL::R2, 16, false, DIR, T, LT>(x, row, tw, l);
            stockham_pass<N, PL::R3, 16 * PL::R2, true, DIR, T, LT>(x, row, tw, l);
        }
    }
}

// ---------------------------------------------------------------------------
// Split-exchange variant: the same Stockham passes, but every exchange moves
// the real parts and then the imaginary parts through a real-valued row
// buffer (lds_row_elems(N) elements of T), halving the LDS a row needs.
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

// Stockham pass of radix R on values already gathered into y (butterfly
// t of this lane holds inputs y[t R + j] = points b + j N/R, b = l + P t).
template <int N, int R, int PSTRIDE, int DIR, typename T, bool LT>
__device__ __forceinline__ void stockham_compute(cpx<T> (&y)[16], Twiddles<T, N, LT> tw, int l) {
    constexpr int P = N / 16;
    constexpr int NB = 16 / R;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int k = (l + P * t) & (PSTRIDE - 1);
#pragma unroll
        for (int j = 1; j < R; ++j) {
            cpx<T> w = tw.template get<R, PSTRIDE>(j, k);
            if (DIR > 0) w.y = -w.y;
            y[t * R + j] = cmul(y[t * R + j], w);
        }
        Dft<R, DIR, T>::run(&y[t * R]);
    }
}

template <int N, int DIR, typename T, bool LT>
__device__ __forceinline__ void fft_row_split(cpx<T> (&x)[16], T* row, Twiddles<T, N, LT> tw, int l) {
    using PL = Plan<N>;
    constexpr int P = N / 16;
    Dft<16, DIR, T>::run(x);  // pass 1: outputs at points 16 l + j
    if constexpr (N > 16) {
        constexpr int R2 = PL::R2, NB2 = 16 / R2;
        cpx<T> y[16];
        exchange_split<16, 16, T>(x, y, row, [&](int j) { return 16 * l + j; },
                                  [&](int i) { return (l + P * (i / R2)) + (i % R2) * (N / R2); });
        stockham_compute<N, R2, 16, DIR, T, LT>(y, tw, l);
        if constexpr (PL::R3 == 1) {
#pragma unroll
            for (int t = 0; t < NB2; ++t)
#pragma unroll
                for (int j = 0; j < R2; ++j) x[t + j * NB2] = y[t * R2 + j];
        } else {
            constexpr int R3 = PL::R3, NB3 = 16 / R3, PS3 = 16 * R2;
            cpx<T> z[16];
            exchange_split<16, 16, T>(
                y, z, row,
                [&](int i) {
                    const int b = l + P * (i / R2), k = b & 15;
                    return (b - k) * R2 + k + (i % R2) * 16;
                },
                [&](int i) { return (l + P * (i / R3)) + (i % R3) * (N / R3); });
            stockham_compute<N, R3, PS3, DIR, T, LT>(z, tw, l);
#pragma unroll
            for (int t = 0; t < NB3; ++t)
#pragma unroll
                for (int j = 0; j < R3; ++j) x[t + j * NB3] = z[t * R3 + j];
        }
    }
}

// Block-index remap so that consecutive logical blocks (which write adjacent
// pieces of the same cache lines) run on the same XCD: the hardware deals
// blocks round-robin over 8 XCDs.
__device__ __forceinline__ uint32_t xcd_block(uint32_t phys, uint32_t total) {
    if (total % 8u != 0u) return phys;
    return (phys % 8u) * (total / 8u) + phys / 8u;
}

}  // namespace gridspt

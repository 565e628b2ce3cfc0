// Host runtime shared by every translation unit of libgridspt: the context,
// the kernel-launch wrapper with optional event timing, argument validation,
// and the workspace layout of the transform pipeline.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/gridspt.h"
#include "estimators.hpp"
#include "passes.hpp"

namespace gridspt {

// ---------------------------------------------------------------------------
// kernel kinds (profiling groups and autotuner slots)
// ---------------------------------------------------------------------------
enum Kind {
    KD_TWIDDLE,
    KD_ZFWD_FIELD,
    KD_ZFWD_NOISE,
    KD_ZFWD_PRODUCTS,  // the product pass of an order (k_zchain: z inverse of order n - 1 + P1)
    KD_YFWD,
    KD_XFUSED_LINEAR,
    KD_XFUSED_ORDER1,
    KD_XFUSED_ORDER,
    KD_XFUSED_FORWARD,
    KD_XSHELL,
    KD_YINV,
    KD_ZINV,
    KD_POWER,
    KD_POWER_FINAL,
    KD_TRIPLE,
    KD_TRIPLE_FINAL,
    KD_BISP_FINAL,
    KD_SUM_ORDERS,
    KD_COPY,
    KD_BATCH_STATS,
    KD_ZFWD_ADJ,
    KD_XREGEN,
    KD_XFUSED_ADJ,
    KD_XFUSED_ADJ1,
    KD_ADJ_PRODUCTS,
    KD_PFORM_PRODUCTS,
    KD_ZFWD_PAIR,
    KD_XFUSED_PFORM,
    KD_XDERIVED,
    KD_XSMOOTH,
    KD_MOMENTS,
    KD_HIST,
    KD_COUNT
};

inline const char* const kKindNames[KD_COUNT] = {
    "twiddles",      "zfwd_field",     "zfwd_noise",   "zfwd_products", "yfwd",        "xfused_linear",
    "xfused_order1", "xfused_order",   "xfused_forward", "xshell",      "yinv",        "zinv",
    "power_partial", "power_final",    "triple_partial", "triple_final", "bisp_final", "sum_orders",
    "copy",          "batch_stats",    "zfwd_adjoint", "xregen",        "xfused_adj",  "xfused_adj1",
    "adj_products",  "pform_products", "zfwd_pair",    "xfused_pform",  "xderived",    "xsmooth",
    "moments",       "histogram"};

// Launch variant of each pass kind (see Rows): 0 is the default shape.
struct Tuning {
    int v[KD_COUNT] = {};
};

// Variants compiled per (precision, size), for the autotuner: FP32 grids of
// 64..1024 (power of two) get rows-per-block halvings and the radix-4 split
// (variants 0, 1, 4, 5), FP32 grids of 96..384 (3 * 2^a) halvings (0, 1, 2),
// everything else only variant 0.
constexpr bool tuned_pow2(bool f32, int n) {
    return f32 && (n == 64 || n == 128 || n == 256 || n == 512 || n == 1024);
}
constexpr bool tuned_three(bool f32, int n) { return f32 && (n == 96 || n == 192 || n == 384); }
inline int variant_list(int dtype, int n, int* out) {
    const bool f32 = dtype == GRIDSPT_F32;
    if (tuned_pow2(f32, n)) {
        out[0] = 0, out[1] = 1, out[2] = 4, out[3] = 5;
        return 4;
    }
    if (tuned_three(f32, n)) {
        out[0] = 0, out[1] = 1, out[2] = 2;
        return 3;
    }
    out[0] = 0;
    return 1;
}

}  // namespace gridspt

struct gridspt_ctx {
    struct Record {
        int kind;
        int order;  // order of the recursion the launch belongs to, 0 for none
        hipEvent_t start, stop;
        double bytes;
    };
    struct Tuned {
        int n, dtype;
        gridspt::Tuning tu;
        double ms[gridspt::KD_COUNT];
    };
    hipStream_t stream = nullptr;
    bool profile = false;
    int order_tag = 0;  // stamped on every record (set by the orders' pass sequences)
    std::vector<Record> recs;
    // per order 0..kMaxOrderTag, from the last gridspt_profile_read
    static constexpr int kMaxOrderTag = 8;
    double order_ms[kMaxOrderTag + 1] = {}, order_bytes[kMaxOrderTag + 1] = {};
    std::vector<hipEvent_t> pool;
    std::vector<Tuned> tuned;  // autotuner choices per grid (size, precision)
    const gridspt::Tuning& tuning(const gridspt_grid* g) const {
        static const gridspt::Tuning none{};
        for (const auto& t : tuned)
            if (t.n == g->n && t.dtype == g->dtype) return t.tu;
        return none;
    }
};

namespace gridspt {

inline hipEvent_t take_event(gridspt_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Enqueue one kernel on the context's stream; with profiling on, bracket it
// with events.  `bytes` is the launch's algorithmic HBM traffic.
template <typename Kern, typename... Args>
int launch(gridspt_ctx* c, int kind, double bytes, dim3 grid, dim3 block, size_t shmem, Kern kern, Args... args) {
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return GRIDSPT_OK;
    gridspt_ctx::Record r{kind, c->order_tag, nullptr, nullptr, bytes};
    if (c->profile) {
        r.start = take_event(c);
        r.stop = take_event(c);
        if (!r.start || !r.stop) return GRIDSPT_EHIP;
        if (hipEventRecord(r.start, c->stream) != hipSuccess) return GRIDSPT_EHIP;
    }
    hipLaunchKernelGGL(kern, grid, block, shmem, c->stream, args...);
    if (hipGetLastError() != hipSuccess) return GRIDSPT_EHIP;
    if (c->profile) {
        if (hipEventRecord(r.stop, c->stream) != hipSuccess) return GRIDSPT_EHIP;
        c->recs.push_back(r);
    }
    return GRIDSPT_OK;
}

// Stamps the launches enqueued while it lives with order n (per-order timing).
struct OrderTag {
    gridspt_ctx* c;
    int saved;
    OrderTag(gridspt_ctx* ctx, int n) : c(ctx), saved(ctx->order_tag) { c->order_tag = n; }
    void set(int n) { c->order_tag = n; }
    ~OrderTag() { c->order_tag = saved; }
};

#define GRIDSPT_CHECK(x)                   \
    do {                                   \
        const int rc_ = (x);               \
        if (rc_ != GRIDSPT_OK) return rc_; \
    } while (0)

// ---------------------------------------------------------------------------
// validation and sizes
// ---------------------------------------------------------------------------

constexpr int64_t kAlign = 256;

// grid sizes with compiled pipelines: 2^a (16..1024) and 3 * 2^a (48..768)
inline bool n_supported(int n) {
    switch (n) {
        case 16: case 32: case 64: case 128: case 256: case 512: case 1024:
        case 48: case 96: case 192: case 384: case 768: return true;
        default: return false;
    }
}

inline int64_t isqrt64(int64_t v) {
    if (v < 0) return -1;
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

inline int check_grid(const gridspt_grid* g) {
    if (!g) return GRIDSPT_EINVAL;
    if (g->flags & ~(uint32_t)GRIDSPT_CHECK_FINITE) return GRIDSPT_EINVAL;
    if (g->dtype != GRIDSPT_F32 && g->dtype != GRIDSPT_F64) return GRIDSPT_EINVAL;
    if (!(g->box > 0.0) || !std::isfinite(g->box)) return GRIDSPT_EINVAL;
    if (g->n < 2 || (g->n & 1)) return GRIDSPT_EINVAL;
    if (g->kc < 1 || 2 * (int64_t)g->kc >= g->n) return GRIDSPT_EINVAL;
    if (!n_supported(g->n)) return GRIDSPT_EUNSUPPORTED;
    return GRIDSPT_OK;
}

inline int check_mask(const gridspt_grid* g, int64_t n2max) {
    if (n2max < 1) return GRIDSPT_EINVAL;
    const int64_t h = g->n / 2;
    if (n2max >= h * h) return GRIDSPT_EINVAL;  // the cut must lie below Nyquist
    if (isqrt64(n2max) > g->kc) return GRIDSPT_EINVAL;
    return GRIDSPT_OK;
}

inline int check_ptr(const void* p) {
    if (!p) return GRIDSPT_EALIGN;
    if (reinterpret_cast<uintptr_t>(p) % kAlign) return GRIDSPT_EALIGN;
    return GRIDSPT_OK;
}

inline int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Dims {
    int64_t N, Kc, Kz, Ky;
    int64_t real_bytes, cpx_bytes;  // element sizes
    int64_t ncell() const { return N * N * N; }
    int64_t s1() const { return Kz * N * N; }  // complex elements per field
    int64_t s2() const { return Kz * Ky * N; }
    // S2 rows (kz, x) start every s2_row() complex elements: Ky rounded up to a multiple of
    // 16, so every row starts on a 128-byte boundary (256 in FP64) and the x pass's short
    // runs of consecutive ky' cross no more cache lines than they must
    int64_t s2_row() const { return (Ky + 15) / 16 * 16; }
    int64_t s2_alloc() const { return Kz * s2_row() * N; }
    int64_t s3() const { return Kz * N * Ky; }
    int64_t s4() const { return N * N * Kz; }
    int64_t cube() const { return Kz * Ky * Ky; }
};

inline Dims dims_of(const gridspt_grid* g) {
    Dims d;
    d.N = g->n;
    d.Kc = g->kc;
    d.Kz = g->kc + 1;
    d.Ky = 2 * (int64_t)g->kc + 1;
    d.real_bytes = g->dtype == GRIDSPT_F64 ? 8 : 4;
    d.cpx_bytes = 2 * d.real_bytes;
    return d;
}

// Workspace of the transform pipeline: the input check's flag word (256 bytes)
// | twiddles | radial amplitude table ((Kc + 1)^2 doubles) | buffer A (S1, S3)
// | buffer B (S2, S4) | u_m real fields for m <= nmax - 2 (the product pass of
// order nmax takes u_{nmax-1} from registers).  S1/S3 and S2/S4 are never live
// at once.
struct Layout {
    int64_t chk, tw, amp, a, b, u, end;
    int64_t a_field_s1, a_field_s3, b_field_s2, b_field_s4;  // field strides (elements)
};

inline Layout layout_of(const Dims& d, int nmax) {
    Layout L;
    L.chk = 0;
    L.tw = kAlign;
    L.amp = align_up(L.tw + d.N * d.cpx_bytes);
    L.a = align_up(L.amp + (d.Kc + 1) * (d.Kc + 1) * 8);
    const int64_t asz = std::max(4 * d.s1(), 5 * d.s3()) * d.cpx_bytes;
    L.b = align_up(L.a + asz);
    const int64_t bsz = std::max(4 * d.s2_alloc(), 5 * d.s4()) * d.cpx_bytes;
    L.u = align_up(L.b + bsz);
    const int nu = std::max(nmax - 2, 0) * 3;
    L.end = align_up(L.u + (int64_t)nu * d.ncell() * d.real_bytes);
    L.a_field_s1 = d.s1();
    L.a_field_s3 = d.s3();
    L.b_field_s2 = d.s2_alloc();
    L.b_field_s4 = d.s4();
    return L;
}

template <typename T>
struct tag_t {
    using type = T;
};

// Realisation batch of one pipeline call: nreal realisations whose buffers
// (workspace, inputs, outputs) sit at byte stride zs from the first.
struct Batch {
    int nreal = 1;
    size_t zs = 0;
};

// ---------------------------------------------------------------------------
// pass sequences, defined in pipeline.hpp and instantiated per grid size
// ---------------------------------------------------------------------------
// noise: a given white-noise field (N^3 real), or null to draw it (Philox)
template <typename T, int N>
int run_linear_field(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, const void* noise,
                     void* delta1, void* delta1_k, void* work, const Tuning& tu, Batch b);
template <typename T, int N>
int run_forward(gridspt_ctx* c, const gridspt_grid* g, int64_t n2max, const void* field, void* field_k, void* work,
                const Tuning& tu, Batch b);
// lp: draw delta_1 from this spectrum and seed (linear field and order 1 in
// one pass sequence; W1 = lp->n2max, delta1 unused), or null to read delta1
template <typename T, int N>
int run_orders(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int nmax, int64_t n2max1,
               int64_t n2max2, const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
               void* const* theta_k, void* work, const Tuning& tu, Batch b);
// bispectrum slots: shell-filtered C2R of cube fields (null: the indicator)
// into real fields out[i]; lo/hi the n^2 range of each slot
template <typename T, int N>
int run_shells(gridspt_ctx* c, const gridspt_grid* g, int nslots, const void* const* cubes, const int64_t* lo,
               const int64_t* hi, void* const* out, void* work, const Tuning& tu, Batch b);

// reverse mode of run_linear_field (given noise) + run_orders, see adjoint_layout
template <typename T, int N>
int run_adjoint(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int nmax, int64_t n2max2,
                const void* const* delta_k, const void* const* theta_k, const void* const* gdelta, void* gnoise,
                void* work, const Tuning& tu, Batch b);

// Gaussian-smoothed (cumulative) sums of up to five cube spectra into real fields
template <typename T, int N>
int run_smooth(gridspt_ctx* c, const gridspt_grid* g, int nfields, const void* const* fields_k, const double* coef,
               int cumulative, double radius, void* const* out, void* work, const Tuning& tu, Batch b);

// the printed (P-form) sources of Eq. 10 instead of the divergence form; same
// arguments as run_orders, workspace pform_layout
template <typename T, int N>
int run_orders_pform(gridspt_ctx* c, const gridspt_grid* g, int nmax, int64_t n2max1, int64_t n2max2,
                     const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
                     void* const* theta_k, void* work, const Tuning& tu, Batch b);

// Workspace of the P-form: the pipeline (no u fields) | 15 derived real fields
// per order < nmax | S_delta, S_theta | the current order's two spectra.
struct PFormLayout {
    int64_t fields, cubes, end;
};
inline PFormLayout pform_layout(const Dims& d, int nmax) {
    PFormLayout a;
    a.fields = layout_of(d, 1).end;
    a.cubes = align_up(a.fields + (15 * (int64_t)(nmax - 1) + 2) * d.ncell() * d.real_bytes);
    a.end = align_up(a.cubes + 2 * d.cube() * d.cpx_bytes);
    return a;
}

// Workspace of the reverse mode: the pipeline (no u fields) | delta_m, u_m
// (m < nmax, regenerated) | their gradient accumulators | g V, g W.
struct AdjLayout {
    int64_t fields, end;  // first real field, total bytes
    int64_t nfield;       // real fields
};
inline AdjLayout adjoint_layout(const Dims& d, int nmax) {
    AdjLayout a;
    a.fields = layout_of(d, 1).end;
    a.nfield = 8 * (int64_t)(nmax - 1) + 4;
    a.end = align_up(a.fields + a.nfield * d.ncell() * d.real_bytes);
    return a;
}

// Call f(tag_t<T>, integral_constant<int, N>) for the grid's precision and size.
template <typename F>
int dispatch(const gridspt_grid* g, F&& f) {
    auto on_n = [&](auto tag) -> int {
        switch (g->n) {
#define GRIDSPT_CASE(n) \
    case n: return f(tag, std::integral_constant<int, n>{});
            GRIDSPT_CASE(16) GRIDSPT_CASE(32) GRIDSPT_CASE(64) GRIDSPT_CASE(128) GRIDSPT_CASE(256)
            GRIDSPT_CASE(512) GRIDSPT_CASE(1024) GRIDSPT_CASE(48) GRIDSPT_CASE(96) GRIDSPT_CASE(192)
            GRIDSPT_CASE(384) GRIDSPT_CASE(768)
#undef GRIDSPT_CASE
            default: return GRIDSPT_EUNSUPPORTED;
        }
    };
    if (g->dtype == GRIDSPT_F64) return on_n(tag_t<double>{});
    return on_n(tag_t<float>{});
}

}  // namespace gridspt

// libgridspt: C ABI (include/gridspt.h) over the gfx950 kernels in
// passes.hpp and estimators.hpp.  Host code validates arguments, lays out the
// caller's workspace, and enqueues the pass sequence of each entry point on
// the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/gridspt.h"
#include "estimators.hpp"
#include "passes.hpp"

using namespace gridspt;

// ---------------------------------------------------------------------------
// context and kernel timing
// ---------------------------------------------------------------------------

enum Kind {
    KD_TWIDDLE,
    KD_ZFWD_FIELD,
    KD_ZFWD_NOISE,
    KD_ZFWD_PRODUCTS,
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
    KD_COUNT
};

static const char* kKindNames[KD_COUNT] = {
    "twiddles",     "zfwd_field", "zfwd_noise",    "zfwd_products", "yfwd",         "xfused_linear",
    "xfused_order1", "xfused_order", "xfused_forward", "xshell",       "yinv",         "zinv",
    "power_partial", "power_final", "triple_partial", "triple_final", "bisp_final",   "sum_orders",
    "copy"};

struct Record {
    int kind;
    hipEvent_t start, stop;
    double bytes;
};

struct gridspt_ctx {
    hipStream_t stream = nullptr;
    bool profile = false;
    std::vector<Record> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

hipEvent_t take_event(gridspt_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Enqueue one kernel; with profiling on, bracket it with events.
template <typename Kern, typename... Args>
int launch(gridspt_ctx* c, int kind, double bytes, dim3 grid, dim3 block, size_t shmem, Kern kern, Args... args) {
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return GRIDSPT_OK;
    Record r{kind, nullptr, nullptr, bytes};
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

#define CHECK(x)                           \
    do {                                   \
        const int rc_ = (x);               \
        if (rc_ != GRIDSPT_OK) return rc_; \
    } while (0)

// ---------------------------------------------------------------------------
// validation and sizes
// ---------------------------------------------------------------------------

constexpr int64_t kAlign = 256;

bool pow2_supported(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

int64_t isqrt64(int64_t v) {
    if (v < 0) return -1;
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

int check_grid(const gridspt_grid* g) {
    if (!g) return GRIDSPT_EINVAL;
    if (g->dtype != GRIDSPT_F32 && g->dtype != GRIDSPT_F64) return GRIDSPT_EINVAL;
    if (!(g->box > 0.0) || !std::isfinite(g->box)) return GRIDSPT_EINVAL;
    if (g->n < 2 || (g->n & 1)) return GRIDSPT_EINVAL;
    if (g->kc < 1 || 2 * (int64_t)g->kc >= g->n) return GRIDSPT_EINVAL;
    if (!pow2_supported(g->n)) return GRIDSPT_EUNSUPPORTED;
    return GRIDSPT_OK;
}

int check_mask(const gridspt_grid* g, int64_t n2max) {
    if (n2max < 1) return GRIDSPT_EINVAL;
    const int64_t h = g->n / 2;
    if (n2max >= h * h) return GRIDSPT_EINVAL;  // the cut must lie below Nyquist
    if (isqrt64(n2max) > g->kc) return GRIDSPT_EINVAL;
    return GRIDSPT_OK;
}

int check_ptr(const void* p) {
    if (!p) return GRIDSPT_EALIGN;
    if (reinterpret_cast<uintptr_t>(p) % kAlign) return GRIDSPT_EALIGN;
    return GRIDSPT_OK;
}

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Dims {
    int64_t N, Kc, Kz, Ky;
    int64_t real_bytes, cpx_bytes;  // element sizes
    int64_t ncell() const { return N * N * N; }
    int64_t s1() const { return Kz * N * N; }  // complex elements per field
    int64_t s2() const { return Kz * Ky * N; }
    int64_t s3() const { return Kz * N * Ky; }
    int64_t s4() const { return N * N * Kz; }
    int64_t cube() const { return Kz * Ky * Ky; }
};

Dims dims_of(const gridspt_grid* g) {
    Dims d;
    d.N = g->n;
    d.Kc = g->kc;
    d.Kz = g->kc + 1;
    d.Ky = 2 * (int64_t)g->kc + 1;
    d.real_bytes = g->dtype == GRIDSPT_F64 ? 8 : 4;
    d.cpx_bytes = 2 * d.real_bytes;
    return d;
}

// Workspace of the transform pipeline: twiddles | buffer A (S1, S3) |
// buffer B (S2, S4) | u_m real fields.  S1/S3 and S2/S4 are never live at once.
struct Layout {
    int64_t tw, a, b, u, end;
    int64_t a_field_s1, a_field_s3, b_field_s2, b_field_s4;  // field strides (elements)
};

Layout layout_of(const Dims& d, int nmax) {
    Layout L;
    L.tw = 0;
    L.a = align_up(d.N * d.cpx_bytes);
    const int64_t asz = std::max(4 * d.s1(), 5 * d.s3()) * d.cpx_bytes;
    L.b = align_up(L.a + asz);
    const int64_t bsz = std::max(4 * d.s2(), 5 * d.s4()) * d.cpx_bytes;
    L.u = align_up(L.b + bsz);
    const int nu = std::max(nmax - 1, 0) * 3;
    L.end = align_up(L.u + (int64_t)nu * d.ncell() * d.real_bytes);
    L.a_field_s1 = d.s1();
    L.a_field_s3 = d.s3();
    L.b_field_s2 = d.s2();
    L.b_field_s4 = d.s4();
    return L;
}

template <typename T>
struct tag_t {
    using type = T;
};

template <typename F>
int dispatch(const gridspt_grid* g, F&& f) {
    auto on_n = [&](auto tag) -> int {
        using T = typename decltype(tag)::type;
        switch (g->n) {
            case 16: return f(tag, std::integral_constant<int, 16>{});
            case 32: return f(tag, std::integral_constant<int, 32>{});
            case 64: return f(tag, std::integral_constant<int, 64>{});
            case 128: return f(tag, std::integral_constant<int, 128>{});
            case 256: return f(tag, std::integral_constant<int, 256>{});
            case 512: return f(tag, std::integral_constant<int, 512>{});
            case 1024: return f(tag, std::integral_constant<int, 1024>{});
            default: return GRIDSPT_EUNSUPPORTED;
        }
        (void)sizeof(T);
    };
    if (g->dtype == GRIDSPT_F64) return on_n(tag_t<double>{});
    return on_n(tag_t<float>{});
}

// ---------------------------------------------------------------------------
// pass sequences
// ---------------------------------------------------------------------------

template <typename T, int N>
struct Pipe {
    using RW = Rows<T, N>;
    gridspt_ctx* c;
    Dims d;
    Layout L;
    char* ws;
    CubeDims cd;

    Pipe(gridspt_ctx* ctx, const gridspt_grid* g, void* work, int nmax) : c(ctx), d(dims_of(g)) {
        L = layout_of(d, nmax);
        ws = static_cast<char*>(work);
        cd = {(int)d.Kc, (int)d.Kz, (int)d.Ky};
    }
    cpx<T>* tw() const { return reinterpret_cast<cpx<T>*>(ws + L.tw); }
    cpx<T>* A() const { return reinterpret_cast<cpx<T>*>(ws + L.a); }
    cpx<T>* B() const { return reinterpret_cast<cpx<T>*>(ws + L.b); }
    T* U(int m, int j) const {  // u_m component j, m >= 1
        return reinterpret_cast<T*>(ws + L.u) + ((size_t)(m - 1) * 3 + j) * (size_t)d.ncell();
    }

    int twiddles() {
        return launch(c, KD_TWIDDLE, (double)N * d.cpx_bytes, dim3((N + 255) / 256), dim3(256), 0, k_twiddles<T>,
                      tw(), N);
    }

    // P1 from a real field (SRC 0) or from noise (SRC 1) -> S1 field 0 in A
    int zfwd_single(const T* f, bool noise, uint64_t seed, uint64_t stream) {
        ProductInputs<T> pin{};
        const double bytes = (noise ? 0.0 : (double)d.ncell() * d.real_bytes) + (double)d.s1() * d.cpx_bytes;
        const dim3 grid(N * (N / (2 * RW::RPB))), block(RW::THREADS);  // two rows per transform
        if (noise)
            return launch(c, KD_ZFWD_NOISE, bytes, grid, block, 0, k_zfwd<T, N, 1, 0>, f, pin, seed, stream, A(),
                          (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz);
        return launch(c, KD_ZFWD_FIELD, bytes, grid, block, 0, k_zfwd<T, N, 0, 0>, f, pin, seed, stream, A(),
                      (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz);
    }

    // P1 with the products of order n -> S1 fields 0..3 (V_x, V_y, V_z, W) in A
    int zfwd_products(int n, const ProductInputs<T>& pin) {
        const double bytes = 4.0 * (n - 1) * d.ncell() * d.real_bytes + 4.0 * d.s1() * d.cpx_bytes;
        const dim3 grid(N * (N / RW::RPB)), block(RW::THREADS);
        auto go = [&](auto kern) {
            return launch(c, KD_ZFWD_PRODUCTS, bytes, grid, block, 0, kern, (const T*)nullptr, pin, (uint64_t)0,
                          (uint64_t)0, A(), (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz);
        };
        switch (n) {
            case 2: return go(k_zfwd<T, N, 2, 2>);
            case 3: return go(k_zfwd<T, N, 2, 3>);
            case 4: return go(k_zfwd<T, N, 2, 4>);
            case 5: return go(k_zfwd<T, N, 2, 5>);
            default: return GRIDSPT_EINVAL;
        }
    }

    // P2: nf fields S1 (A) -> S2 (B)
    int yfwd(int nf) {
        const double bytes = (double)nf * (d.s1() + d.s2()) * d.cpx_bytes;
        return launch(c, KD_YFWD, bytes, dim3((unsigned)(d.Kz * (N / RW::RPB)), nf), dim3(RW::THREADS), 0,
                      k_yfwd<T, N>, (const cpx<T>*)A(), (size_t)L.a_field_s1, B(), (size_t)L.b_field_s2,
                      (const cpx<T>*)tw(), cd);
    }

    // P3: S2 (B) -> S3 (A), with the k-space step of `mode`
    int xfused(int mode, XArgs<T> a) {
        a.s2 = B();
        a.s2_field = (size_t)L.b_field_s2;
        a.s3 = A();
        a.s3_field = (size_t)L.a_field_s3;
        const int nin = mode == XM_ORDER ? 4 : 1;
        const int ncube = (a.cube_d ? 1 : 0) + (a.cube_t ? 1 : 0);
        const double bytes =
            ((double)nin * d.s2() + (double)a.nout * d.s3() + (double)ncube * d.cube()) * d.cpx_bytes;
        const dim3 grid((unsigned)(d.Kz * ((d.Ky + RW::RPB - 1) / RW::RPB))), block(RW::THREADS);
        const cpx<T>* t = tw();
        switch (mode) {
            case XM_ORDER: return launch(c, KD_XFUSED_ORDER, bytes, grid, block, 0, k_xfused<T, N, XM_ORDER>, a, t, cd);
            case XM_ORDER1:
                return launch(c, KD_XFUSED_ORDER1, bytes, grid, block, 0, k_xfused<T, N, XM_ORDER1>, a, t, cd);
            case XM_LINEAR:
                return launch(c, KD_XFUSED_LINEAR, bytes, grid, block, 0, k_xfused<T, N, XM_LINEAR>, a, t, cd);
            default:
                return launch(c, KD_XFUSED_FORWARD, bytes, grid, block, 0, k_xfused<T, N, XM_FORWARD>, a, t, cd);
        }
    }

    // P3 for shells: nslot cube fields -> S3 (A)
    int xshell(ShellSlots<T> s, int nslot) {
        s.s3 = A();
        s.s3_field = (size_t)L.a_field_s3;
        int ncube = 0;
        for (int i = 0; i < nslot; ++i) ncube += s.cube[i] ? 1 : 0;
        const double bytes = ((double)ncube * d.cube() + (double)nslot * d.s3()) * d.cpx_bytes;
        return launch(c, KD_XSHELL, bytes, dim3((unsigned)(d.Kz * ((d.Ky + RW::RPB - 1) / RW::RPB)), nslot),
                      dim3(RW::THREADS), 0, k_xshell<T, N>, s, (const cpx<T>*)tw(), cd);
    }

    // P4: nf fields S3 (A) -> S4 (B)
    int yinv(int nf) {
        const double bytes = (double)nf * (d.s3() + d.s4()) * d.cpx_bytes;
        return launch(c, KD_YINV, bytes, dim3((unsigned)(N * ((d.Kz + RW::RPB - 1) / RW::RPB)), nf),
                      dim3(RW::THREADS), 0, k_yinv<T, N>, (const cpx<T>*)A(), (size_t)L.a_field_s3, B(),
                      (size_t)L.b_field_s4, (const cpx<T>*)tw(), cd);
    }

    // P5: S4 (B) -> real outputs, two real rows per complex transform
    int zinv(const ZJobs<T>& zj, int njobs) {
        int nout = 0;
        for (int i = 0; i < njobs; ++i) nout += zj.fb[i] >= 0 ? 2 : 1;
        const double bytes = (double)nout * ((double)d.s4() * d.cpx_bytes + (double)d.ncell() * d.real_bytes);
        return launch(c, KD_ZINV, bytes, dim3((unsigned)(N * N / RW::RPB), njobs), dim3(RW::THREADS), 0,
                      k_zinv<T, N>, (const cpx<T>*)B(), (size_t)L.b_field_s4, zj, (const cpx<T>*)tw(), cd);
    }

    // P4 + P5 for nf fields of S3 into real outputs out[0..nf-1]: fields two
    // by two, an odd last field two rows at a time
    int to_real(int nf, T* const* out) {
        CHECK(yinv(nf));
        ZJobs<T> zj{};
        int nj = 0;
        for (int i = 0; i < nf; i += 2, ++nj) {
            zj.fa[nj] = i;
            zj.outa[nj] = out[i];
            zj.fb[nj] = (i + 1 < nf) ? i + 1 : -1;
            zj.outb[nj] = (i + 1 < nf) ? out[i + 1] : nullptr;
        }
        return zinv(zj, nj);
    }

    int copy(const T* src, T* dst) {
        return launch(c, KD_COPY, 2.0 * d.ncell() * d.real_bytes, dim3(2048), dim3(256), 0, k_copy<T>, src, dst,
                      (size_t)d.ncell());
    }
};

template <typename T>
XArgs<T> make_xargs(const Dims& d, int n, int nout, int64_t n2max, cpx<T>* cube_d, cpx<T>* cube_t) {
    XArgs<T> a{};
    a.cube_d = cube_d;
    a.cube_t = cube_t;
    a.n = n;
    a.nout = nout;
    a.n2max = n2max;
    a.kF = 2.0 * M_PI;  // replaced by the caller with 2 pi / L
    a.invN3 = 1.0 / ((double)d.N * d.N * d.N);
    return a;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

int32_t gridspt_version(void) { return 100; }

const char* gridspt_status_string(int s) {
    switch (s) {
        case GRIDSPT_OK: return "ok";
        case GRIDSPT_EINVAL: return "invalid argument";
        case GRIDSPT_EUNSUPPORTED: return "unsupported configuration";
        case GRIDSPT_EWORKSPACE: return "workspace missing or too small";
        case GRIDSPT_EALIGN: return "device pointer null or not 256-byte aligned";
        case GRIDSPT_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

int gridspt_create(gridspt_ctx** out, void* hip_stream) {
    if (!out) return GRIDSPT_EINVAL;
    gridspt_ctx* c = new (std::nothrow) gridspt_ctx();
    if (!c) return GRIDSPT_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    return GRIDSPT_OK;
}

void gridspt_destroy(gridspt_ctx* c) {
    if (!c) return;
    for (auto& r : c->recs) {
        if (r.start) (void)hipEventDestroy(r.start);
        if (r.stop) (void)hipEventDestroy(r.stop);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

int gridspt_sync(gridspt_ctx* c) {
    if (!c) return GRIDSPT_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return GRIDSPT_EHIP;
    if (hipGetLastError() != hipSuccess) return GRIDSPT_EHIP;
    return GRIDSPT_OK;
}

int gridspt_set_profiling(gridspt_ctx* c, int32_t enable) {
    if (!c) return GRIDSPT_EINVAL;
    c->profile = enable != 0;
    return GRIDSPT_OK;
}

int gridspt_profile_read(gridspt_ctx* c, int32_t max, char* names, int64_t* launches, double* ms, double* bytes) {
    if (!c || max < 0) return GRIDSPT_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return GRIDSPT_EHIP;
    double tot_ms[KD_COUNT] = {0}, tot_b[KD_COUNT] = {0};
    int64_t cnt[KD_COUNT] = {0};
    for (auto& r : c->recs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) return GRIDSPT_EHIP;
        tot_ms[r.kind] += t;
        tot_b[r.kind] += r.bytes;
        cnt[r.kind] += 1;
        c->pool.push_back(r.start);
        c->pool.push_back(r.stop);
    }
    c->recs.clear();
    int k = 0;
    for (int i = 0; i < KD_COUNT && k < max; ++i) {
        if (!cnt[i]) continue;
        if (names) {
            std::memset(names + 32 * k, 0, 32);
            std::strncpy(names + 32 * k, kKindNames[i], 31);
        }
        if (launches) launches[k] = cnt[i];
        if (ms) ms[k] = tot_ms[i];
        if (bytes) bytes[k] = tot_b[i];
        ++k;
    }
    return k;
}

int64_t gridspt_cut_n2max(int32_t n, double box, double kcut) {
    if (n < 2 || (n & 1) || !(box > 0.0)) return GRIDSPT_EINVAL;
    if (!(kcut > 0.0)) {
        const int64_t nn = (int64_t)n * n;
        return (nn + 8) / 9 - 1;  // ceil(N^2 / 9) - 1
    }
    const long double x = (long double)kcut * (long double)box / (2.0L * 3.14159265358979323846264338327950288L);
    return (int64_t)std::floor(x * x);
}

int32_t gridspt_cube_kc(int64_t n2max) {
    if (n2max < 0) return GRIDSPT_EINVAL;
    return (int32_t)isqrt64(n2max);
}

int64_t gridspt_cube_elems(const gridspt_grid* g) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    return dims_of(g).cube();
}

int gridspt_linear_edges(int32_t nbins, int64_t num, int64_t den, int64_t n2max, int64_t* e) {
    if (nbins < 1 || num < 1 || den < 1 || n2max < 1 || !e) return GRIDSPT_EINVAL;
    if (nbins > kMaxBins) return GRIDSPT_EINVAL;
    const __int128 q = (__int128)nbins * nbins * den * den;
    e[0] = 1;
    for (int b = 1; b < nbins; ++b) {
        const __int128 p = (__int128)b * b * num * num;
        e[b] = (int64_t)((p + q - 1) / q);
        if (e[b] < 1) e[b] = 1;
    }
    const int64_t closed = (int64_t)((__int128)num * num / ((__int128)den * den)) + 1;
    e[nbins] = std::min(closed, n2max + 1);
    for (int b = 1; b <= nbins; ++b)
        if (e[b] < e[b - 1]) e[b] = e[b - 1];
    return GRIDSPT_OK;
}

// BBKS transfer function (Bardeen, Bond, Kaiser & Szalay 1986, Eq. G3)
static double host_p0(double k, double A, double ns, double gamma) {
    if (k <= 0.0) return 0.0;
    const double q = k / gamma, a = 2.34 * q;
    const double t = std::log1p(a) / a *
                     std::pow(1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4),
                              -0.25);
    return A * std::pow(k, ns) * t * t;
}

int gridspt_sigma8_amp(double sigma8, double ns, double gamma, double* amp) {
    if (!amp || !(sigma8 > 0.0) || !(gamma > 0.0)) return GRIDSPT_EINVAL;
    // sigma^2(8) = (1 / 2 pi^2) int d ln k k^3 P(k) W(8k)^2, Gauss-Legendre on
    // 400 panels in ln k over [1e-6, 1e4] h/Mpc
    static const double xg[5] = {0.0, -0.5384693101056831, 0.5384693101056831, -0.9061798459386640,
                                 0.9061798459386640};
    static const double wg[5] = {0.5688888888888889, 0.4786286704993665, 0.4786286704993665, 0.2369268850561891,
                                 0.2369268850561891};
    const double lo = std::log(1e-6), hi = std::log(1e4);
    const int panels = 4000;
    const double h = (hi - lo) / panels;
    double acc = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double mid = lo + (p + 0.5) * h;
        for (int i = 0; i < 5; ++i) {
            const double k = std::exp(mid + 0.5 * h * xg[i]), x = 8.0 * k;
            const double w = x < 1e-3 ? 1.0 - x * x / 10.0 : 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
            acc += 0.5 * h * wg[i] * k * k * k * host_p0(k, 1.0, ns, gamma) * w * w;
        }
    }
    const double s2 = acc / (2.0 * M_PI * M_PI);
    *amp = sigma8 * sigma8 / s2;
    return GRIDSPT_OK;
}

int gridspt_growth(double om, double ol, double z, double* dz) {
    if (!dz || !(om > 0.0) || ol < 0.0 || z < 0.0) return GRIDSPT_EINVAL;
    const double ok = 1.0 - om - ol;
    // D(a) propto E(a) int_0^a dx / (x E(x))^3, Gauss-Legendre panels in x
    static const double xg[5] = {0.0, -0.5384693101056831, 0.5384693101056831, -0.9061798459386640,
                                 0.9061798459386640};
    static const double wg[5] = {0.5688888888888889, 0.4786286704993665, 0.4786286704993665, 0.2369268850561891,
                                 0.2369268850561891};
    auto E = [&](double x) { return std::sqrt(om / (x * x * x) + ok / (x * x) + ol); };
    auto D = [&](double a) {
        const int panels = 2000;
        const double h = a / panels;
        double acc = 0.0;
        for (int p = 0; p < panels; ++p)
            for (int i = 0; i < 5; ++i) {
                const double x = (p + 0.5) * h + 0.5 * h * xg[i];
                acc += 0.5 * h * wg[i] / std::pow(x * E(x), 3);
            }
        return E(a) * acc;
    };
    *dz = D(1.0 / (1.0 + z)) / D(1.0);
    return GRIDSPT_OK;
}

int64_t gridspt_workspace_bytes(const gridspt_grid* g, int32_t nmax) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    return layout_of(dims_of(g), nmax).end;
}

int gridspt_linear_field(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, void* delta1,
                         void* delta1_k, void* work, int64_t work_bytes) {
    if (!c || !lp) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_mask(g, lp->n2max));
    if (!(lp->amp >= 0.0) || !(lp->gamma > 0.0) || !std::isfinite(lp->ns) || !std::isfinite(lp->growth))
        return GRIDSPT_EINVAL;
    CHECK(check_ptr(delta1));
    if (delta1_k) CHECK(check_ptr(delta1_k));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_workspace_bytes(g, 1)) return GRIDSPT_EWORKSPACE;
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        Pipe<T, N> p(c, g, work, 1);
        CHECK(p.twiddles());
        CHECK(p.zfwd_single(nullptr, true, lp->seed, lp->stream));
        CHECK(p.yfwd(1));
        XArgs<T> a = make_xargs<T>(p.d, 1, 1, lp->n2max, (cpx<T>*)delta1_k, nullptr);
        a.kF = 2.0 * M_PI / g->box;
        a.lin = {lp->amp, lp->ns, lp->gamma, lp->growth, (double)N * N * N / (g->box * g->box * g->box)};
        CHECK(p.xfused(XM_LINEAR, a));
        T* out[1] = {static_cast<T*>(delta1)};
        return p.to_real(1, out);
    });
}

int gridspt_forward(gridspt_ctx* c, const gridspt_grid* g, int64_t n2max, const void* field, void* field_k,
                    void* work, int64_t work_bytes) {
    if (!c) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_mask(g, n2max));
    CHECK(check_ptr(field));
    CHECK(check_ptr(field_k));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_workspace_bytes(g, 1)) return GRIDSPT_EWORKSPACE;
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        Pipe<T, N> p(c, g, work, 1);
        CHECK(p.twiddles());
        CHECK(p.zfwd_single(static_cast<const T*>(field), false, 0, 0));
        CHECK(p.yfwd(1));
        XArgs<T> a = make_xargs<T>(p.d, 1, 0, n2max, (cpx<T>*)field_k, nullptr);
        a.kF = 2.0 * M_PI / g->box;
        return p.xfused(XM_FORWARD, a);
    });
}

int gridspt_orders(gridspt_ctx* c, const gridspt_grid* g, int32_t nmax, int64_t n2max1, int64_t n2max2,
                   const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
                   void* const* theta_k, void* work, int64_t work_bytes) {
    if (!c) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    CHECK(check_mask(g, n2max1));
    if (nmax > 1) CHECK(check_mask(g, n2max2));
    CHECK(check_ptr(delta1));
    if (!delta || !theta) return GRIDSPT_EINVAL;
    for (int i = 0; i < nmax; ++i) {
        CHECK(check_ptr(delta[i]));
        if (i > 0) CHECK(check_ptr(theta[i]));
        else if (theta[0]) CHECK(check_ptr(theta[0]));
        if (delta_k && delta_k[i]) CHECK(check_ptr(delta_k[i]));
        if (theta_k && theta_k[i]) CHECK(check_ptr(theta_k[i]));
    }
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_workspace_bytes(g, nmax)) return GRIDSPT_EWORKSPACE;
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        Pipe<T, N> p(c, g, work, nmax);
        const double kF = 2.0 * M_PI / g->box;
        auto dk = [&](int i) { return delta_k ? (cpx<T>*)delta_k[i] : nullptr; };
        auto tk = [&](int i) { return theta_k ? (cpx<T>*)theta_k[i] : nullptr; };
        CHECK(p.twiddles());

        // order 1: delta_1 = theta_1 = W1 delta1_in; u_1 = (-ik/k^2) delta_1
        CHECK(p.zfwd_single(static_cast<const T*>(delta1), false, 0, 0));
        CHECK(p.yfwd(1));
        {
            const int nout = nmax > 1 ? 4 : 1;
            cpx<T>* ct = (tk(0) && tk(0) != dk(0)) ? tk(0) : nullptr;
            XArgs<T> a = make_xargs<T>(p.d, 1, nout, n2max1, dk(0), ct);
            a.kF = kF;
            CHECK(p.xfused(XM_ORDER1, a));
            T* out[4] = {static_cast<T*>(delta[0]), p.U(1, 0), p.U(1, 1), p.U(1, 2)};
            CHECK(p.to_real(nout, out));
            if (theta[0] && theta[0] != delta[0]) CHECK(p.copy(static_cast<const T*>(delta[0]), static_cast<T*>(theta[0])));
        }
        // orders n >= 2
        for (int n = 2; n <= nmax; ++n) {
            ProductInputs<T> pin{};
            for (int m = 1; m < n; ++m) {
                pin.d[m - 1] = static_cast<const T*>(delta[m - 1]);
                for (int j = 0; j < 3; ++j) pin.u[m - 1][j] = p.U(m, j);
            }
            CHECK(p.zfwd_products(n, pin));
            CHECK(p.yfwd(4));
            const int nout = n < nmax ? 5 : 2;
            XArgs<T> a = make_xargs<T>(p.d, n, nout, n2max2, dk(n - 1), tk(n - 1));
            a.kF = kF;
            CHECK(p.xfused(XM_ORDER, a));
            T* out[5] = {static_cast<T*>(delta[n - 1]), static_cast<T*>(theta[n - 1]), nullptr, nullptr, nullptr};
            if (n < nmax)
                for (int j = 0; j < 3; ++j) out[2 + j] = p.U(n, j);
            CHECK(p.to_real(nout, out));
        }
        return GRIDSPT_OK;
    });
}

int gridspt_sum_orders(gridspt_ctx* c, const gridspt_grid* g, int32_t nmax, const void* const* delta,
                       const double* coef, double* out) {
    if (!c || !delta || !coef) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nmax < 1 || nmax > 8) return GRIDSPT_EINVAL;
    for (int i = 0; i < nmax; ++i) CHECK(check_ptr(delta[i]));
    CHECK(check_ptr(out));
    const Dims d = dims_of(g);
    auto go = [&](auto tag) -> int {
        using T = typename decltype(tag)::type;
        SumArgs<T> s{};
        for (int i = 0; i < nmax; ++i) {
            s.d[i] = static_cast<const T*>(delta[i]);
            s.coef[i] = coef[i];
        }
        s.nmax = nmax;
        s.ncell = (size_t)d.ncell();
        s.out = out;
        const double bytes = (double)d.ncell() * (nmax * d.real_bytes + 8.0);
        return launch(c, KD_SUM_ORDERS, bytes, dim3(4096), dim3(256), 0, k_sum_orders<T>, s);
    };
    if (g->dtype == GRIDSPT_F64) return go(tag_t<double>{});
    return go(tag_t<float>{});
}

// per-wave LDS accumulators: nbins * (pairs + 2) doubles, at most 1792 (56 KB per block)
static int power_chunk(int nbins) {
    return std::max(1, std::min(kPowerPairsPerLaunch, 1792 / nbins - 2));
}
static int power_blocks(const Dims& d) {
    const int64_t halves = 2 * d.Kz * d.Ky;
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (halves + kPowerWaves - 1) / kPowerWaves));
}

int64_t gridspt_power_workspace_bytes(const gridspt_grid* g, int32_t npairs, int32_t nbins) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (npairs < 1 || npairs > kMaxPairs || nbins < 1 || nbins > kMaxBins) return GRIDSPT_EINVAL;
    const Dims d = dims_of(g);
    const int q = std::min(npairs, power_chunk(nbins)) + 2;
    // block partials, then the reduced sums
    return align_up((int64_t)power_blocks(d) * nbins * q * 8) + align_up((int64_t)nbins * q * 8);
}

int gridspt_power(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                  int32_t npairs, const int32_t* pairs, int32_t nbins, const int64_t* edge_n2, double* pk,
                  double* kmean, double* nmodes, void* work, int64_t work_bytes) {
    if (!c || !fields_k || !pairs || !edge_n2) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nfields < 1 || nfields > kMaxFields || npairs < 1 || npairs > kMaxPairs || nbins < 1 || nbins > kMaxBins)
        return GRIDSPT_EINVAL;
    for (int i = 0; i < 2 * npairs; ++i)
        if (pairs[i] < 0 || pairs[i] >= nfields) return GRIDSPT_EINVAL;
    if (edge_n2[0] < 1) return GRIDSPT_EINVAL;
    for (int b = 0; b < nbins; ++b)
        if (edge_n2[b + 1] < edge_n2[b]) return GRIDSPT_EINVAL;
    for (int i = 0; i < nfields; ++i) CHECK(check_ptr(fields_k[i]));
    CHECK(check_ptr(pk));
    if (kmean) CHECK(check_ptr(kmean));
    if (nmodes) CHECK(check_ptr(nmodes));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_power_workspace_bytes(g, npairs, nbins)) return GRIDSPT_EWORKSPACE;
    const Dims d = dims_of(g);
    const int nblk = power_blocks(d);
    const int chunk = power_chunk(nbins);
    auto go = [&](auto tag) -> int {
        using T = typename decltype(tag)::type;
        double* partial = static_cast<double*>(work);
        double* sums = reinterpret_cast<double*>(static_cast<char*>(work) +
                                                 align_up((int64_t)nblk * nbins * (std::min(npairs, chunk) + 2) * 8));
        for (int p0 = 0; p0 < npairs; p0 += chunk) {
            const int np = std::min(chunk, npairs - p0);
            PowerArgs<T> a{};
            // distinct fields of this chunk
            int slot_of[kMaxFields];
            for (int i = 0; i < kMaxFields; ++i) slot_of[i] = -1;
            int nf = 0;
            for (int q = 0; q < np; ++q)
                for (int k = 0; k < 2; ++k) {
                    const int f = pairs[2 * (p0 + q) + k];
                    if (slot_of[f] < 0) {
                        slot_of[f] = nf;
                        a.f[nf++] = static_cast<const cpx<T>*>(fields_k[f]);
                    }
                }
            for (int q = 0; q < np; ++q) {
                a.pa[q] = slot_of[pairs[2 * (p0 + q)]];
                a.pb[q] = slot_of[pairs[2 * (p0 + q) + 1]];
            }
            for (int b = 0; b <= nbins; ++b) a.edges[b] = edge_n2[b];
            a.nf = nf;
            a.npairs = np;
            a.nbins = nbins;
            a.kF = 2.0 * M_PI / g->box;
            a.partial = partial;
            const int nq = np + 2;
            const size_t shm = (size_t)kPowerWaves * nbins * nq * sizeof(double);
            CHECK(launch(c, KD_POWER, (double)nf * d.cube() * d.cpx_bytes, dim3(nblk), dim3(64 * kPowerWaves), shm,
                         k_power_partial<T>, a, CubeDims{(int)d.Kc, (int)d.Kz, (int)d.Ky}));
            CHECK(launch(c, KD_POWER_FINAL, (double)nblk * nbins * nq * 8.0, dim3(nbins * nq), dim3(kReduceThreads),
                         0, k_power_reduce, (const double*)partial, nblk, nq, sums));
            CHECK(launch(c, KD_POWER_FINAL, 0.0, dim3((nbins + 63) / 64), dim3(64), 0, k_power_final,
                         (const double*)sums, nbins, np, g->box * g->box * g->box, pk + (size_t)p0 * nbins, nbins,
                         p0 == 0 ? kmean : nullptr, p0 == 0 ? nmodes : nullptr));
        }
        return GRIDSPT_OK;
    };
    if (g->dtype == GRIDSPT_F64) return go(tag_t<double>{});
    return go(tag_t<float>{});
}

// ---------------------------------------------------------------------------
// bispectrum
// ---------------------------------------------------------------------------

namespace {

struct BispPlan {
    std::vector<std::pair<int, int>> slots;  // (field or -1 for the indicator, bin)
    std::map<std::pair<int, int>, int> index;
    int slot(int f, int b) {
        auto key = std::make_pair(f, b);
        auto it = index.find(key);
        if (it != index.end()) return it->second;
        const int s = (int)slots.size();
        slots.push_back(key);
        index[key] = s;
        return s;
    }
};

constexpr int kTripleBlocks = 1024;

int bisp_plan(int ntri, const int32_t* tri_bins, int nterms, const int32_t* terms, BispPlan& bp) {
    for (int t = 0; t < ntri; ++t)
        for (int i = 0; i < 3; ++i) bp.slot(-1, tri_bins[3 * t + i]);
    for (int u = 0; u < nterms; ++u) {
        const int t = terms[4 * u + 3];
        for (int i = 0; i < 3; ++i) bp.slot(terms[4 * u + i], tri_bins[3 * t + i]);
    }
    return GRIDSPT_OK;
}

int64_t bisp_bytes(const Dims& d, int nslots) {
    const Layout L = layout_of(d, 1);
    int64_t off = L.end;
    off = align_up(off + (int64_t)nslots * d.ncell() * d.real_bytes);
    off = align_up(off + (int64_t)kTripleBlocks * 8 * 8);
    return off;
}

}  // namespace

int64_t gridspt_bispectrum_workspace_bytes(const gridspt_grid* g, int32_t ntri, const int32_t* tri_bins,
                                           int32_t nterms, const int32_t* terms) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (ntri < 1 || nterms < 1 || !tri_bins || !terms) return GRIDSPT_EINVAL;
    BispPlan bp;
    for (int u = 0; u < nterms; ++u)
        if (terms[4 * u + 3] < 0 || terms[4 * u + 3] >= ntri) return GRIDSPT_EINVAL;
    bisp_plan(ntri, tri_bins, nterms, terms, bp);
    return bisp_bytes(dims_of(g), (int)bp.slots.size());
}

int gridspt_bispectrum(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                       int32_t ntri, const int32_t* tri_bins, int32_t nterms, const int32_t* terms, int32_t nbins,
                       const int64_t* edge_n2, double* bk, double* ntriangles, void* work, int64_t work_bytes) {
    if (!c || !fields_k || !tri_bins || !terms || !edge_n2) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nfields < 1 || nfields > kMaxFields || ntri < 1 || nterms < 1 || nbins < 1 || nbins > kMaxBins)
        return GRIDSPT_EINVAL;
    if (ntri > 4096 || nterms > 16384) return GRIDSPT_EINVAL;
    for (int t = 0; t < 3 * ntri; ++t)
        if (tri_bins[t] < 0 || tri_bins[t] >= nbins) return GRIDSPT_EINVAL;
    for (int u = 0; u < nterms; ++u) {
        for (int i = 0; i < 3; ++i)
            if (terms[4 * u + i] < 0 || terms[4 * u + i] >= nfields) return GRIDSPT_EINVAL;
        if (terms[4 * u + 3] < 0 || terms[4 * u + 3] >= ntri) return GRIDSPT_EINVAL;
    }
    if (edge_n2[0] < 1) return GRIDSPT_EINVAL;
    for (int b = 0; b < nbins; ++b)
        if (edge_n2[b + 1] < edge_n2[b]) return GRIDSPT_EINVAL;
    if (isqrt64(edge_n2[nbins] - 1) > g->kc) return GRIDSPT_EINVAL;  // shells must lie inside the cube
    for (int i = 0; i < nfields; ++i) CHECK(check_ptr(fields_k[i]));
    CHECK(check_ptr(bk));
    CHECK(check_ptr(ntriangles));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    BispPlan bp;
    bisp_plan(ntri, tri_bins, nterms, terms, bp);
    const Dims d = dims_of(g);
    if (work_bytes < bisp_bytes(d, (int)bp.slots.size())) return GRIDSPT_EWORKSPACE;
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        Pipe<T, N> p(c, g, work, 1);
        const int ns = (int)bp.slots.size();
        char* base = static_cast<char*>(work);
        T* slotmem = reinterpret_cast<T*>(base + p.L.end);
        double* partial = reinterpret_cast<double*>(base + align_up(p.L.end + (int64_t)ns * d.ncell() * d.real_bytes));
        auto slot_ptr = [&](int s) { return slotmem + (size_t)s * d.ncell(); };
        CHECK(p.twiddles());
        // shell-filtered fields, five at a time
        for (int s0 = 0; s0 < ns; s0 += 5) {
            const int nb = std::min(5, ns - s0);
            ShellSlots<T> sh{};
            for (int i = 0; i < nb; ++i) {
                const auto& sl = bp.slots[s0 + i];
                sh.cube[i] = sl.first >= 0 ? static_cast<const cpx<T>*>(fields_k[sl.first]) : nullptr;
                sh.lo[i] = edge_n2[sl.second];
                sh.hi[i] = edge_n2[sl.second + 1];
            }
            CHECK(p.xshell(sh, nb));
            T* outs[5];
            for (int i = 0; i < nb; ++i) outs[i] = slot_ptr(s0 + i);
            CHECK(p.to_real(nb, outs));
        }
        // triple products: the terms, then the triangle counts; sums land in
        // the first nterms + ntri doubles after the partials
        double* sums = reinterpret_cast<double*>(p.B());  // S2/S4 buffer is free now
        auto triple = [&](const std::vector<std::array<int, 3>>& items, double* dst) -> int {
            for (size_t u0 = 0; u0 < items.size(); u0 += 8) {
                TripleArgs<T> t{};
                t.nterms = (int)std::min<size_t>(8, items.size() - u0);
                t.ncell = (size_t)d.ncell();
                t.partial = partial;
                for (int i = 0; i < t.nterms; ++i) {
                    t.a[i] = slot_ptr(items[u0 + i][0]);
                    t.b[i] = slot_ptr(items[u0 + i][1]);
                    t.c[i] = slot_ptr(items[u0 + i][2]);
                }
                CHECK(launch(c, KD_TRIPLE, 3.0 * t.nterms * d.ncell() * d.real_bytes, dim3(kTripleBlocks),
                             dim3(kTripleThreads), 0, k_triple_partial<T>, t));
                CHECK(launch(c, KD_TRIPLE_FINAL, kTripleBlocks * 8.0 * 8.0, dim3(1), dim3(64), 0, k_triple_final,
                             (const double*)partial, kTripleBlocks, t.nterms, dst + u0));
            }
            return GRIDSPT_OK;
        };
        std::vector<std::array<int, 3>> titems(nterms), jitems(ntri);
        for (int u = 0; u < nterms; ++u) {
            const int t = terms[4 * u + 3];
            for (int i = 0; i < 3; ++i) titems[u][i] = bp.index[{terms[4 * u + i], tri_bins[3 * t + i]}];
        }
        for (int t = 0; t < ntri; ++t)
            for (int i = 0; i < 3; ++i) jitems[t][i] = bp.index[{-1, tri_bins[3 * t + i]}];
        CHECK(triple(titems, sums));
        CHECK(triple(jitems, sums + nterms));
        // bk = L^6 T / J per term, the term -> triangle map in the argument buffer
        const double vol2 = std::pow(g->box, 6);
        const double invN3 = 1.0 / (double)d.ncell();
        for (int u0 = 0; u0 < std::max(nterms, ntri); u0 += 64) {
            TriMap m{};
            const int nu = std::max(0, std::min(64, nterms - u0));
            const int nt = std::max(0, std::min(64, ntri - u0));
            for (int i = 0; i < nu; ++i) m.tri[i] = terms[4 * (u0 + i) + 3];
            CHECK(launch(c, KD_BISP_FINAL, 0.0, dim3(1), dim3(64), 0, k_bisp_final, (const double*)sums,
                         (const double*)(sums + nterms), m, u0, nu, nt, vol2, invN3, bk, ntriangles));
        }
        return GRIDSPT_OK;
    });
}

}  // extern "C"

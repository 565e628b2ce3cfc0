// Pass sequences of the entry points (Sec. II C): the five-pass transform
// pipeline of one grid size, with each pass launched in the variant the
// tuning table names and over a batch of realisations (gridDim.z).
// Included once per grid size by the files under sizes/, which instantiate
// the run_* functions declared in runtime.hpp.
#pragma once
#include "runtime.hpp"

namespace gridspt {

// Launch variants compiled per (precision, size) (see variant_list): the
// autotuner chooses among these per pass kind.
template <typename T, int N>
struct Variants {
    static constexpr bool two = tuned_pow2(sizeof(T) == 4, N);
    static constexpr bool three = tuned_three(sizeof(T) == 4, N);
    using list = std::conditional_t<two, std::integer_sequence<int, 0, 1, 4, 5>,
                                    std::conditional_t<three, std::integer_sequence<int, 0, 1, 2>,
                                                       std::integer_sequence<int, 0>>>;
};

template <typename F, int... Vs>
int with_variant_impl(int v, F&& f, std::integer_sequence<int, Vs...>) {
    int rc = GRIDSPT_EUNSUPPORTED;
    (void)((v == Vs ? (rc = f(std::integral_constant<int, Vs>{}), true) : false) || ...);
    return rc;
}
template <typename T, int N, typename F>
int with_variant(int v, F&& f) {
    return with_variant_impl(v, f, typename Variants<T, N>::list{});
}

template <typename T, int N>
struct Pipe {
    gridspt_ctx* c;
    Dims d;
    Layout L;
    char* ws;  // realisation 0's workspace
    CubeDims cd;
    const Tuning& tu;
    Batch bt;

    Pipe(gridspt_ctx* ctx, const gridspt_grid* g, void* work, int nmax, const Tuning& t, Batch b)
        : c(ctx), d(dims_of(g)), tu(t), bt(b) {
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
    double nb() const { return (double)bt.nreal; }
    unsigned nz() const { return (unsigned)bt.nreal; }

    // radial amplitude table of the linear field (realisation 0's workspace)
    double* amp() const { return reinterpret_cast<double*>(ws + L.amp); }
    int amp_table(const gridspt_grid* g, const gridspt_linpk* lp) {
        const LinParams lin{lp->amp, lp->ns, lp->gamma, lp->growth, (double)N * N * N / (g->box * g->box * g->box)};
        const int64_t n = lp->n2max + 1;
        return launch(c, KD_TWIDDLE, (double)n * 8.0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, k_amp_table,
                      amp(), lp->n2max, 2.0 * M_PI / g->box, 1.0 / ((double)N * N * N), lin);
    }

    // the shared table, computed once (realisation 0's workspace)
    int twiddles() {
        return launch(c, KD_TWIDDLE, (double)N * d.cpx_bytes, dim3((N + 255) / 256), dim3(256), 0, k_twiddles<T>,
                      tw(), N);
    }

    // P1 from a real field (SRC 0) or from noise (SRC 1) -> S1 field 0 in A
    int zfwd_single(const T* f, bool noise, uint64_t seed, uint64_t stream) {
        const int kind = noise ? KD_ZFWD_NOISE : KD_ZFWD_FIELD;
        return with_variant<T, N>(tu.v[kind], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            ProductInputs<T> pin{};
            const double bytes = nb() * ((noise ? 0.0 : (double)d.ncell() * d.real_bytes) + (double)d.s1() * d.cpx_bytes);
            const dim3 grid(N * (N / (2 * RW::RPB)), 1, nz()), block(RW::THREADS);  // two rows per transform
            if (noise)
                return launch(c, kind, bytes, grid, block, 0, k_zfwd<T, N, V, 1>, f, pin, seed, stream, A(),
                              (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz, bt.zs);
            return launch(c, kind, bytes, grid, block, 0, k_zfwd<T, N, V, 0>, f, pin, seed, stream, A(),
                          (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz, bt.zs);
        });
    }

    // P1 of four real fields (packed two per transform) -> S1 fields 0..3 in A
    int zfwd_four(const T* const* f) {
        return with_variant<T, N>(tu.v[KD_ZFWD_ADJ], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            ProductInputs<T> pin{};
            for (int i = 0; i < 4; ++i) pin.d[i] = f[i];
            const double bytes = nb() * (4.0 * d.ncell() * d.real_bytes + 4.0 * d.s1() * d.cpx_bytes);
            return launch(c, KD_ZFWD_ADJ, bytes, dim3(N * (N / RW::RPB), 1, nz()), dim3(RW::THREADS), 0,
                          k_zfwd<T, N, V, 3>, (const T*)nullptr, pin, (uint64_t)0, (uint64_t)0, A(),
                          (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz, bt.zs);
        });
    }

    // P1 of two real fields packed as one complex transform -> S1 fields 0, 1 in A
    int zfwd_pair(const T* f0, const T* f1) {
        return with_variant<T, N>(tu.v[KD_ZFWD_PAIR], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            ProductInputs<T> pin{};
            pin.d[0] = f0;
            pin.d[1] = f1;
            const double bytes = nb() * (2.0 * d.ncell() * d.real_bytes + 2.0 * d.s1() * d.cpx_bytes);
            return launch(c, KD_ZFWD_PAIR, bytes, dim3(N * (N / RW::RPB), 1, nz()), dim3(RW::THREADS), 0,
                          k_zfwd<T, N, V, 4>, (const T*)nullptr, pin, (uint64_t)0, (uint64_t)0, A(),
                          (size_t)L.a_field_s1, (const cpx<T>*)tw(), (int)d.Kz, bt.zs);
        });
    }

    // P3 of the P-form derived fields of one order, chunk 0..2 (five fields) -> S3 (A)
    int xderived(RegenArgs<T> r, int chunk) {
        r.s3 = A();
        r.s3_field = (size_t)L.a_field_s3;
        return with_variant<T, N>(tu.v[KD_XDERIVED], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const double bytes = nb() * ((chunk == 0 ? 2.0 : 1.0) * d.cube() + 5.0 * d.s3()) * d.cpx_bytes;
            const dim3 grid((unsigned)(d.Kz * ((d.Ky + RW::RPB - 1) / RW::RPB)), 1, nz()), block(RW::THREADS);
            const cpx<T>* t = tw();
            switch (chunk) {
                case 0: return launch(c, KD_XDERIVED, bytes, grid, block, 0, k_xderived<T, N, V, 0>, r, t, cd, bt.zs);
                case 1: return launch(c, KD_XDERIVED, bytes, grid, block, 0, k_xderived<T, N, V, 1>, r, t, cd, bt.zs);
                default: return launch(c, KD_XDERIVED, bytes, grid, block, 0, k_xderived<T, N, V, 2>, r, t, cd, bt.zs);
            }
        });
    }

    // P3 of smoothed spectra -> S3 (A), one output per input
    int xsmooth(SmoothArgs<T> sa) {
        sa.s3 = A();
        sa.s3_field = (size_t)L.a_field_s3;
        return with_variant<T, N>(tu.v[KD_XSMOOTH], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const double bytes = nb() * ((double)sa.nin * d.cube() + (double)sa.nin * d.s3()) * d.cpx_bytes;
            return launch(c, KD_XSMOOTH, bytes, dim3((unsigned)(d.Kz * ((d.Ky + RW::RPB - 1) / RW::RPB)), 1, nz()),
                          dim3(RW::THREADS), 0, k_xsmooth<T, N, V>, sa, (const cpx<T>*)tw(), cd, bt.zs);
        });
    }

    // P3 from stored spectra: delta_m, u_m (4 fields) -> S3 (A)
    int xregen(RegenArgs<T> r) {
        r.s3 = A();
        r.s3_field = (size_t)L.a_field_s3;
        return with_variant<T, N>(tu.v[KD_XREGEN], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const double bytes = nb() * (2.0 * d.cube() + 4.0 * d.s3()) * d.cpx_bytes;
            return launch(c, KD_XREGEN, bytes, dim3((unsigned)(d.Kz * ((d.Ky + RW::RPB - 1) / RW::RPB)), 1, nz()),
                          dim3(RW::THREADS), 0, k_xregen<T, N, V>, r, (const cpx<T>*)tw(), cd, bt.zs);
        });
    }

    // P5 of the latest order's delta, u (S4 fields of ch, in B) chained into P1
    // with the products of order n -> S1 fields 0..3 (V_x, V_y, V_z, W) in A
    int zchain(int n, const ProductInputs<T>& pin, ChainArgs<T> ch) {
        ch.s4 = B();
        ch.s4_field = (size_t)L.b_field_s4;
        return with_variant<T, N>(tu.v[KD_ZFWD_PRODUCTS], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            int nst = ch.dup ? 1 : 0;
            for (int i = 0; i < 4; ++i) nst += ch.out[i] ? 1 : 0;
            const double bytes = nb() * ((4.0 * (n - 2) + nst) * d.ncell() * d.real_bytes +
                                         (4.0 * N * N * cd.Kz + 4.0 * d.s1()) * d.cpx_bytes);
            const dim3 grid(N * (N / RW::RPB), 1, nz()), block(RW::THREADS);
            auto go = [&](auto kern) {
                return launch(c, KD_ZFWD_PRODUCTS, bytes, grid, block, 0, kern, pin, ch, A(), (size_t)L.a_field_s1,
                              (const cpx<T>*)tw(), (int)d.Kz, bt.zs);
            };
            switch (n) {
                case 2: return go(k_zchain<T, N, V, 2>);
                case 3: return go(k_zchain<T, N, V, 3>);
                case 4: return go(k_zchain<T, N, V, 4>);
                case 5: return go(k_zchain<T, N, V, 5>);
                default: return (int)GRIDSPT_EINVAL;
            }
        });
    }

    // P2: nf fields S1 (A) -> S2 (B)
    int yfwd(int nf) {
        return with_variant<T, N>(tu.v[KD_YFWD], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const double bytes = nb() * nf * (d.s1() + d.s2()) * d.cpx_bytes;
            return launch(c, KD_YFWD, bytes, dim3((unsigned)(N * ((d.Kz + RW::RPB - 1) / RW::RPB)), nf, nz()),
                          dim3(RW::THREADS), 0,
                          k_yfwd<T, N, V>, (const cpx<T>*)A(), (size_t)L.a_field_s1, B(), (size_t)L.b_field_s2,
                          (const cpx<T>*)tw(), cd, bt.zs, 1, 1, (int)d.s2_row());
        });
    }

    // P2 for the products of an order: S1 fields V_x, V_y, V_z, W (A) -> S2 fields
    // V_x, i (ky V_y + kz V_z), W (B); V_x and W in one plain launch (inputs 0, 3
    // to outputs 0, 2), the combined field in its own
    int yfwd_products() {
        return with_variant<T, N>(tu.v[KD_YFWD], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const dim3 grid((unsigned)(N * ((d.Kz + RW::RPB - 1) / RW::RPB)), 2, nz()), block(RW::THREADS);
            GRIDSPT_CHECK(launch(c, KD_YFWD, nb() * 2.0 * (d.s1() + d.s2()) * d.cpx_bytes, grid, block, 0,
                                 k_yfwd<T, N, V>, (const cpx<T>*)A(), (size_t)L.a_field_s1, B(),
                                 (size_t)L.b_field_s2, (const cpx<T>*)tw(), cd, bt.zs, 3, 2, (int)d.s2_row()));
            return launch(c, KD_YFWD, nb() * (2.0 * d.s1() + d.s2()) * d.cpx_bytes, dim3(grid.x, 1, nz()),
                          dim3(2 * RW::THREADS), 0, k_yfwd<T, N, V, true>, (const cpx<T>*)A(), (size_t)L.a_field_s1, B(), (size_t)L.b_field_s2,
                          (const cpx<T>*)tw(), cd, bt.zs, 0, 0, (int)d.s2_row());
        });
    }

    // P3: S2 (B) -> S3 (A), with the k-space step of `mode`
    int xfused(int mode, XArgs<T> a) {
        a.s2 = B();
        a.s2_field = (size_t)L.b_field_s2;
        a.s2_row = (int)d.s2_row();
        a.s3 = A();
        a.s3_field = (size_t)L.a_field_s3;
        const int kind = mode == XM_ORDER    ? KD_XFUSED_ORDER
                         : mode == XM_ORDER1 ? KD_XFUSED_ORDER1
                         : mode == XM_LINEAR ? KD_XFUSED_LINEAR
                         : mode == XM_ADJ    ? KD_XFUSED_ADJ
                         : mode == XM_ADJ1   ? KD_XFUSED_ADJ1
                         : mode == XM_PFORM  ? KD_XFUSED_PFORM
                         : mode == XM_LIN_ORDER1 ? KD_XFUSED_LINEAR
                                             : KD_XFUSED_FORWARD;
        return with_variant<T, N>(tu.v[kind], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const int nin = mode == XM_ORDER ? 3 : ((mode == XM_ADJ || mode == XM_ADJ1) ? a.nin : (mode == XM_PFORM ? 2 : 1));
            const int ncube = (a.cube_d ? 1 : 0) + (a.cube_t ? 1 : 0);
            const double bytes =
                nb() * ((double)nin * d.s2() + (double)a.nout * d.s3() + (double)ncube * d.cube()) * d.cpx_bytes;
            const dim3 grid((unsigned)(d.Kz * ((d.Ky + RW::RPB - 1) / RW::RPB)), 1, nz()), block(RW::THREADS);
            const cpx<T>* t = tw();
            switch (mode) {
                case XM_ORDER: return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_ORDER>, a, t, cd, bt.zs);
                case XM_ORDER1:
                    return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_ORDER1>, a, t, cd, bt.zs);
                case XM_LINEAR:
                    return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_LINEAR>, a, t, cd, bt.zs);
                case XM_ADJ: return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_ADJ>, a, t, cd, bt.zs);
                case XM_PFORM:
                    return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_PFORM>, a, t, cd, bt.zs);
                case XM_LIN_ORDER1:
                    return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_LIN_ORDER1>, a, t, cd, bt.zs);
                case XM_ADJ1:
                    return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_ADJ1>, a, t, cd, bt.zs);
                default:
                    return launch(c, kind, bytes, grid, block, 0, k_xfused<T, N, V, XM_FORWARD>, a, t, cd, bt.zs);
            }
        });
    }

    // P3 for shells: nslot cube fields -> S3 (A)
    int xshell(ShellSlots<T> s, int nslot) {
        s.s3 = A();
        s.s3_field = (size_t)L.a_field_s3;
        return with_variant<T, N>(tu.v[KD_XSHELL], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            int ncube = 0;
            for (int i = 0; i < nslot; ++i) ncube += s.cube[i] ? 1 : 0;
            // cd may be smaller than the cube of s.src (shells of small radius)
            const double rows = (double)cd.Kz * cd.Ky;
            const double bytes = nb() * ((double)ncube * rows * cd.Ky + (double)nslot * rows * N) * d.cpx_bytes;
            return launch(c, KD_XSHELL, bytes, dim3((unsigned)(cd.Kz * ((cd.Ky + RW::RPB - 1) / RW::RPB)), nslot, nz()),
                          dim3(RW::THREADS), 0, k_xshell<T, N, V>, s, (const cpx<T>*)tw(), cd, bt.zs);
        });
    }

    // P4: nf fields S3 (A) -> S4 (B)
    int yinv(int nf) {
        return with_variant<T, N>(tu.v[KD_YINV], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const double bytes = nb() * nf * ((double)cd.Kz * N * cd.Ky + (double)N * N * cd.Kz) * d.cpx_bytes;
            return launch(c, KD_YINV, bytes, dim3((unsigned)(cd.Kz * (N / RW::RPB)), nf, nz()),
                          dim3(RW::THREADS), 0, k_yinv<T, N, V>, (const cpx<T>*)A(), (size_t)L.a_field_s3, B(),
                          (size_t)L.b_field_s4, (const cpx<T>*)tw(), cd, bt.zs);
        });
    }

    // P4 of phi (S3 field f in A) -> S4 fields f (the transform of ky phi, u_y) and
    // f + 1 (phi, u_z / kz) in B
    int yinv_yz(int f) {
        return with_variant<T, N>(tu.v[KD_YINV], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            const double bytes = nb() * ((double)cd.Kz * N * cd.Ky + 2.0 * N * N * cd.Kz) * d.cpx_bytes;
            return launch(c, KD_YINV, bytes, dim3((unsigned)(cd.Kz * (N / RW::RPB)), 1, nz()), dim3(RW::THREADS), 0,
                          k_yinv<T, N, V, true>, (const cpx<T>*)(A() + (size_t)f * L.a_field_s3),
                          (size_t)L.a_field_s3, B() + (size_t)f * L.b_field_s4, (size_t)L.b_field_s4,
                          (const cpx<T>*)tw(), cd, bt.zs);
        });
    }

    // P5: S4 (B) -> real outputs, two real rows per complex transform
    int zinv(const ZJobs<T>& zj, int njobs) {
        return with_variant<T, N>(tu.v[KD_ZINV], [&](auto vc) {
            constexpr int V = decltype(vc)::value;
            using RW = Rows<T, N, V>;
            int ndup = 0;
            for (int j = 0; j < njobs; ++j) ndup += zj.dup[j] != nullptr;
            const double bytes = nb() * (njobs * (double)N * N * cd.Kz * d.cpx_bytes +
                                         (njobs + ndup) * (double)d.ncell() * d.real_bytes);
            return launch(c, KD_ZINV, bytes, dim3((unsigned)(N * N / (2 * RW::RPB)), njobs, nz()),
                          dim3(RW::THREADS), 0, k_zinv<T, N, V>, (const cpx<T>*)B(), (size_t)L.b_field_s4, zj,
                          (const cpx<T>*)tw(), cd, bt.zs);
        });
    }

    // P4 + P5 for nf <= 8 fields of S3 into real outputs out[0..nf-1], one z
    // inverse job per field; dup0, if set, receives a second copy of field 0
    int to_real(int nf, T* const* out, T* dup0 = nullptr) {
        if (nf < 1 || nf > 8) return GRIDSPT_EINVAL;
        GRIDSPT_CHECK(yinv(nf));
        ZJobs<T> zj{};
        for (int i = 0; i < nf; ++i) {
            zj.f[i] = i;
            zj.out[i] = out[i];
        }
        zj.dup[0] = dup0;
        return zinv(zj, nf);
    }
};

template <typename T>
XArgs<T> make_xargs(const Dims& d, const gridspt_grid* g, int n, int nout, int64_t n2max, cpx<T>* cube_d,
                    cpx<T>* cube_t) {
    XArgs<T> a{};
    a.cube_d = cube_d;
    a.cube_t = cube_t;
    a.n = n;
    a.nout = nout;
    a.n2max = n2max;
    a.kF = 2.0 * M_PI / g->box;
    a.invN3 = 1.0 / ((double)d.N * d.N * d.N);
    return a;
}

// Step 1: Gaussian noise (drawn, or given in `noise`) -> masked linear field
// delta_1 (and its cube)
template <typename T, int N>
int run_linear_field(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, const void* noise,
                     void* delta1, void* delta1_k, void* work, const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, 1, tu, b);
    GRIDSPT_CHECK(p.twiddles());
    GRIDSPT_CHECK(p.amp_table(g, lp));
    GRIDSPT_CHECK(p.zfwd_single(static_cast<const T*>(noise), noise == nullptr, lp->seed, lp->stream));
    GRIDSPT_CHECK(p.yfwd(1));
    XArgs<T> a = make_xargs<T>(p.d, g, 1, 1, lp->n2max, (cpx<T>*)delta1_k, nullptr);
    a.amp = p.amp();
    GRIDSPT_CHECK(p.xfused(XM_LINEAR, a));
    T* out[1] = {static_cast<T*>(delta1)};
    return p.to_real(1, out);
}

// Masked forward transform of a real field into the cube layout
template <typename T, int N>
int run_forward(gridspt_ctx* c, const gridspt_grid* g, int64_t n2max, const void* field, void* field_k, void* work,
                const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, 1, tu, b);
    GRIDSPT_CHECK(p.twiddles());
    GRIDSPT_CHECK(p.zfwd_single(static_cast<const T*>(field), false, 0, 0));
    GRIDSPT_CHECK(p.yfwd(1));
    XArgs<T> a = make_xargs<T>(p.d, g, 1, 0, n2max, (cpx<T>*)field_k, nullptr);
    return p.xfused(XM_FORWARD, a);
}

// Orders 1..nmax of the recursion (Eq. 10 in the divergence form)
template <typename T, int N>
int run_orders(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int nmax, int64_t n2max1,
               int64_t n2max2, const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
               void* const* theta_k, void* work, const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, nmax, tu, b);
    auto dk = [&](int i) { return delta_k ? (cpx<T>*)delta_k[i] : nullptr; };
    auto tk = [&](int i) { return theta_k ? (cpx<T>*)theta_k[i] : nullptr; };
    OrderTag tag(c, 1);  // launches of order 1 (with the linear field), then of each order n
    GRIDSPT_CHECK(p.twiddles());

    // order 1: delta_1 = theta_1 = W1 delta1_in (or the linear field of lp);
    // u_1 = (-ik/k^2) delta_1
    if (lp) {
        GRIDSPT_CHECK(p.amp_table(g, lp));
        GRIDSPT_CHECK(p.zfwd_single(nullptr, true, lp->seed, lp->stream));
    } else {
        GRIDSPT_CHECK(p.zfwd_single(static_cast<const T*>(delta1), false, 0, 0));
    }
    GRIDSPT_CHECK(p.yfwd(1));
    ChainArgs<T> chain{};
    {
        const int nout = nmax > 1 ? 3 : 1;  // delta_1 (, u_x, phi)
        cpx<T>* ct = (tk(0) && tk(0) != dk(0)) ? tk(0) : nullptr;
        XArgs<T> a = make_xargs<T>(p.d, g, 1, nout, lp ? lp->n2max : n2max1, dk(0), ct);
        a.amp = p.amp();
        GRIDSPT_CHECK(p.xfused(lp ? XM_LIN_ORDER1 : XM_ORDER1, a));
        // theta_1 = delta_1: the z inverse stores the same rows twice
        T* t1 = (theta[0] && theta[0] != delta[0]) ? static_cast<T*>(theta[0]) : nullptr;
        if (nmax == 1) {
            T* out[1] = {static_cast<T*>(delta[0])};
            return p.to_real(1, out, t1);
        }
        GRIDSPT_CHECK(p.yinv(2));     // delta_1, u_x
        GRIDSPT_CHECK(p.yinv_yz(2));  // phi -> u_y, phi
        chain = ChainArgs<T>{nullptr, 0, {0, 1, 2, 3}, {static_cast<T*>(delta[0]), nullptr, nullptr, nullptr}, t1};
    }
    // orders n >= 2.  The z inverse of delta_{n-1}, u_{n-1} runs inside order n's
    // product pass (k_zchain); u_m is stored only while a later product pass
    // reads it from HBM (m < nmax - 1).
    for (int n = 2; n <= nmax; ++n) {
        tag.set(n);
        if (n - 1 < nmax - 1)
            for (int j = 0; j < 3; ++j) chain.out[1 + j] = p.U(n - 1, j);
        ProductInputs<T> pin{};
        for (int m = 1; m < n - 1; ++m) {
            pin.d[m - 1] = static_cast<const T*>(delta[m - 1]);
            for (int j = 0; j < 3; ++j) pin.u[m - 1][j] = p.U(m, j);
        }
        GRIDSPT_CHECK(p.zchain(n, pin, chain));
        GRIDSPT_CHECK(p.yfwd_products());
        const int nout = n < nmax ? 4 : 2;  // delta_n, theta_n (, u_x, phi)
        XArgs<T> a = make_xargs<T>(p.d, g, n, nout, n2max2, dk(n - 1), tk(n - 1));
        GRIDSPT_CHECK(p.xfused(XM_ORDER, a));
        if (n == nmax) {
            T* out[2] = {static_cast<T*>(delta[n - 1]), static_cast<T*>(theta[n - 1])};
            return p.to_real(2, out);
        }
        // S4 fields delta_n, theta_n, u_x, u_y, phi: theta_n to real space now, the
        // rest in the next order's chained pass
        GRIDSPT_CHECK(p.yinv(3));     // delta_n, theta_n, u_x
        GRIDSPT_CHECK(p.yinv_yz(3));  // phi -> u_y, phi
        ZJobs<T> zj{};
        zj.f[0] = 1;
        zj.out[0] = static_cast<T*>(theta[n - 1]);
        GRIDSPT_CHECK(p.zinv(zj, 1));
        chain = ChainArgs<T>{nullptr, 0, {0, 2, 3, 4}, {static_cast<T*>(delta[n - 1]), nullptr, nullptr, nullptr},
                             nullptr};
    }
    return GRIDSPT_OK;
}

// Shell-filtered inverse transforms of the bispectrum estimator, five slots
// per pass sequence.  Slots go in order of their outer radius, and each
// group of five is transformed on the smallest cube holding its shells
// (Kc = floor(sqrt(largest n^2 in them))), so inner shells cost less.
template <typename T, int N>
int run_shells(gridspt_ctx* c, const gridspt_grid* g, int nslots, const void* const* cubes, const int64_t* lo,
               const int64_t* hi, void* const* out, void* work, const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, 1, tu, b);
    GRIDSPT_CHECK(p.twiddles());
    const CubeDims full = p.cd;
    std::vector<int> order(nslots);
    for (int i = 0; i < nslots; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return hi[x] < hi[y]; });
    for (int s0 = 0; s0 < nslots; s0 += 5) {
        const int nb = std::min(5, nslots - s0);
        ShellSlots<T> sh{};
        sh.src = full;
        T* outs[5];
        int64_t top = 1;
        for (int i = 0; i < nb; ++i) {
            const int k = order[s0 + i];
            sh.cube[i] = static_cast<const cpx<T>*>(cubes[k]);
            sh.lo[i] = lo[k];
            sh.hi[i] = hi[k];
            outs[i] = static_cast<T*>(out[k]);
            top = std::max(top, hi[k] - 1);
        }
        const int kc = (int)std::min<int64_t>(std::max<int64_t>(isqrt64(top), 1), full.Kc);
        p.cd = {kc, kc + 1, 2 * kc + 1};
        GRIDSPT_CHECK(p.xshell(sh, nb));
        GRIDSPT_CHECK(p.to_real(nb, outs));
    }
    p.cd = full;
    return GRIDSPT_OK;
}

// Gaussian smoothing of cube spectra, cumulative or one by one (nfields <= 5)
template <typename T, int N>
int run_smooth(gridspt_ctx* c, const gridspt_grid* g, int nfields, const void* const* fields_k, const double* coef,
               int cumulative, double radius, void* const* out, void* work, const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, 1, tu, b);
    GRIDSPT_CHECK(p.twiddles());
    SmoothArgs<T> sa{};
    for (int i = 0; i < nfields; ++i) {
        sa.cube[i] = static_cast<const cpx<T>*>(fields_k[i]);
        sa.coef[i] = coef[i];
    }
    sa.nin = nfields;
    sa.cumulative = cumulative ? 1 : 0;
    sa.kF = 2.0 * M_PI / g->box;
    sa.radius = radius;
    GRIDSPT_CHECK(p.xsmooth(sa));
    T* outs[5];
    for (int i = 0; i < nfields; ++i) outs[i] = static_cast<T*>(out[i]);
    return p.to_real(nfields, outs);
}

// Orders 1..nmax with the printed sources of Eq. 10 (the P-form): after each
// order the 15 derived fields of Eq. 15/16 are made from its spectra; the
// sources of order n are formed pointwise from the 17 fields of every earlier
// order, transformed two per complex transform, and combined with the matrix
// of Eq. 10 in the fused x pass.
template <typename T, int N>
int run_orders_pform(gridspt_ctx* c, const gridspt_grid* g, int nmax, int64_t n2max1, int64_t n2max2,
                     const void* delta1, void* const* delta, void* const* theta, void* const* delta_k,
                     void* const* theta_k, void* work, const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, 1, tu, b);
    const PFormLayout pl = pform_layout(p.d, nmax);
    char* wb = static_cast<char*>(work);
    T* base = reinterpret_cast<T*>(wb + pl.fields);
    const size_t nc = (size_t)p.d.ncell();
    auto derived = [&](int m, int q) { return base + ((size_t)(m - 1) * 15 + q) * nc; };  // q = 0..14
    T* sdel = base + (size_t)(nmax - 1) * 15 * nc;
    T* sthe = sdel + nc;
    cpx<T>* wcube_d = reinterpret_cast<cpx<T>*>(wb + pl.cubes);
    cpx<T>* wcube_t = wcube_d + p.d.cube();
    auto dk = [&](int i) { return (delta_k && delta_k[i]) ? (cpx<T>*)delta_k[i] : wcube_d; };
    auto tk = [&](int i) {
        const bool own = theta_k && theta_k[i] && !(delta_k && theta_k[i] == delta_k[i]);
        return own ? (cpx<T>*)theta_k[i] : wcube_t;
    };
    const double kF = 2.0 * M_PI / g->box;
    OrderTag tag(c, 1);  // per-order timing: order 1, then each order n with its derived fields
    GRIDSPT_CHECK(p.twiddles());
    // the derived fields of order m from its spectra
    auto make_derived = [&](int m, const cpx<T>* cd_, const cpx<T>* ct_) -> int {
        RegenArgs<T> r{};
        r.cube_d = cd_;
        r.cube_t = ct_;
        r.kF = kF;
        for (int ch = 0; ch < 3; ++ch) {
            GRIDSPT_CHECK(p.xderived(r, ch));
            T* out[5];
            for (int i = 0; i < 5; ++i) out[i] = derived(m, 5 * ch + i);
            GRIDSPT_CHECK(p.to_real(5, out));
        }
        return GRIDSPT_OK;
    };
    // order 1: delta_1 = theta_1 = W1 F[delta1_in]
    GRIDSPT_CHECK(p.zfwd_single(static_cast<const T*>(delta1), false, 0, 0));
    GRIDSPT_CHECK(p.yfwd(1));
    {
        cpx<T>* c1 = dk(0);
        XArgs<T> a = make_xargs<T>(p.d, g, 1, 1, n2max1, c1, nullptr);
        GRIDSPT_CHECK(p.xfused(XM_ORDER1, a));
        T* out[1] = {static_cast<T*>(delta[0])};
        GRIDSPT_CHECK(p.to_real(1, out, (theta[0] && theta[0] != delta[0]) ? static_cast<T*>(theta[0]) : nullptr));
        if (theta_k && theta_k[0] && theta_k[0] != (void*)c1)
            GRIDSPT_CHECK(launch(c, KD_COPY, 4.0 * p.d.cube() * p.d.real_bytes, dim3(512), dim3(256), 0, k_copy<T>,
                                 (const T*)c1, (T*)theta_k[0], (size_t)(2 * p.d.cube()), (size_t)0));
        if (nmax > 1) GRIDSPT_CHECK(make_derived(1, c1, c1));
    }
    for (int n = 2; n <= nmax; ++n) {
        tag.set(n);
        PFormProducts<T> pp{};
        for (int m = 1; m < n; ++m) {
            pp.f[m - 1][0] = static_cast<const T*>(delta[m - 1]);
            pp.f[m - 1][1] = static_cast<const T*>(m == 1 ? delta[0] : theta[m - 1]);
            for (int q = 0; q < 15; ++q) pp.f[m - 1][2 + q] = derived(m, q);
        }
        pp.sd = sdel;
        pp.st = sthe;
        pp.ncell = nc;
        const double bytes = (double)nc * p.d.real_bytes * (17.0 * (n - 1) + 2.0);
        auto go = [&](auto kern) {
            return launch(c, KD_PFORM_PRODUCTS, bytes, dim3(4096), dim3(256), 0, kern, pp);
        };
        switch (n) {
            case 2: GRIDSPT_CHECK(go(k_pform_products<T, 2>)); break;
            case 3: GRIDSPT_CHECK(go(k_pform_products<T, 3>)); break;
            case 4: GRIDSPT_CHECK(go(k_pform_products<T, 4>)); break;
            case 5: GRIDSPT_CHECK(go(k_pform_products<T, 5>)); break;
            default: return GRIDSPT_EINVAL;
        }
        GRIDSPT_CHECK(p.zfwd_pair(sdel, sthe));
        GRIDSPT_CHECK(p.yfwd(2));
        cpx<T>* cdn = dk(n - 1);
        cpx<T>* ctn = tk(n - 1);
        XArgs<T> a = make_xargs<T>(p.d, g, n, 2, n2max2, cdn, ctn);
        GRIDSPT_CHECK(p.xfused(XM_PFORM, a));
        T* out[2] = {static_cast<T*>(delta[n - 1]), static_cast<T*>(theta[n - 1])};
        GRIDSPT_CHECK(p.to_real(2, out));
        if (n < nmax) GRIDSPT_CHECK(make_derived(n, cdn, ctn));
    }
    return GRIDSPT_OK;
}

// Reverse mode of noise -> delta_1 .. delta_nmax (linear field from given
// noise, then the D-form orders), for an objective of the delta_n only:
// regenerate delta_m, u_m (m < nmax) from the stored spectra, then run the
// orders backwards (the transposed order step, then the transposed products),
// then the transposed linear field.
template <typename T, int N>
int run_adjoint(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int nmax, int64_t n2max2,
                const void* const* delta_k, const void* const* theta_k, const void* const* gdelta, void* gnoise,
                void* work, const Tuning& tu, Batch b) {
    Pipe<T, N> p(c, g, work, 1, tu, b);
    const AdjLayout al = adjoint_layout(p.d, nmax);
    T* base = reinterpret_cast<T*>(static_cast<char*>(work) + al.fields);
    const size_t nc = (size_t)p.d.ncell();
    auto fld = [&](int64_t i) { return base + (size_t)i * nc; };
    // field map: D(m) 0..nmax-2, U(m, j), GD(m), GU(m, j), GV(q)
    const int nm = nmax - 1;
    auto D = [&](int m) { return fld(m - 1); };
    auto U = [&](int m, int j) { return fld(nm + 3 * (m - 1) + j); };
    auto GD = [&](int m) { return fld(4 * nm + (m - 1)); };
    auto GU = [&](int m, int j) { return fld(5 * nm + 3 * (m - 1) + j); };
    auto GV = [&](int q) { return fld(8 * nm + q); };
    GRIDSPT_CHECK(p.twiddles());
    const double kF = 2.0 * M_PI / g->box;
    for (int m = 1; m <= nm; ++m) {
        RegenArgs<T> r{};
        r.cube_d = static_cast<const cpx<T>*>(delta_k[m - 1]);
        r.cube_t = static_cast<const cpx<T>*>((m == 1 || !theta_k[m - 1]) ? delta_k[m - 1] : theta_k[m - 1]);
        r.kF = kF;
        GRIDSPT_CHECK(p.xregen(r));
        T* out[4] = {D(m), U(m, 0), U(m, 1), U(m, 2)};
        GRIDSPT_CHECK(p.to_real(4, out));
    }
    // forward transform of the objective gradient of order n (and g u_n)
    auto fwd = [&](int n) -> int {
        if (n == nmax) {
            GRIDSPT_CHECK(p.zfwd_single(static_cast<const T*>(gdelta[n - 1]), false, 0, 0));
            return p.yfwd(1);
        }
        const T* f[4] = {GD(n), GU(n, 0), GU(n, 1), GU(n, 2)};
        GRIDSPT_CHECK(p.zfwd_four(f));
        return p.yfwd(4);
    };
    for (int n = nmax; n >= 2; --n) {
        GRIDSPT_CHECK(fwd(n));
        XArgs<T> a = make_xargs<T>(p.d, g, n, 4, n2max2, nullptr, nullptr);
        a.nin = n == nmax ? 1 : 4;
        GRIDSPT_CHECK(p.xfused(XM_ADJ, a));
        T* out[4] = {GV(0), GV(1), GV(2), GV(3)};
        GRIDSPT_CHECK(p.to_real(4, out));
        AdjProducts<T> ap{};
        for (int q = 0; q < 4; ++q) ap.gv[q] = GV(q);
        for (int i = 1; i < n; ++i) {
            ap.d[i - 1] = D(i);
            ap.gd_in[i - 1] = static_cast<const T*>(gdelta[i - 1]);
            ap.gd[i - 1] = GD(i);
            for (int j = 0; j < 3; ++j) {
                ap.u[i - 1][j] = U(i, j);
                ap.gu[i - 1][j] = GU(i, j);
            }
        }
        ap.ncell = nc;
        const double bytes = (double)nc * p.d.real_bytes * (4.0 + 4.0 * (n - 1) + 8.0 * (n - 1) - (n == nmax ? 3.0 * (n - 1) : 0.0));
        const int first = n == nmax ? 1 : 0;
        auto go = [&](auto kern) {
            return launch(c, KD_ADJ_PRODUCTS, bytes, dim3(4096), dim3(256), 0, kern, ap, first);
        };
        switch (n) {
            case 2: GRIDSPT_CHECK(go(k_adj_products<T, 2>)); break;
            case 3: GRIDSPT_CHECK(go(k_adj_products<T, 3>)); break;
            case 4: GRIDSPT_CHECK(go(k_adj_products<T, 4>)); break;
            case 5: GRIDSPT_CHECK(go(k_adj_products<T, 5>)); break;
            default: return GRIDSPT_EINVAL;
        }
    }
    GRIDSPT_CHECK(fwd(1));
    GRIDSPT_CHECK(p.amp_table(g, lp));
    XArgs<T> a = make_xargs<T>(p.d, g, 1, 1, lp->n2max, nullptr, nullptr);
    a.nin = nmax == 1 ? 1 : 4;
    a.amp = p.amp();
    GRIDSPT_CHECK(p.xfused(XM_ADJ1, a));
    T* out[1] = {static_cast<T*>(gnoise)};
    return p.to_real(1, out);
}

}  // namespace gridspt

// explicit instantiations for one grid size, both precisions
#define GRIDSPT_INSTANTIATE_T(T, N)                                                                                \
    template int gridspt::run_linear_field<T, N>(gridspt_ctx*, const gridspt_grid*, const gridspt_linpk*,         \
                                                 const void*, void*, void*, void*, const gridspt::Tuning&,         \
                                                 gridspt::Batch);                                                  \
    template int gridspt::run_smooth<T, N>(gridspt_ctx*, const gridspt_grid*, int, const void* const*,            \
                                           const double*, int, double, void* const*, void*,                      \
                                           const gridspt::Tuning&, gridspt::Batch);                              \
    template int gridspt::run_orders_pform<T, N>(gridspt_ctx*, const gridspt_grid*, int, int64_t, int64_t,       \
                                                 const void*, void* const*, void* const*, void* const*,            \
                                                 void* const*, void*, const gridspt::Tuning&, gridspt::Batch);     \
    template int gridspt::run_adjoint<T, N>(gridspt_ctx*, const gridspt_grid*, const gridspt_linpk*, int, int64_t, \
                                            const void* const*, const void* const*, const void* const*, void*,     \
                                            void*, const gridspt::Tuning&, gridspt::Batch);                        \
    template int gridspt::run_forward<T, N>(gridspt_ctx*, const gridspt_grid*, int64_t, const void*, void*, void*, \
                                            const gridspt::Tuning&, gridspt::Batch);                               \
    template int gridspt::run_orders<T, N>(gridspt_ctx*, const gridspt_grid*, const gridspt_linpk*, int, int64_t,  \
                                           int64_t, const void*,                                                   \
                                           void* const*, void* const*, void* const*, void* const*, void*,          \
                                           const gridspt::Tuning&, gridspt::Batch);                                \
    template int gridspt::run_shells<T, N>(gridspt_ctx*, const gridspt_grid*, int, const void* const*,             \
                                           const int64_t*, const int64_t*, void* const*, void*,                    \
                                           const gridspt::Tuning&, gridspt::Batch);
#define GRIDSPT_INSTANTIATE(N)        \
    GRIDSPT_INSTANTIATE_T(float, N)   \
    GRIDSPT_INSTANTIATE_T(double, N)

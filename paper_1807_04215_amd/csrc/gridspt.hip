// libgridspt: C ABI (include/gridspt.h) over the gfx950 kernels in
// passes.hpp and estimators.hpp.  Host code validates arguments, lays out the
// caller's workspace, and enqueues the pass sequences (pipeline.hpp,
// instantiated per grid size under sizes/) on the context's stream; batches
// of realisations are captured into one HIP graph.
#include <array>
#include <climits>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <utility>

#include "runtime.hpp"

using namespace gridspt;

#define CHECK GRIDSPT_CHECK

namespace {

// ---------------------------------------------------------------------------
// cross spectra: enqueue for one call or a realisation batch
// ---------------------------------------------------------------------------

// per-wave LDS accumulators: nbins * (pairs + 2) doubles, at most 1792 (56 KB per block)
int power_chunk(int nbins) { return std::max(1, std::min(kPowerPairsPerLaunch, 1792 / nbins - 2)); }
// Block partials are sized for power_blocks (at most 1024 blocks); a launch
// uses no more blocks than the GPU holds at once (power_launch_blocks), so that
// every wavefront's share of half-rows runs in one round.
int power_blocks(const Dims& d) {
    const int64_t halves = 2 * d.Kz * d.Ky;
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (halves + kPowerWaves - 1) / kPowerWaves));
}
template <typename Kern>
int power_launch_blocks(const Dims& d, Kern kern, size_t shm, unsigned nz) {
    const int most = power_blocks(d);
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
        hipSuccess || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * kPowerWaves, shm) != hipSuccess)
        return most;
    const int64_t resident = (int64_t)std::max(cus, 1) * std::max(per_cu, 1) / std::max(nz, 1u);
    return (int)std::max<int64_t>(1, std::min<int64_t>(most, resident));
}
// Columns of a launch's partial sums: at most power_chunk products per mode (the
// requested pairs of the chunk, or, from up to five fields, every pair i <= j of
// them, which that mode takes only when they fit the chunk), then the mode count
// and the sum of |k|.  Sized for the chunk whatever npairs is: a single pair of
// two fields still accumulates all three of their pairs.
int power_cols(int nbins) { return power_chunk(nbins) + 2; }
int64_t power_ws(const Dims& d, int nbins) {
    const int q = power_cols(nbins);
    // block partials and the reduced sums
    return align_up((int64_t)power_blocks(d) * nbins * q * 8) + align_up((int64_t)nbins * q * 8);
}

// Modes of the cube with e0 <= |n|^2 < e1: what the cross-spectrum kernel
// reads of each field (its algorithmic traffic, for the launch records).
int64_t modes_in_shells(const Dims& d, int64_t e0, int64_t e1) {
    static std::mutex mu;
    static std::array<int64_t, 4> last{-1, -1, -1, -1};
    std::lock_guard<std::mutex> lock(mu);
    if (last[0] == d.Kc && last[1] == e0 && last[2] == e1) return last[3];
    const int64_t kc = d.Kc, kc1 = kc + 1;
    // the number of a in [0, Kc] with a^2 < x
    auto below = [&](int64_t x) -> int64_t {
        if (x <= 0) return 0;
        if (x > kc * kc) return kc1;
        int64_t r = (int64_t)std::sqrt((double)x);
        while (r * r >= x) --r;
        while ((r + 1) * (r + 1) < x) ++r;
        return r + 1;
    };
    int64_t n = 0;
    for (int64_t kz = 0; kz <= kc; ++kz)
        for (int64_t ky = 0; ky <= kc; ++ky) {
            const int64_t c2 = ky * ky + kz * kz;
            // kx in [-Kc, Kc]: a = 0 once, a >= 1 twice
            const int64_t lo = below(e0 - c2), hi = below(e1 - c2);
            const int64_t in0 = hi > 0 && lo == 0 ? 1 : 0;  // a = 0 inside
            const int64_t row = std::max<int64_t>(0, hi - lo) * 2 - in0;
            n += ky == 0 ? row : 2 * row;
        }
    last = {d.Kc, e0, e1, n};
    return n;
}

int check_power_args(int nfields, int npairs, const int32_t* pairs, int nbins, const int64_t* edge_n2) {
    if (!pairs || !edge_n2) return GRIDSPT_EINVAL;
    if (nfields < 1 || nfields > kMaxFields || npairs < 1 || npairs > kMaxPairs || nbins < 1 || nbins > kMaxBins)
        return GRIDSPT_EINVAL;
    for (int i = 0; i < 2 * npairs; ++i)
        if (pairs[i] < 0 || pairs[i] >= nfields) return GRIDSPT_EINVAL;
    if (edge_n2[0] < 1) return GRIDSPT_EINVAL;
    for (int b = 0; b < nbins; ++b)
        if (edge_n2[b + 1] < edge_n2[b]) return GRIDSPT_EINVAL;
    return GRIDSPT_OK;
}

int power_enqueue(gridspt_ctx* c, const gridspt_grid* g, const void* const* fields_k, int npairs,
                  const int32_t* pairs, int nbins, const int64_t* edge_n2, double* pk, double* kmean, double* nmodes,
                  void* work, Batch bt) {
    const Dims d = dims_of(g);
    const int nblk = power_blocks(d);
    const int chunk = power_chunk(nbins);
    const unsigned nz = (unsigned)bt.nreal;
    auto go = [&](auto tag) -> int {
        using T = typename decltype(tag)::type;
        double* partial = static_cast<double*>(work);
        const int64_t part_bytes = align_up((int64_t)nblk * nbins * power_cols(nbins) * 8);
        double* sums = reinterpret_cast<double*>(static_cast<char*>(work) + part_bytes);
        BinEdges be{};
        for (int b = 0; b <= nbins; ++b) be.e[b] = edge_n2[b];
        be.nbins = nbins;
        // modes read per field (only counted for the launch records)
        const int64_t nread = c->profile ? modes_in_shells(d, edge_n2[0], edge_n2[nbins]) : 0;
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
            PairCols pc{};
            for (int q = 0; q < np; ++q) {
                a.pa[q] = slot_of[pairs[2 * (p0 + q)]];
                a.pb[q] = slot_of[pairs[2 * (p0 + q) + 1]];
                pc.col[q] = q;
            }
            // all pairs of up to five fields: each field loaded once per mode
            const int tri = nf <= 5 && nf * (nf + 1) / 2 <= chunk ? nf : 0;
            int nacc = np;  // accumulated products per mode
            if (tri) {
                nacc = tri * (tri + 1) / 2;
                for (int q = 0; q < np; ++q)
                    pc.col[q] = tri_index(std::min(a.pa[q], a.pb[q]), std::max(a.pa[q], a.pb[q]), tri);
            }
            a.nf = nf;
            a.npairs = nacc;
            a.nbins = nbins;
            a.kF = 2.0 * M_PI / g->box;
            a.partial = partial;
            const int nq = nacc + 2;
            const CubeDims cdims{(int)d.Kc, (int)d.Kz, (int)d.Ky};
            const dim3 pblock(64 * kPowerWaves);
            const double pbytes = (double)nz * nf * nread * d.cpx_bytes;
            int used = nblk;  // blocks of this launch (<= nblk, the partials' capacity)
            auto go = [&](auto kern, size_t stage_bytes) {
                const size_t shm = (size_t)kPowerWaves * power_wave_bytes(nbins, nq, stage_bytes);
                used = power_launch_blocks(d, kern, shm, nz);
                return launch(c, KD_POWER, pbytes, dim3(used, 1, nz), pblock, shm, kern, a, be, cdims, bt.zs);
            };
            switch (tri) {
                case 1: CHECK(go(k_power_partial<T, 1>, power_stage_bytes<T, 1>())); break;
                case 2: CHECK(go(k_power_partial<T, 2>, power_stage_bytes<T, 2>())); break;
                case 3: CHECK(go(k_power_partial<T, 3>, power_stage_bytes<T, 3>())); break;
                case 4: CHECK(go(k_power_partial<T, 4>, power_stage_bytes<T, 4>())); break;
                case 5: CHECK(go(k_power_partial<T, 5>, power_stage_bytes<T, 5>())); break;
                default: CHECK(go(k_power_partial<T, 0>, power_stage_bytes<T, 0>()));
            }
            CHECK(launch(c, KD_POWER_FINAL, (double)nz * used * nbins * nq * 8.0, dim3(nbins * nq, 1, nz),
                         dim3(kReduceThreads), 0, k_power_reduce, (const double*)partial, used, sums, bt.zs));
            CHECK(launch(c, KD_POWER_FINAL, 0.0, dim3((nbins + 63) / 64, 1, nz), dim3(64), 0, k_power_final,
                         (const double*)sums, nbins, nq, np, pc, g->box * g->box * g->box, pk + (size_t)p0 * nbins,
                         nbins, p0 == 0 ? kmean : nullptr, p0 == 0 ? nmodes : nullptr, bt.zs));
        }
        return GRIDSPT_OK;
    };
    if (g->dtype == GRIDSPT_F64) return go(tag_t<double>{});
    return go(tag_t<float>{});
}

// ---------------------------------------------------------------------------
// Scratch of gridspt_power_static, for callers that cannot allocate: one array
// per GPU, held for the life of the process.  Its largest use: 1024 blocks x
// 1792 partial sums (nbins power_cols(nbins) <= 1792 for every nbins <= 256)
// of 8 bytes, and the reduced sums: about 14.7 MB.  In host code
// `scratch` only names the symbol; the device address comes from
// hipGetSymbolAddress, once per device.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticScratchBytes = 16ll << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`.
int static_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return GRIDSPT_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return GRIDSPT_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GRIDSPT_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GRIDSPT_OK;
}

// ---------------------------------------------------------------------------
// bispectrum: slots (field or indicator restricted to a shell) are made in
// chunks of triangles, at most `cap` distinct slots per chunk, and consumed
// by the triple sums of that chunk's terms and triangles
// ---------------------------------------------------------------------------

struct BispChunk {
    std::vector<std::pair<int, int>> slots;  // (field, or -1 for the indicator; bin)
    std::vector<std::array<int, 4>> titems;  // slots a, b, c; term index
    std::vector<std::array<int, 4>> jitems;  // slots a, b, c; triangle index
};
struct BispPlan {
    std::vector<BispChunk> chunks;
    int max_slots = 0;
    std::vector<int> rep;  // term -> the term whose sum it takes (same factors in another order)
};

constexpr int kTripleBlocks = 1024;

int check_bisp_args(int nfields, int ntri, const int32_t* tri_bins, int nterms, const int32_t* terms, int nbins,
                    const int64_t* edge_n2) {
    if (!tri_bins || !terms || !edge_n2) return GRIDSPT_EINVAL;
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
    return GRIDSPT_OK;
}

// terms and triangles are assumed validated; with_terms / with_j select the
// term sums and the triangle counts (indicator slots) the plan makes
BispPlan bisp_make_plan(int ntri, const int32_t* tri_bins, int nterms, const int32_t* terms, int cap,
                        bool with_terms = true, bool with_j = true) {
    BispPlan bp;
    // a triple sum does not depend on the order of its three (field, shell)
    // factors: terms with the same factors share one sum
    bp.rep.resize(nterms);
    {
        std::map<std::array<std::pair<int, int>, 3>, int> seen;
        for (int u = 0; u < nterms; ++u) {
            const int* b = tri_bins + 3 * terms[4 * u + 3];
            std::array<std::pair<int, int>, 3> key = {std::make_pair(terms[4 * u], b[0]),
                                                      std::make_pair(terms[4 * u + 1], b[1]),
                                                      std::make_pair(terms[4 * u + 2], b[2])};
            std::sort(key.begin(), key.end());
            auto it = seen.find(key);
            bp.rep[u] = it == seen.end() ? (seen[key] = u) : it->second;
        }
    }
    std::vector<std::vector<int>> terms_of(ntri);
    for (int u = 0; u < nterms; ++u)
        if (bp.rep[u] == u) terms_of[terms[4 * u + 3]].push_back(u);
    std::map<std::pair<int, int>, int> index;
    std::vector<int> tris;
    auto flush = [&]() {
        if (tris.empty()) return;
        BispChunk ch;
        ch.slots.resize(index.size());
        for (auto& kv : index) ch.slots[kv.second] = kv.first;
        for (int t : tris) {
            const int* b = tri_bins + 3 * t;
            if (with_j) ch.jitems.push_back({index[{-1, b[0]}], index[{-1, b[1]}], index[{-1, b[2]}], t});
            if (with_terms)
            for (int u : terms_of[t]) {
                const int* f = terms + 4 * u;
                ch.titems.push_back({index[{f[0], b[0]}], index[{f[1], b[1]}], index[{f[2], b[2]}], u});
            }
        }
        bp.max_slots = std::max(bp.max_slots, (int)ch.slots.size());
        bp.chunks.push_back(std::move(ch));
        index.clear();
        tris.clear();
    };
    for (int t = 0; t < ntri; ++t) {
        std::set<std::pair<int, int>> need;
        const int* b = tri_bins + 3 * t;
        if (with_j)
            for (int i = 0; i < 3; ++i) need.insert({-1, b[i]});
        if (with_terms)
            for (int u : terms_of[t])
                for (int i = 0; i < 3; ++i) need.insert({terms[4 * u + i], b[i]});
        if (need.empty()) continue;
        int fresh = 0;
        for (auto& k : need) fresh += index.count(k) ? 0 : 1;
        if (!tris.empty() && (int)index.size() + fresh > cap) flush();
        for (auto& k : need)
            if (!index.count(k)) {
                const int s = (int)index.size();
                index[k] = s;
            }
        tris.push_back(t);
    }
    flush();
    return bp;
}

// scratch of the estimator: sums (nterms term sums, then ntri triangle sums) |
// triple partials | slots.  The first two do not depend on the precision of
// the slots, so the triangle counts (made in FP64) and the term sums (in the
// grid's precision) share them.
struct BispLayout {
    int64_t sums, partial, slots, end;
};
BispLayout bisp_layout(const Dims& d, int max_slots, int nterms, int ntri) {
    BispLayout b;
    b.sums = 0;
    b.partial = align_up(b.sums + (int64_t)(nterms + ntri) * 8);
    b.slots = align_up(b.partial + (int64_t)kTripleBlocks * 8 * 8);
    b.end = align_up(b.slots + (int64_t)max_slots * d.ncell() * d.real_bytes);
    return b;
}

// The grid on which the triangle counts are made: the same grid in FP64, so
// that N_123 comes out as an exact integer whatever the fields' precision.
gridspt_grid count_grid(const gridspt_grid* g) {
    gridspt_grid c = *g;
    c.dtype = GRIDSPT_F64;
    c.flags = 0;
    return c;
}

// Exact closure (Eq. 22-23 ask for k1 + k2 + k3 = 0; the estimator's sum over
// cells closes modulo N): every component of k1 + k2 + k3 lies within the sum
// of the shells' outer radii, so the two agree when that sum is below N.
int check_closure(const gridspt_grid* g, int ntri, const int32_t* tri_bins, const int64_t* edge_n2) {
    auto radius = [&](int b) { return edge_n2[b + 1] > edge_n2[b] ? isqrt64(edge_n2[b + 1] - 1) : 0; };
    for (int t = 0; t < ntri; ++t) {
        const int32_t* b = tri_bins + 3 * t;
        if (radius(b[0]) + radius(b[1]) + radius(b[2]) >= g->n) return GRIDSPT_EINVAL;
    }
    return GRIDSPT_OK;
}

// pipe: a pipeline workspace (layout_of(d, 1) or larger); est: the
// estimator's own region (bisp_layout).  The plan's slots are made on grid g
// (count_grid(g) for the triangle counts).
// final: also form bk and ntriangles from the sums; jzs: byte stride of the
// triangle counts between realisations (0: realisation 0's, made once)
int bisp_enqueue(gridspt_ctx* c, const gridspt_grid* g, const void* const* fields_k, const BispPlan& bp, int ntri,
                 int nterms, const int32_t* terms, const int64_t* edge_n2, double* bk, double* ntriangles, void* pipe,
                 void* est, const Tuning& tu, Batch bt, bool final = true, size_t jzs = SIZE_MAX) {
    if (jzs == SIZE_MAX) jzs = bt.zs;
    const Dims d = dims_of(g);
    const BispLayout bl = bisp_layout(d, bp.max_slots, nterms, ntri);
    char* base = static_cast<char*>(est);
    double* partial = reinterpret_cast<double*>(base + bl.partial);
    double* sums = reinterpret_cast<double*>(base + bl.sums);
    const unsigned nz = (unsigned)bt.nreal;
    for (const BispChunk& ch : bp.chunks) {
        const int ns = (int)ch.slots.size();
        std::vector<const void*> cubes(ns);
        std::vector<int64_t> lo(ns), hi(ns);
        std::vector<void*> outs(ns);
        for (int i = 0; i < ns; ++i) {
            const auto& sl = ch.slots[i];
            cubes[i] = sl.first >= 0 ? fields_k[sl.first] : nullptr;
            lo[i] = edge_n2[sl.second];
            hi[i] = edge_n2[sl.second + 1];
            outs[i] = base + bl.slots + (int64_t)i * d.ncell() * d.real_bytes;
        }
        CHECK(dispatch(g, [&](auto tag, auto nc) -> int {
            using T = typename decltype(tag)::type;
            constexpr int N = decltype(nc)::value;
            return run_shells<T, N>(c, g, ns, cubes.data(), lo.data(), hi.data(), outs.data(), pipe, tu, bt);
        }));
        auto triple = [&](const std::vector<std::array<int, 4>>& items, double* dst) -> int {
            auto go = [&](auto tag) -> int {
                using T = typename decltype(tag)::type;
                for (size_t u0 = 0; u0 < items.size(); u0 += 8) {
                    TripleArgs<T> t{};
                    TripleDst td{};
                    t.nterms = (int)std::min<size_t>(8, items.size() - u0);
                    t.ncell = (size_t)d.ncell();
                    t.partial = partial;
                    for (int i = 0; i < t.nterms; ++i) {
                        t.a[i] = static_cast<const T*>(outs[items[u0 + i][0]]);
                        t.b[i] = static_cast<const T*>(outs[items[u0 + i][1]]);
                        t.c[i] = static_cast<const T*>(outs[items[u0 + i][2]]);
                        td.idx[i] = items[u0 + i][3];
                    }
                    // the kernel reads 16-byte vectors of cells
                    bool aligned = bt.zs % 16 == 0 && t.ncell % (16 / sizeof(T)) == 0;
                    for (int i = 0; i < t.nterms; ++i)
                        for (const T* q : {t.a[i], t.b[i], t.c[i]})
                            aligned = aligned && reinterpret_cast<uintptr_t>(q) % 16 == 0;
                    if (!aligned) return GRIDSPT_EALIGN;
                    int rc = GRIDSPT_OK;
                    static_for<8>([&](auto k) {
                        constexpr int NT = decltype(k)::value + 1;
                        if (NT == t.nterms)
                            rc = launch(c, KD_TRIPLE, (double)nz * 3.0 * NT * d.ncell() * d.real_bytes,
                                        dim3(kTripleBlocks, 1, nz), dim3(kTripleThreads), 0,
                                        k_triple_partial<T, NT>, t, bt.zs);
                    });
                    CHECK(rc);
                    CHECK(launch(c, KD_TRIPLE_FINAL, (double)nz * kTripleBlocks * 8.0 * 8.0, dim3(1, 1, nz),
                                 dim3(kReduceThreads), 0, k_triple_final, (const double*)partial, kTripleBlocks,
                                 t.nterms, td, dst, bt.zs));
                }
                return GRIDSPT_OK;
            };
            if (g->dtype == GRIDSPT_F64) return go(tag_t<double>{});
            return go(tag_t<float>{});
        };
        CHECK(triple(ch.titems, sums));
        CHECK(triple(ch.jitems, sums + nterms));
    }
    if (!final) return GRIDSPT_OK;
    // bk = L^6 T / J per term, the term -> triangle map in the argument buffer
    const double vol2 = std::pow(g->box, 6);
    const double invN3 = 1.0 / (double)d.ncell();
    for (int u0 = 0; u0 < std::max(nterms, ntri); u0 += 64) {
        TriMap m{};
        const int nu = std::max(0, std::min(64, nterms - u0));
        const int nt = std::max(0, std::min(64, ntri - u0));
        for (int i = 0; i < nu; ++i) {
            m.tri[i] = terms[4 * (u0 + i) + 3];
            m.rep[i] = bp.rep[u0 + i];
        }
        CHECK(launch(c, KD_BISP_FINAL, 0.0, dim3(1, 1, nz), dim3(64), 0, k_bisp_final, (const double*)sums,
                     (const double*)(sums + nterms), m, u0, nu, nt, vol2, invN3, bk, ntriangles, bt.zs, jzs));
    }
    return GRIDSPT_OK;
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
        case GRIDSPT_ENONFINITE: return "an input field holds a NaN or an infinity";
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
    for (int i = 0; i <= gridspt_ctx::kMaxOrderTag; ++i) c->order_ms[i] = c->order_bytes[i] = 0.0;
    for (auto& r : c->recs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) return GRIDSPT_EHIP;
        tot_ms[r.kind] += t;
        tot_b[r.kind] += r.bytes;
        cnt[r.kind] += 1;
        const int o = std::min(std::max(r.order, 0), gridspt_ctx::kMaxOrderTag);
        c->order_ms[o] += t;
        c->order_bytes[o] += r.bytes;
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

int gridspt_profile_orders(const gridspt_ctx* c, int32_t max, double* ms, double* bytes) {
    if (!c || max < 0) return GRIDSPT_EINVAL;
    int top = 0;
    for (int i = 0; i <= gridspt_ctx::kMaxOrderTag; ++i) {
        if (c->order_ms[i] > 0.0 || c->order_bytes[i] > 0.0) top = i;
        if (i < max) {
            if (ms) ms[i] = c->order_ms[i];
            if (bytes) bytes[i] = c->order_bytes[i];
        }
    }
    return top;
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

int64_t gridspt_workspace_bytes(const gridspt_grid* g, int32_t nmax, uint32_t flags) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    if (flags & ~(uint32_t)GRIDSPT_CHECK_FINITE) return GRIDSPT_EINVAL;
    return layout_of(dims_of(g), nmax).end;  // the check's flag word is part of every layout
}

// The pipeline workspace of the entry points below (their grid flags are checked by check_grid)
static int64_t pipe_bytes(const gridspt_grid* g, int nmax) { return layout_of(dims_of(g), nmax).end; }

// GRIDSPT_CHECK_FINITE: every real input field is scanned on the device, the
// flag word at the head of `work` comes back to the host, and a non-finite
// value ends the call with GRIDSPT_ENONFINITE before anything else is enqueued.
static int check_finite(gridspt_ctx* c, const gridspt_grid* g, const void* const* fields, int nf, void* work) {
    if (!(g->flags & GRIDSPT_CHECK_FINITE)) return GRIDSPT_OK;
    const Dims d = dims_of(g);
    uint32_t* flag = reinterpret_cast<uint32_t*>(static_cast<char*>(work) + layout_of(d, 1).chk);
    CHECK(launch(c, KD_COPY, 4.0, dim3(1), dim3(64), 0, k_clear_word, flag));
    for (int i = 0; i < nf; ++i) {
        const double bytes = (double)d.ncell() * d.real_bytes;
        if (g->dtype == GRIDSPT_F64)
            CHECK(launch(c, KD_COPY, bytes, dim3(2048), dim3(256), 0, k_nonfinite<double>,
                         static_cast<const double*>(fields[i]), (size_t)d.ncell(), flag));
        else
            CHECK(launch(c, KD_COPY, bytes, dim3(2048), dim3(256), 0, k_nonfinite<float>,
                         static_cast<const float*>(fields[i]), (size_t)d.ncell(), flag));
    }
    uint32_t h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return GRIDSPT_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return GRIDSPT_EHIP;
    return h ? GRIDSPT_ENONFINITE : GRIDSPT_OK;
}

static int check_linpk(const gridspt_grid* g, const gridspt_linpk* lp) {
    if (!lp) return GRIDSPT_EINVAL;
    CHECK(check_mask(g, lp->n2max));
    if (!(lp->amp >= 0.0) || !(lp->gamma > 0.0) || !std::isfinite(lp->ns) || !std::isfinite(lp->growth))
        return GRIDSPT_EINVAL;
    return GRIDSPT_OK;
}

int gridspt_linear_field(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, void* delta1,
                         void* delta1_k, void* work, int64_t work_bytes) {
    if (!c || !lp) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_linpk(g, lp));
    CHECK(check_ptr(delta1));
    if (delta1_k) CHECK(check_ptr(delta1_k));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < pipe_bytes(g, 1)) return GRIDSPT_EWORKSPACE;
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_linear_field<T, N>(c, g, lp, nullptr, delta1, delta1_k, work, tu, Batch{});
    });
}

int gridspt_noise_field(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, const void* noise,
                        void* delta1, void* delta1_k, void* work, int64_t work_bytes) {
    if (!c || !lp) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_linpk(g, lp));
    CHECK(check_ptr(noise));
    CHECK(check_ptr(delta1));
    if (delta1_k) CHECK(check_ptr(delta1_k));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < pipe_bytes(g, 1)) return GRIDSPT_EWORKSPACE;
    CHECK(check_finite(c, g, &noise, 1, work));
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_linear_field<T, N>(c, g, lp, noise, delta1, delta1_k, work, tu, Batch{});
    });
}

int64_t gridspt_adjoint_workspace_bytes(const gridspt_grid* g, int32_t nmax) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    return adjoint_layout(dims_of(g), nmax).end;
}

int gridspt_adjoint(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int32_t nmax, int64_t n2max2,
                    const void* const* delta_k, const void* const* theta_k, const void* const* gdelta, void* gnoise,
                    void* work, int64_t work_bytes) {
    if (!c || !lp || !gdelta) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    CHECK(check_linpk(g, lp));
    if (nmax > 1) {
        CHECK(check_mask(g, n2max2));
        if (!delta_k) return GRIDSPT_EINVAL;
        for (int m = 0; m < nmax - 1; ++m) {
            CHECK(check_ptr(delta_k[m]));
            if (m > 0) {
                if (!theta_k) return GRIDSPT_EINVAL;
                CHECK(check_ptr(theta_k[m]));
            }
        }
    }
    for (int m = 0; m < nmax; ++m) CHECK(check_ptr(gdelta[m]));
    CHECK(check_ptr(gnoise));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_adjoint_workspace_bytes(g, nmax)) return GRIDSPT_EWORKSPACE;
    CHECK(check_finite(c, g, gdelta, nmax, work));
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_adjoint<T, N>(c, g, lp, nmax, n2max2, delta_k, theta_k, gdelta, gnoise, work, tu, Batch{});
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
    if (work_bytes < pipe_bytes(g, 1)) return GRIDSPT_EWORKSPACE;
    CHECK(check_finite(c, g, &field, 1, work));
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_forward<T, N>(c, g, n2max, field, field_k, work, tu, Batch{});
    });
}

int gridspt_spectrum_half(gridspt_ctx* c, const gridspt_grid* g, const void* cube, void* half) {
    if (!c) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_ptr(cube));
    CHECK(check_ptr(half));
    const Dims d = dims_of(g);
    const CubeDims cd{(int)d.Kc, (int)d.Kz, (int)d.Ky};
    const double bytes = ((double)d.N * d.N * (d.N / 2 + 1) + (double)d.cube()) * d.cpx_bytes;
    const unsigned blocks = (unsigned)std::min<int64_t>(8192, (d.N * d.N * (d.N / 2 + 1) + 255) / 256);
    if (g->dtype == GRIDSPT_F64)
        return launch(c, KD_COPY, bytes, dim3(blocks), dim3(256), 0, k_spectrum_half<double>,
                      static_cast<const cpx<double>*>(cube), static_cast<cpx<double>*>(half), g->n, cd);
    return launch(c, KD_COPY, bytes, dim3(blocks), dim3(256), 0, k_spectrum_half<float>,
                  static_cast<const cpx<float>*>(cube), static_cast<cpx<float>*>(half), g->n, cd);
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
    if (work_bytes < pipe_bytes(g, nmax)) return GRIDSPT_EWORKSPACE;
    CHECK(check_finite(c, g, &delta1, 1, work));
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_orders<T, N>(c, g, nullptr, nmax, n2max1, n2max2, delta1, delta, theta, delta_k, theta_k, work, tu,
                                Batch{});
    });
}

int gridspt_orders_linear(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int32_t nmax,
                          int64_t n2max2, void* const* delta, void* const* theta, void* const* delta_k,
                          void* const* theta_k, void* work, int64_t work_bytes) {
    if (!c || !lp) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    CHECK(check_linpk(g, lp));
    if (nmax > 1) CHECK(check_mask(g, n2max2));
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
    if (work_bytes < pipe_bytes(g, nmax)) return GRIDSPT_EWORKSPACE;
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_orders<T, N>(c, g, lp, nmax, lp->n2max, n2max2, nullptr, delta, theta, delta_k, theta_k, work, tu,
                                Batch{});
    });
}

// The pass kinds the autotuner times, and one timed trial of the seeded
// orders with every kind in variant v.
static const int kOrderKinds[] = {KD_ZFWD_NOISE, KD_ZFWD_PRODUCTS, KD_YFWD, KD_XFUSED_LINEAR, KD_XFUSED_ORDER,
                                  KD_YINV, KD_ZINV};

int gridspt_tune_orders(gridspt_ctx* c, const gridspt_grid* g, const gridspt_linpk* lp, int32_t nmax, int64_t n2max2,
                        void* const* delta, void* const* theta, void* const* delta_k, void* const* theta_k,
                        void* work, int64_t work_bytes) {
    if (!c || !lp) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    CHECK(check_linpk(g, lp));
    if (nmax > 1) CHECK(check_mask(g, n2max2));
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
    if (work_bytes < pipe_bytes(g, nmax)) return GRIDSPT_EWORKSPACE;
    int vl[8];
    const int nv = variant_list(g->dtype, g->n, vl);
    gridspt_ctx::Tuned best{g->n, g->dtype, Tuning{}, {}};
    for (int k = 0; k < KD_COUNT; ++k) best.ms[k] = 1e300;
    auto trial = [&](int v, bool keep) -> int {
        gridspt_ctx t;
        t.stream = c->stream;
        t.profile = true;
        Tuning tu;
        for (int k = 0; k < KD_COUNT; ++k) tu.v[k] = v;
        const int rc = dispatch(g, [&](auto tag, auto nc) -> int {
            using T = typename decltype(tag)::type;
            constexpr int N = decltype(nc)::value;
            return run_orders<T, N>(&t, g, lp, nmax, lp->n2max, n2max2, nullptr, delta, theta, delta_k, theta_k, work,
                                    tu, Batch{});
        });
        double ms[KD_COUNT] = {};
        const bool synced = hipStreamSynchronize(t.stream) == hipSuccess;
        for (auto& r : t.recs) {
            float x = 0.f;
            if (synced && rc == GRIDSPT_OK && hipEventElapsedTime(&x, r.start, r.stop) == hipSuccess) ms[r.kind] += x;
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        for (auto e : t.pool) (void)hipEventDestroy(e);
        if (!synced) return GRIDSPT_EHIP;
        if (rc != GRIDSPT_OK) return rc;
        if (keep)
            for (int k : kOrderKinds)
                if (ms[k] > 0.0 && ms[k] < best.ms[k]) {
                    best.ms[k] = ms[k];
                    best.tu.v[k] = v;
                }
        return GRIDSPT_OK;
    };
    CHECK(trial(0, false));  // warm-up
    for (int i = 0; i < nv; ++i) CHECK(trial(vl[i], true));
    for (int k = 0; k < KD_COUNT; ++k)
        if (best.ms[k] >= 1e300) best.ms[k] = 0.0;
    // the same variant for the other uses of a pass kind
    best.tu.v[KD_ZFWD_FIELD] = best.tu.v[KD_ZFWD_NOISE];
    best.tu.v[KD_XFUSED_ORDER1] = best.tu.v[KD_XFUSED_LINEAR];
    for (auto& t : c->tuned)
        if (t.n == g->n && t.dtype == g->dtype) {
            t = best;
            return nv;
        }
    c->tuned.push_back(best);
    return nv;
}

int gridspt_set_tuning(gridspt_ctx* c, const gridspt_grid* g, int32_t variant) {
    if (!c) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    int vl[8];
    const int nv = variant_list(g->dtype, g->n, vl);
    bool ok = false;
    for (int i = 0; i < nv; ++i) ok = ok || vl[i] == variant;
    if (!ok) return GRIDSPT_EINVAL;
    gridspt_ctx::Tuned t{g->n, g->dtype, Tuning{}, {}};
    for (int k = 0; k < KD_COUNT; ++k) {
        t.tu.v[k] = variant;
        t.ms[k] = 0.0;
    }
    for (auto& x : c->tuned)
        if (x.n == g->n && x.dtype == g->dtype) {
            x = t;
            return GRIDSPT_OK;
        }
    c->tuned.push_back(t);
    return GRIDSPT_OK;
}

int gridspt_tuning(const gridspt_ctx* c, const gridspt_grid* g, int32_t max, char* names, int32_t* variant,
                   double* ms) {
    if (!c || !g || max < 0) return GRIDSPT_EINVAL;
    const gridspt_ctx::Tuned* t = nullptr;
    for (const auto& x : c->tuned)
        if (x.n == g->n && x.dtype == g->dtype) t = &x;
    int k = 0;
    for (int kind : kOrderKinds) {
        if (k >= max) break;
        if (names) {
            std::memset(names + 32 * k, 0, 32);
            std::strncpy(names + 32 * k, kKindNames[kind], 31);
        }
        if (variant) variant[k] = t ? t->tu.v[kind] : 0;
        if (ms) ms[k] = t ? t->ms[kind] : 0.0;
        ++k;
    }
    return k;
}

int64_t gridspt_pform_workspace_bytes(const gridspt_grid* g, int32_t nmax) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (nmax < 1 || nmax > 5) return GRIDSPT_EINVAL;
    return pform_layout(dims_of(g), nmax).end;
}

int gridspt_orders_pform(gridspt_ctx* c, const gridspt_grid* g, int32_t nmax, int64_t n2max1, int64_t n2max2,
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
        if (i > 0 && delta_k && theta_k && delta_k[i] && delta_k[i] == theta_k[i]) return GRIDSPT_EINVAL;
    }
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_pform_workspace_bytes(g, nmax)) return GRIDSPT_EWORKSPACE;
    CHECK(check_finite(c, g, &delta1, 1, work));
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_orders_pform<T, N>(c, g, nmax, n2max1, n2max2, delta1, delta, theta, delta_k, theta_k, work, tu,
                                      Batch{});
    });
}

int gridspt_smooth(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                   const double* coef, int32_t cumulative, double radius, void* const* out, void* work,
                   int64_t work_bytes) {
    if (!c || !fields_k || !coef || !out) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nfields < 1 || nfields > 5 || !(radius >= 0.0) || !std::isfinite(radius)) return GRIDSPT_EINVAL;
    for (int i = 0; i < nfields; ++i) {
        CHECK(check_ptr(fields_k[i]));
        CHECK(check_ptr(out[i]));
        if (!std::isfinite(coef[i])) return GRIDSPT_EINVAL;
    }
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < pipe_bytes(g, 1)) return GRIDSPT_EWORKSPACE;
    const Tuning& tu = c->tuning(g);
    return dispatch(g, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_smooth<T, N>(c, g, nfields, fields_k, coef, cumulative, radius, out, work, tu, Batch{});
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
        auto run = [&](auto kern) { return launch(c, KD_SUM_ORDERS, bytes, dim3(4096), dim3(256), 0, kern, s); };
        switch (nmax) {
            case 1: return run(k_sum_orders<T, 1>);
            case 2: return run(k_sum_orders<T, 2>);
            case 3: return run(k_sum_orders<T, 3>);
            case 4: return run(k_sum_orders<T, 4>);
            case 5: return run(k_sum_orders<T, 5>);
            case 6: return run(k_sum_orders<T, 6>);
            case 7: return run(k_sum_orders<T, 7>);
            default: return run(k_sum_orders<T, 8>);
        }
    };
    if (g->dtype == GRIDSPT_F64) return go(tag_t<double>{});
    return go(tag_t<float>{});
}

int64_t gridspt_power_workspace_bytes(const gridspt_grid* g, int32_t npairs, int32_t nbins) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (npairs < 1 || npairs > kMaxPairs || nbins < 1 || nbins > kMaxBins) return GRIDSPT_EINVAL;
    return power_ws(dims_of(g), nbins);
}

int gridspt_power(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                  int32_t npairs, const int32_t* pairs, int32_t nbins, const int64_t* edge_n2, double* pk,
                  double* kmean, double* nmodes, void* work, int64_t work_bytes) {
    if (!c || !fields_k) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_power_args(nfields, npairs, pairs, nbins, edge_n2));
    for (int i = 0; i < nfields; ++i) CHECK(check_ptr(fields_k[i]));
    CHECK(check_ptr(pk));
    if (kmean) CHECK(check_ptr(kmean));
    if (nmodes) CHECK(check_ptr(nmodes));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < gridspt_power_workspace_bytes(g, npairs, nbins)) return GRIDSPT_EWORKSPACE;
    return power_enqueue(c, g, fields_k, npairs, pairs, nbins, edge_n2, pk, kmean, nmodes, work, Batch{});
}

int gridspt_power_static(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                         int32_t npairs, const int32_t* pairs, int32_t nbins, const int64_t* edge_n2, double* pk,
                         double* kmean, double* nmodes) {
    if (!c || !fields_k) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_power_args(nfields, npairs, pairs, nbins, edge_n2));
    for (int i = 0; i < nfields; ++i) CHECK(check_ptr(fields_k[i]));
    CHECK(check_ptr(pk));
    if (kmean) CHECK(check_ptr(kmean));
    if (nmodes) CHECK(check_ptr(nmodes));
    if (power_ws(dims_of(g), nbins) > kStaticScratchBytes) return GRIDSPT_EWORKSPACE;
    void* ws = nullptr;
    CHECK(static_scratch(&ws));
    // every word of the scratch the kernels read is written earlier in the same call
    return power_enqueue(c, g, fields_k, npairs, pairs, nbins, edge_n2, pk, kmean, nmodes, ws, Batch{});
}

// ---- one-point statistics ----

// kMomentBlocks: the moments pass (with the one-point histograms); kHistBlocks:
// the joint histograms
static constexpr int kMomentBlocks = 1024, kHistBlocks = 512;

static int64_t stats_ws(int nfields, int nbins, int nbins2) {
    int64_t b = align_up((int64_t)kMomentBlocks * kStatsQ * 8) + align_up((int64_t)kStatsQ * 8);
    if (nbins > 0) b += align_up((int64_t)nfields * kMomentBlocks * nbins * 4);
    if (nbins2 > 0 && nfields > 1) b += align_up((int64_t)(nfields - 1) * kHistBlocks * nbins2 * nbins2 * 4);
    return b;
}

int64_t gridspt_stats_workspace_bytes(int32_t nfields, int32_t nbins, int32_t nbins2) {
    if (nfields < 1 || nfields > kStatsMaxFields || nbins < 0 || nbins > 1024 || nbins2 < 0 || nbins2 > 64)
        return GRIDSPT_EINVAL;
    return stats_ws(nfields, nbins, nbins2);
}

int gridspt_field_stats(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields,
                        int32_t nbins, double lo, double hi, int32_t nbins2, double* moments, double* corr,
                        double* counts, double* joint, void* work, int64_t work_bytes) {
    if (!c || !fields) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    if (nfields < 1 || nfields > kStatsMaxFields || nbins < 0 || nbins > 1024 || nbins2 < 0 || nbins2 > 64)
        return GRIDSPT_EINVAL;
    if ((counts && nbins < 1) || (joint && (nbins2 < 1 || nfields < 2))) return GRIDSPT_EINVAL;
    if ((counts || joint) && !(std::isfinite(lo) && std::isfinite(hi) && lo < hi)) return GRIDSPT_EINVAL;
    for (int i = 0; i < nfields; ++i) CHECK(check_ptr(fields[i]));
    for (double* p : {moments, corr, counts, joint})
        if (p) CHECK(check_ptr(p));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    if (work_bytes < stats_ws(nfields, counts ? nbins : 0, joint ? nbins2 : 0)) return GRIDSPT_EWORKSPACE;
    const Dims d = dims_of(g);
    const size_t ncell = (size_t)d.ncell();
    char* base = static_cast<char*>(work);
    double* mpart = reinterpret_cast<double*>(base);
    double* msum = reinterpret_cast<double*>(base + align_up((int64_t)kMomentBlocks * kStatsQ * 8));
    char* hbase = base + align_up((int64_t)kMomentBlocks * kStatsQ * 8) + align_up((int64_t)kStatsQ * 8);
    uint32_t* hpart = reinterpret_cast<uint32_t*>(hbase);
    uint32_t* jpart =
        reinterpret_cast<uint32_t*>(hbase + (counts ? align_up((int64_t)nfields * kMomentBlocks * nbins * 4) : 0));
    auto go = [&](auto tag) -> int {
        using T = typename decltype(tag)::type;
        if (moments || corr || counts) {
            // one pass over the fields: the moment sums and, if asked, the one-point counts
            MomentArgs<T> a{};
            for (int i = 0; i < nfields; ++i) a.f[i] = static_cast<const T*>(fields[i]);
            a.nf = nfields;
            a.ncell = ncell;
            a.partial = mpart;
            a.hpart = hpart;
            a.nbins = counts ? nbins : 0;
            a.lo = lo;
            a.scale = counts ? (double)nbins / (hi - lo) : 0.0;
            // one LDS histogram per wavefront while they fit in 64 KB, else one per block
            const size_t hone = (size_t)nfields * nbins * 4;
            a.hcopies = (kStatsThreads / 64) * hone <= 65536 ? kStatsThreads / 64 : 1;
            const size_t hlds = counts ? a.hcopies * hone : 0;
            int rc = GRIDSPT_OK;
            static_for<kStatsMaxFields>([&](auto k) {
                constexpr int NF = decltype(k)::value + 1;
                if (NF == nfields)
                    rc = counts ? launch(c, KD_MOMENTS, (double)nfields * ncell * d.real_bytes, dim3(kMomentBlocks),
                                         dim3(kStatsThreads), hlds, k_moments_partial<T, NF, true>, a)
                                : launch(c, KD_MOMENTS, (double)nfields * ncell * d.real_bytes, dim3(kMomentBlocks),
                                         dim3(kStatsThreads), 0, k_moments_partial<T, NF, false>, a);
            });
            CHECK(rc);
            if (moments || corr) {
                CHECK(launch(c, KD_MOMENTS, (double)kMomentBlocks * kStatsQ * 8, dim3(kStatsQ), dim3(kReduceThreads),
                             0, k_power_reduce, (const double*)mpart, kMomentBlocks, msum, (size_t)0));
                CHECK(launch(c, KD_MOMENTS, 0.0, dim3(1), dim3(64), 0, k_moments_final, (const double*)msum, nfields,
                             (double)ncell, moments, corr));
            }
            if (counts)
                CHECK(launch(c, KD_HIST, 0.0, dim3((nbins + kHistRedBins - 1) / kHistRedBins, nfields),
                             dim3(kHistRedBins, kHistRedSlices), 0, k_hist_reduce, (const uint32_t*)hpart,
                             kMomentBlocks, nbins, counts));
        }
        HistArgs<T> h{};
        for (int i = 0; i < nfields; ++i) h.f[i] = static_cast<const T*>(fields[i]);
        h.lo = lo;
        h.ncell = ncell;
        if (joint) {
            const int nb2 = nbins2 * nbins2;
            h.nbins = nbins2;
            h.scale = (double)nbins2 / (hi - lo);
            h.partial = jpart;
            CHECK(launch(c, KD_HIST, 2.0 * (nfields - 1) * ncell * d.real_bytes, dim3(kHistBlocks, nfields - 1),
                         dim3(kStatsThreads), (size_t)nb2 * 4 * (kStatsThreads / 64), k_joint_partial<T>, h));
            CHECK(launch(c, KD_HIST, 0.0, dim3((nb2 + kHistRedBins - 1) / kHistRedBins, nfields - 1),
                         dim3(kHistRedBins, kHistRedSlices), 0, k_hist_reduce, (const uint32_t*)jpart, kHistBlocks,
                         nb2, joint));
        }
        return GRIDSPT_OK;
    };
    if (g->dtype == GRIDSPT_F64) return go(tag_t<double>{});
    return go(tag_t<float>{});
}

// Single-call bispectrum workspace: a pipeline workspace for the slot
// transforms of either precision, then the estimator's region, sized for the
// term slots (grid precision) and the triangle-count slots (FP64).
struct BispSizes {
    int64_t pipe, end;
};
BispSizes bisp_sizes(const gridspt_grid* g, const BispPlan& bt, const BispPlan& bj, int nterms, int ntri) {
    const gridspt_grid g64 = count_grid(g);
    const Dims d = dims_of(g), d64 = dims_of(&g64);
    BispSizes z;
    z.pipe = std::max(layout_of(d, 1).end, layout_of(d64, 1).end);
    z.end = z.pipe + std::max(bisp_layout(d, bt.max_slots, nterms, ntri).end,
                              bisp_layout(d64, bj.max_slots, nterms, ntri).end);
    return z;
}

int64_t gridspt_bispectrum_workspace_bytes(const gridspt_grid* g, int32_t ntri, const int32_t* tri_bins,
                                           int32_t nterms, const int32_t* terms) {
    const int rc = check_grid(g);
    if (rc != GRIDSPT_OK) return rc;
    if (ntri < 1 || nterms < 1 || !tri_bins || !terms || ntri > 4096 || nterms > 16384) return GRIDSPT_EINVAL;
    for (int t = 0; t < 3 * ntri; ++t)
        if (tri_bins[t] < 0) return GRIDSPT_EINVAL;
    for (int u = 0; u < nterms; ++u)
        if (terms[4 * u + 3] < 0 || terms[4 * u + 3] >= ntri) return GRIDSPT_EINVAL;
    const BispPlan bt = bisp_make_plan(ntri, tri_bins, nterms, terms, INT_MAX, true, false);
    const BispPlan bj = bisp_make_plan(ntri, tri_bins, nterms, terms, INT_MAX, false, true);
    return bisp_sizes(g, bt, bj, nterms, ntri).end;
}

int gridspt_bispectrum(gridspt_ctx* c, const gridspt_grid* g, int32_t nfields, const void* const* fields_k,
                       int32_t ntri, const int32_t* tri_bins, int32_t nterms, const int32_t* terms, int32_t nbins,
                       const int64_t* edge_n2, double* bk, double* ntriangles, void* work, int64_t work_bytes) {
    if (!c || !fields_k) return GRIDSPT_EINVAL;
    CHECK(check_grid(g));
    CHECK(check_bisp_args(nfields, ntri, tri_bins, nterms, terms, nbins, edge_n2));
    if (isqrt64(edge_n2[nbins] - 1) > g->kc) return GRIDSPT_EINVAL;  // shells must lie inside the cube
    CHECK(check_closure(g, ntri, tri_bins, edge_n2));
    for (int i = 0; i < nfields; ++i) CHECK(check_ptr(fields_k[i]));
    CHECK(check_ptr(bk));
    CHECK(check_ptr(ntriangles));
    if (!work) return GRIDSPT_EWORKSPACE;
    CHECK(check_ptr(work));
    const BispPlan bt = bisp_make_plan(ntri, tri_bins, nterms, terms, INT_MAX, true, false);
    const BispPlan bj = bisp_make_plan(ntri, tri_bins, nterms, terms, INT_MAX, false, true);
    const BispSizes z = bisp_sizes(g, bt, bj, nterms, ntri);
    if (work_bytes < z.end) return GRIDSPT_EWORKSPACE;
    char* est = static_cast<char*>(work) + z.pipe;
    // the triangle counts in FP64 (indicator slots read no spectrum), then the terms
    const gridspt_grid g64 = count_grid(g);
    const void* none[1] = {nullptr};
    CHECK(bisp_enqueue(c, &g64, none, bj, ntri, nterms, terms, edge_n2, nullptr, nullptr, work, est, c->tuning(&g64),
                       Batch{}, false));
    return bisp_enqueue(c, g, fields_k, bt, ntri, nterms, terms, edge_n2, bk, ntriangles, work, est, c->tuning(g),
                        Batch{});
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

namespace {

// distinct slots per bispectrum chunk of a batch (bounds the slot memory of
// every realisation to this many real fields)
constexpr int kBatchSlotCap = 32;

struct GroupPlan {
    gridspt_batch_group g;  // host arrays below replace the caller's
    std::vector<int32_t> pairs, tri_bins, terms;
    std::vector<int64_t> edges;
    gridspt_batch_out out;
    Dims d;
    BispPlan bp, bpj;  // bispectrum term sums; triangle counts
    // offsets inside one realisation's arena
    int64_t o_pipe, o_delta, o_theta, o_cube, o_pws, o_pk, o_kmean, o_nmodes, o_bws, o_bk, o_ntri, zs;
    int64_t base;  // offset of realisation 0's arena in work
    Tuning tu;
    double tune_ms[KD_COUNT] = {};
};

int64_t plan_group(GroupPlan& p) {
    const Dims& d = p.d;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const int nmax = p.g.nmax;
    // the triangle counts (FP64, once, in realisation 0's arena) reuse the
    // pipeline workspace and the estimator region
    const gridspt_grid g64 = count_grid(&p.g.grid);
    const Dims d64 = dims_of(&g64);
    p.o_pipe = take(std::max(layout_of(d, nmax).end, p.g.ntri > 0 ? layout_of(d64, 1).end : 0));
    p.o_delta = take((int64_t)nmax * d.ncell() * d.real_bytes);
    p.o_theta = take((int64_t)std::max(nmax - 1, 0) * d.ncell() * d.real_bytes);
    p.o_cube = take((int64_t)nmax * d.cube() * d.cpx_bytes);
    p.o_pws = take(power_ws(d, p.g.nbins));
    p.o_pk = take((int64_t)p.g.npairs * p.g.nbins * 8);
    p.o_kmean = take((int64_t)p.g.nbins * 8);
    p.o_nmodes = take((int64_t)p.g.nbins * 8);
    if (p.g.ntri > 0) {
        // the bispectrum's transforms reuse the pipeline workspace (the orders are done)
        p.o_bws = take(std::max(bisp_layout(d, p.bp.max_slots, p.g.nterms, p.g.ntri).end,
                                bisp_layout(d64, p.bpj.max_slots, p.g.nterms, p.g.ntri).end));
        p.o_bk = take((int64_t)p.g.nterms * 8);
        p.o_ntri = take((int64_t)p.g.ntri * 8);
    } else {
        p.o_bws = p.o_bk = p.o_ntri = 0;
    }
    p.zs = o;
    return (int64_t)p.g.nreal * o;
}

int check_group(const gridspt_batch_group& g) {
    CHECK(check_grid(&g.grid));
    if (g.nreal < 1 || g.nmax < 1 || g.nmax > 5) return GRIDSPT_EINVAL;
    CHECK(check_linpk(&g.grid, &g.lin));
    if (g.nmax > 1) CHECK(check_mask(&g.grid, g.n2max2));
    CHECK(check_power_args(g.nmax, g.npairs, g.pairs, g.nbins, g.edge_n2));
    if (g.ntri < 0) return GRIDSPT_EINVAL;
    if (g.ntri > 0) {
        CHECK(check_bisp_args(g.nmax, g.ntri, g.tri_bins, g.nterms, g.terms, g.nbins, g.edge_n2));
        if (isqrt64(g.edge_n2[g.nbins] - 1) > g.grid.kc) return GRIDSPT_EINVAL;
        CHECK(check_closure(&g.grid, g.ntri, g.tri_bins, g.edge_n2));
    }
    return GRIDSPT_OK;
}

int make_group(const gridspt_batch_group& src, GroupPlan& p) {
    CHECK(check_group(src));
    p.g = src;
    p.pairs.assign(src.pairs, src.pairs + 2 * src.npairs);
    p.edges.assign(src.edge_n2, src.edge_n2 + src.nbins + 1);
    if (src.ntri > 0) {
        p.tri_bins.assign(src.tri_bins, src.tri_bins + 3 * src.ntri);
        p.terms.assign(src.terms, src.terms + 4 * src.nterms);
    }
    p.g.pairs = p.pairs.data();
    p.g.edge_n2 = p.edges.data();
    p.g.tri_bins = p.tri_bins.empty() ? nullptr : p.tri_bins.data();
    p.g.terms = p.terms.empty() ? nullptr : p.terms.data();
    p.d = dims_of(&p.g.grid);
    if (src.ntri > 0) {
        // term sums in every launch of the batch; triangle counts once, at plan
        // creation, in FP64 (half as many slots of twice the size for FP32 grids)
        const int jcap = src.grid.dtype == GRIDSPT_F64 ? kBatchSlotCap : kBatchSlotCap / 2;
        p.bp = bisp_make_plan(src.ntri, p.g.tri_bins, src.nterms, p.g.terms, kBatchSlotCap, true, false);
        p.bpj = bisp_make_plan(src.ntri, p.g.tri_bins, src.nterms, p.g.terms, jcap, false, true);
    }
    return GRIDSPT_OK;
}

}  // namespace

struct gridspt_batch {
    gridspt_ctx* ctx = nullptr;
    char* work = nullptr;
    uint32_t flags = 0;
    std::vector<GroupPlan> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;  // capture stream + one per group
    std::vector<hipEvent_t> events;
};

namespace {

char* arena(const gridspt_batch* b, const GroupPlan& p, int64_t off) { return b->work + p.base + off; }

// Everything one group does, enqueued on c's stream over all its realisations.
// stats: also the spectra, bispectra and the realisation statistics.
int enqueue_group(gridspt_ctx* c, gridspt_batch* b, GroupPlan& p, const Tuning& tu, bool stats) {
    const gridspt_batch_group& g = p.g;
    const Dims& d = p.d;
    const Batch bt{g.nreal, (size_t)p.zs};
    const int nmax = g.nmax;
    void* work = arena(b, p, p.o_pipe);
    void* delta[5] = {};
    void* theta[5] = {};
    void* cube[5] = {};
    for (int i = 0; i < nmax; ++i) {
        delta[i] = arena(b, p, p.o_delta + (int64_t)i * d.ncell() * d.real_bytes);
        theta[i] = i == 0 ? delta[0] : arena(b, p, p.o_theta + (int64_t)(i - 1) * d.ncell() * d.real_bytes);
        cube[i] = arena(b, p, p.o_cube + (int64_t)i * d.cube() * d.cpx_bytes);
    }
    const gridspt_grid* gr = &g.grid;
    CHECK(dispatch(gr, [&](auto tag, auto nc) -> int {
        using T = typename decltype(tag)::type;
        constexpr int N = decltype(nc)::value;
        return run_orders<T, N>(c, gr, &g.lin, nmax, g.lin.n2max, g.n2max2, nullptr, delta, theta, cube, nullptr, work,
                                tu, bt);
    }));
    const unsigned one = 1;
    if (stats) {
        double* pk = reinterpret_cast<double*>(arena(b, p, p.o_pk));
        double* km = reinterpret_cast<double*>(arena(b, p, p.o_kmean));
        double* nm = reinterpret_cast<double*>(arena(b, p, p.o_nmodes));
        CHECK(power_enqueue(c, gr, cube, g.npairs, g.pairs, g.nbins, g.edge_n2, pk, km, nm, arena(b, p, p.o_pws), bt));
        const int npk = g.npairs * g.nbins;
        CHECK(launch(c, KD_BATCH_STATS, 0.0, dim3((npk + 63) / 64), dim3(64), 0, k_batch_stats, (const double*)pk,
                     g.nreal, npk, (size_t)p.zs, p.out.pk_mean, p.out.pk_std));
        CHECK(launch(c, KD_BATCH_STATS, 0.0, dim3((g.nbins + 63) / 64), dim3(64), 0, k_batch_stats, (const double*)km,
                     (int)one, g.nbins, (size_t)p.zs, p.out.kmean, (double*)nullptr));
        CHECK(launch(c, KD_BATCH_STATS, 0.0, dim3((g.nbins + 63) / 64), dim3(64), 0, k_batch_stats, (const double*)nm,
                     (int)one, g.nbins, (size_t)p.zs, p.out.nmodes, (double*)nullptr));
    }
    if (g.ntri > 0) {
        double* bk = reinterpret_cast<double*>(arena(b, p, p.o_bk));
        double* nt = reinterpret_cast<double*>(arena(b, p, p.o_ntri));
        if (stats) {
            CHECK(bisp_enqueue(c, gr, cube, p.bp, g.ntri, g.nterms, g.terms, g.edge_n2, bk, nt, work,
                               arena(b, p, p.o_bws), tu, bt, true, 0));
            CHECK(launch(c, KD_BATCH_STATS, 0.0, dim3((g.nterms + 63) / 64), dim3(64), 0, k_batch_stats,
                         (const double*)bk, g.nreal, g.nterms, (size_t)p.zs, p.out.bk_mean, p.out.bk_std));
            CHECK(launch(c, KD_BATCH_STATS, 0.0, dim3((g.ntri + 63) / 64), dim3(64), 0, k_batch_stats,
                         (const double*)nt, (int)one, g.ntri, (size_t)p.zs, p.out.ntriangles, (double*)nullptr));
        } else {
            // the tuner times the shell transforms of the first chunk
            const BispChunk& ch = p.bp.chunks.front();
            const int ns = (int)ch.slots.size();
            const BispLayout bl = bisp_layout(d, p.bp.max_slots, g.nterms, g.ntri);
            std::vector<const void*> cubes(ns);
            std::vector<int64_t> lo(ns), hi(ns);
            std::vector<void*> outs(ns);
            for (int i = 0; i < ns; ++i) {
                cubes[i] = ch.slots[i].first >= 0 ? cube[ch.slots[i].first] : nullptr;
                lo[i] = g.edge_n2[ch.slots[i].second];
                hi[i] = g.edge_n2[ch.slots[i].second + 1];
                outs[i] = arena(b, p, p.o_bws + bl.slots + (int64_t)i * d.ncell() * d.real_bytes);
            }
            CHECK(dispatch(gr, [&](auto tag, auto nc) -> int {
                using T = typename decltype(tag)::type;
                constexpr int N = decltype(nc)::value;
                return run_shells<T, N>(c, gr, ns, cubes.data(), lo.data(), hi.data(), outs.data(), work, tu, bt);
            }));
        }
    }
    return GRIDSPT_OK;
}

constexpr int kTunedKinds[] = {KD_ZFWD_NOISE, KD_ZFWD_FIELD, KD_ZFWD_PRODUCTS, KD_YFWD, KD_XFUSED_LINEAR,
                               KD_XFUSED_ORDER1, KD_XFUSED_ORDER, KD_XSHELL, KD_YINV, KD_ZINV};

// per kind: milliseconds of one trial run of the group with every kind in variant v
int trial(gridspt_batch* b, GroupPlan& p, int v, double (&ms)[KD_COUNT]) {
    gridspt_ctx c;
    c.stream = b->ctx->stream;
    c.profile = true;
    Tuning tu;
    for (int k = 0; k < KD_COUNT; ++k) tu.v[k] = v;
    const int rc = enqueue_group(&c, b, p, tu, false);
    for (int k = 0; k < KD_COUNT; ++k) ms[k] = 0.0;
    if (hipStreamSynchronize(c.stream) != hipSuccess) return GRIDSPT_EHIP;
    for (auto& r : c.recs) {
        float t = 0.f;
        if (rc == GRIDSPT_OK && hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) return GRIDSPT_EHIP;
        ms[r.kind] += t;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : c.pool) (void)hipEventDestroy(e);
    return rc;
}

int tune_group(gridspt_batch* b, GroupPlan& p) {
    int vl[8];
    const int nv = variant_list(p.g.grid.dtype, p.g.grid.n, vl);
    double best[KD_COUNT];
    for (int k = 0; k < KD_COUNT; ++k) best[k] = 1e300;
    double ms[KD_COUNT];
    CHECK(trial(b, p, 0, ms));  // warm-up
    for (int i = 0; i < nv; ++i) {
        CHECK(trial(b, p, vl[i], ms));
        for (int k : kTunedKinds)
            if (ms[k] > 0.0 && ms[k] < best[k]) {
                best[k] = ms[k];
                p.tu.v[k] = vl[i];
                p.tune_ms[k] = ms[k];
            }
    }
    return GRIDSPT_OK;
}

// The triangle counts N_123 of a group's bispectrum depend only on the grid
// and the bins: made once, in FP64, in realisation 0's sums, before any launch
// of the batch (FP64 compiles only the default launch variant).
int setup_triangles(gridspt_batch* b, GroupPlan& p) {
    if (p.g.ntri == 0) return GRIDSPT_OK;
    const void* none[1] = {nullptr};  // indicator slots read no spectrum
    const gridspt_grid g64 = count_grid(&p.g.grid);
    return bisp_enqueue(b->ctx, &g64, none, p.bpj, p.g.ntri, p.g.nterms, p.g.terms, p.g.edge_n2, nullptr, nullptr,
                        arena(b, p, p.o_pipe), arena(b, p, p.o_bws), Tuning{}, Batch{1, 0}, false, 0);
}

void release(gridspt_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto e : b->events) (void)hipEventDestroy(e);
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    b->exec = nullptr;
    b->graph = nullptr;
    b->events.clear();
    b->streams.clear();
}

int capture(gridspt_batch* b) {
    const int ng = (int)b->groups.size();
    b->streams.assign(ng + 1, nullptr);
    for (auto& s : b->streams)
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return GRIDSPT_EHIP;
    b->events.assign(ng + 1, nullptr);
    for (auto& e : b->events)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return GRIDSPT_EHIP;
    hipStream_t cs = b->streams[0];
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return GRIDSPT_EHIP;
    int rc = GRIDSPT_OK;
    if (hipEventRecord(b->events[0], cs) != hipSuccess) rc = GRIDSPT_EHIP;
    for (int i = 0; i < ng && rc == GRIDSPT_OK; ++i) {
        gridspt_ctx c;
        c.stream = b->streams[i + 1];
        if (hipStreamWaitEvent(c.stream, b->events[0], 0) != hipSuccess) {
            rc = GRIDSPT_EHIP;
            break;
        }
        rc = enqueue_group(&c, b, b->groups[i], b->groups[i].tu, true);
        if (rc == GRIDSPT_OK && hipEventRecord(b->events[i + 1], c.stream) != hipSuccess) rc = GRIDSPT_EHIP;
        if (rc == GRIDSPT_OK && hipStreamWaitEvent(cs, b->events[i + 1], 0) != hipSuccess) rc = GRIDSPT_EHIP;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != GRIDSPT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess || !graph) return GRIDSPT_EHIP;
    b->graph = graph;
    if (hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) return GRIDSPT_EHIP;
    return GRIDSPT_OK;
}

int64_t batch_layout(std::vector<GroupPlan>& gp) {
    int64_t total = 0;
    for (auto& p : gp) {
        const int64_t bytes = plan_group(p);
        p.base = total;
        total = align_up(total + bytes);
    }
    return total;
}

}  // namespace

extern "C" {

int64_t gridspt_batch_workspace_bytes(int32_t ngroups, const gridspt_batch_group* groups) {
    if (ngroups < 1 || ngroups > 64 || !groups) return GRIDSPT_EINVAL;
    std::vector<GroupPlan> gp(ngroups);
    for (int i = 0; i < ngroups; ++i) CHECK(make_group(groups[i], gp[i]));
    return batch_layout(gp);
}

int gridspt_batch_create(gridspt_ctx* c, int32_t ngroups, const gridspt_batch_group* groups,
                         const gridspt_batch_out* outs, void* work, int64_t work_bytes, uint32_t flags,
                         gridspt_batch** out) {
    if (!c || !out || !outs || ngroups < 1 || ngroups > 64 || !groups) return GRIDSPT_EINVAL;
    if (flags & ~(uint32_t)(GRIDSPT_BATCH_TUNE | GRIDSPT_BATCH_EAGER)) return GRIDSPT_EINVAL;
    *out = nullptr;
    gridspt_batch* b = new (std::nothrow) gridspt_batch();
    if (!b) return GRIDSPT_EINVAL;
    b->groups.resize(ngroups);
    int rc = GRIDSPT_OK;
    for (int i = 0; i < ngroups && rc == GRIDSPT_OK; ++i) rc = make_group(groups[i], b->groups[i]);
    for (int i = 0; i < ngroups && rc == GRIDSPT_OK; ++i) {
        const gridspt_batch_out& o = outs[i];
        const gridspt_batch_group& g = groups[i];
        b->groups[i].out = o;
        for (double* p : {o.pk_mean, o.pk_std, o.kmean, o.nmodes, o.bk_mean, o.bk_std, o.ntriangles})
            if (p && check_ptr(p) != GRIDSPT_OK) rc = GRIDSPT_EALIGN;
        if (!o.pk_mean || (g.ntri > 0 && !o.bk_mean)) rc = GRIDSPT_EINVAL;
    }
    const int64_t need = rc == GRIDSPT_OK ? batch_layout(b->groups) : 0;
    if (rc == GRIDSPT_OK && (!work || work_bytes < need)) rc = GRIDSPT_EWORKSPACE;
    if (rc == GRIDSPT_OK) rc = check_ptr(work);
    if (rc != GRIDSPT_OK) {
        delete b;
        return rc;
    }
    b->ctx = c;
    b->work = static_cast<char*>(work);
    b->flags = flags;
    if (flags & GRIDSPT_BATCH_TUNE)
        for (auto& p : b->groups)
            if (rc == GRIDSPT_OK) rc = tune_group(b, p);
    for (auto& p : b->groups)
        if (rc == GRIDSPT_OK) rc = setup_triangles(b, p);
    if (rc == GRIDSPT_OK && !(flags & GRIDSPT_BATCH_EAGER)) rc = capture(b);
    if (rc != GRIDSPT_OK) {
        release(b);
        delete b;
        return rc;
    }
    *out = b;
    return GRIDSPT_OK;
}

int gridspt_batch_run(gridspt_batch* b) {
    if (!b) return GRIDSPT_EINVAL;
    if (b->flags & GRIDSPT_BATCH_EAGER) {
        for (auto& p : b->groups) CHECK(enqueue_group(b->ctx, b, p, p.tu, true));
        return GRIDSPT_OK;
    }
    if (hipGraphLaunch(b->exec, b->ctx->stream) != hipSuccess) return GRIDSPT_EHIP;
    return GRIDSPT_OK;
}

void gridspt_batch_destroy(gridspt_batch* b) {
    if (!b) return;
    release(b);
    delete b;
}

int gridspt_batch_buffer(const gridspt_batch* b, int32_t group, int32_t real, int32_t what, int32_t index,
                         void** ptr) {
    if (!b || !ptr || group < 0 || group >= (int)b->groups.size()) return GRIDSPT_EINVAL;
    const GroupPlan& p = b->groups[group];
    if (real < 0 || real >= p.g.nreal) return GRIDSPT_EINVAL;
    const int64_t r0 = (int64_t)real * p.zs;
    const Dims& d = p.d;
    int64_t off;
    switch (what) {
        case GRIDSPT_BATCH_DELTA:
        case GRIDSPT_BATCH_THETA:
            if (index < 0 || index >= p.g.nmax) return GRIDSPT_EINVAL;
            if (what == GRIDSPT_BATCH_DELTA || index == 0) off = p.o_delta + (int64_t)index * d.ncell() * d.real_bytes;
            else off = p.o_theta + (int64_t)(index - 1) * d.ncell() * d.real_bytes;
            break;
        case GRIDSPT_BATCH_DELTA_K:
            if (index < 0 || index >= p.g.nmax) return GRIDSPT_EINVAL;
            off = p.o_cube + (int64_t)index * d.cube() * d.cpx_bytes;
            break;
        case GRIDSPT_BATCH_PK:
            if (index != 0) return GRIDSPT_EINVAL;
            off = p.o_pk;
            break;
        case GRIDSPT_BATCH_BK:
            if (index != 0 || p.g.ntri == 0) return GRIDSPT_EINVAL;
            off = p.o_bk;
            break;
        default: return GRIDSPT_EINVAL;
    }
    *ptr = b->work + p.base + r0 + off;
    return GRIDSPT_OK;
}

int gridspt_batch_tuning(const gridspt_batch* b, int32_t group, int32_t max, char* names, int32_t* variant,
                         double* ms) {
    if (!b || group < 0 || group >= (int)b->groups.size() || max < 0) return GRIDSPT_EINVAL;
    const GroupPlan& p = b->groups[group];
    int k = 0;
    for (int kind : kTunedKinds) {
        if (k >= max) break;
        if (names) {
            std::memset(names + 32 * k, 0, 32);
            std::strncpy(names + 32 * k, kKindNames[kind], 31);
        }
        if (variant) variant[k] = p.tu.v[kind];
        if (ms) ms[k] = p.tune_ms[kind];
        ++k;
    }
    return k;
}

}  // extern "C"

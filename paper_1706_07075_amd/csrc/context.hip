// Host runtime and C ABI of liblmtof.so: context, device buffers, event
// ingest, sensitivity, the graph-replayed MLEM iteration and the projector
// testing surface.  See include/lmtof.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "lmtof.h"
#include "lmtof_internal.h"

using namespace lmtof;

namespace {

constexpr double kDefaultC = 0.299792458;
constexpr int kDefaultEpt = 4;
constexpr int kDefaultBrickChunks = 8192;
constexpr float kAutotuneIters = 10.0f;  // iterations a reconstruction is assumed to run
constexpr double kTofRejectZ = 1.959964;  // two-sided 95 % quantile of the normal distribution
// Event records per graph-replayed iteration: start, after the forward
// kernel, after the forward stage (ratios on the items), after brick
// scales, after brick back projection, after tile reduction, end.
constexpr int kEventsPerIter = 7;

// Device scratch of the allocation-free sampled forward projection: the
// projections in stored event order, before they are put in the caller's
// order.  Each device holds its own copy while the library is loaded.  In
// host code `scratch` only names the symbol: its device address, per
// device, comes from hipGetSymbolAddress (resolved in lmtof_create with the
// device current) and is the only form passed to kernels.
constexpr int64_t kNoAllocMaxEvents = int64_t(1) << 22;
static __device__ __align__(256) float scratch[kNoAllocMaxEvents];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
// autotuner results of this process, by (arch, grid, voxel, FWHM, storage,
// regions, event-count class)
std::mutex g_tune_mu;
std::map<std::string, lmtof_tune_result> g_tune_cache;

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;  // kEventsPerIter per iteration
};

struct Region {
    int z_lo = 0, nz = 0, core_lo = 0, core_hi = 0;
    int64_t n_events = 0, ev_offset = 0;
    float *x = nullptr, *b = nullptr, *s = nullptr;
};

// A device buffer kept between calls (bytes).
struct Scratch {
    void *p = nullptr;
    size_t cap = 0;
};

// Brick item lists of one problem batch (see the projector): items grouped
// by brick; chunks (brick, first item, end item, tile slot) largest first;
// per non-empty brick its tile slots (brick, first slot, end slot); the
// tile scratch (one 16^3 FP32 tile per slot).
struct ItemSet {
    float *pw = nullptr;  // per item: forward partial, then its event's back-projection weight
    // per event (the problems' events, stored order): first entry of its
    // item positions in evitems (+ 1 entry); the positions in brick order
    uint32_t *evoff = nullptr, *evitems = nullptr;
    uint32_t *scan_tmp = nullptr;
    uint16_t *itemslot = nullptr;  // per run item, in run order: its (event in chunk, ordinal) slot
    uint8_t *evflag = nullptr;     // per event: reached through evitems by the combine pass
    uint4 *chunks = nullptr, *bricks = nullptr;
    unsigned long long *tiles = nullptr;
    // per brick of the batch (every problem's, empty ones too): its
    // largest |w| (FP32 bits, set by the combine pass); per problem: the
    // combine pass's flag for weights written outside its runs
    uint32_t *bwmax = nullptr, *gflag = nullptr;
    char *item_recs = nullptr;  // walk records in item order (32 B each)
    size_t item_bytes = 0;
    // builder scratch: per-key counters and offsets, the counting blocks'
    // key tables (then the forward chunks' run lists)
    uint32_t *cnt = nullptr, *off_d = nullptr, *tabs = nullptr;
    // capacities (elements) of every array above: the lists are rebuilt in
    // place and a buffer is only reallocated when it has to grow, so
    // reloading events of a similar size allocates and frees nothing
    size_t pw_cap = 0, evoff_cap = 0, evitems_cap = 0, scan_cap = 0, itemslot_cap = 0, evflag_cap = 0,
           item_recs_cap = 0, tiles_cap = 0, chunks_cap = 0, bricks_cap = 0, bwmax_cap = 0, gflag_cap = 0,
           cnt_cap = 0, off_cap = 0, tabs_cap = 0;
    uint32_t n_chunks = 0, n_bricks = 0, n_slots = 0;
    uint64_t n_items = 0, n_all_bricks = 0;  // n_bricks: non-empty ones
    std::vector<uint4> h_chunks, h_bricks;  // host copies (batching several problems)
};

}  // namespace

struct lmtof_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    // options
    int opt_storage = 0, opt_sort = 1, opt_nphi = 2048, opt_ept = 0, opt_median = 0;
    int opt_forward = LMTOF_FORWARD_BRICKS;
    int opt_bchunks = kDefaultBrickChunks;
    double opt_cell_mm = 16.0;

    bool has_geom = false;
    lmtof_geometry g{};
    int64_t V = 0;

    // events (stored order)
    int64_t n_events = 0;
    int stored_packed = 0;
    void *d_events = nullptr;
    int64_t *d_perm = nullptr;  // stored position -> caller index
    size_t events_cap = 0, perm_cap = 0;  // their allocation sizes (bytes)
    // buffers kept between loads: the spare event store and permutation a
    // load or region split writes into (then swapped with the current
    // ones), and the sort's keys, histogram, scan scratch, error flag and
    // intermediate permutation; the device copy of events handed over in
    // host memory
    Scratch sc_events, sc_perm, sc_keys, sc_hist, sc_tmp, sc_err, sc_inner, sc_raw;

    // whole-volume images
    float *d_s = nullptr, *d_x = nullptr, *d_b = nullptr;
    size_t img_cap = 0;  // voxels each of d_s, d_x, d_b hold
    bool has_sens = false, has_image = false;
    int iter_count = 0;

    // regions (empty: one whole-volume problem); their x, b and s images
    // lie back to back in reg_buf; a region split fills the spare sc_reg
    // and then swaps it in
    std::vector<Region> regions;
    float *reg_buf = nullptr;
    size_t reg_cap = 0;  // bytes
    Scratch sc_reg;
    int margin_used = 0;

    // batch of problems the iteration runs
    std::vector<Problem> probs;
    Problem *d_probs = nullptr;
    int64_t n_chunks = 0, n_vchunks = 0, n_xblk = 0;
    float *d_xb = nullptr;  // blocked image copies the forward pass gathers from
    size_t xb_cap = 0;
    int ept_used = kDefaultEpt;
    ItemSet items;               // brick item lists of the iteration batch
    float *d_rw = nullptr;       // per stored event: 1 / f (MLEM) or a weight
    size_t rw_cap = 0;
    // per-event ratio weights (attenuation correction on the LOR): caller
    // order as given, stored order for the iteration
    bool has_evw = false;
    float *d_evw_caller = nullptr, *d_evw = nullptr;
    size_t evw_cap = 0, evw_stored_cap = 0;
    float4 *d_lut = nullptr;     // kernel-CDF table
    float2 *d_lin = nullptr;     // piecewise-linear kernel-CDF table (brick projectors)
    double lut_k = -1.0;
    int *d_part_neff = nullptr;
    double *d_part_ll = nullptr, *d_part_old = nullptr, *d_part_new = nullptr;
    size_t part_cap = 0, vpart_cap = 0;
    DevStats *d_stats = nullptr;
    size_t stats_cap = 0;
    double *d_scratch = nullptr;  // FP64 reduction scratch (partials + result)
    bool probs_dirty = true;

    std::map<int, GraphEntry> graphs;
};

namespace {

thread_local std::string g_create_err;

int fail(lmtof_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, expr)                                                                          \
    do {                                                                                         \
        hipError_t e__ = (expr);                                                                 \
        if (e__ != hipSuccess) return fail((c), LMTOF_EHIP, "%s: %s", #expr, hipGetErrorString(e__)); \
    } while (0)

template <class T>
int dev_alloc(lmtof_ctx *c, T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(c, LMTOF_ENOMEM, "device allocation of %zu bytes failed: %s", n * sizeof(T),
                    hipGetErrorString(e));
    }
    return LMTOF_OK;
}

template <class T>
void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// (Re)size a reusable buffer: kept when it already holds n elements, so
// repeated loads of similar size allocate nothing large.
template <class T>
int take(lmtof_ctx *c, Scratch &s, T **out, size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (!s.p || s.cap < bytes) {
        dev_free(s.p);
        s.cap = 0;
        char *q = nullptr;
        int rc = dev_alloc(c, &q, bytes);
        if (rc) return rc;
        s.p = q;
        s.cap = bytes;
    }
    *out = static_cast<T *>(s.p);
    return LMTOF_OK;
}

void scratch_free(Scratch &s) {
    dev_free(s.p);
    s.cap = 0;
}

void free_items(ItemSet &it) {
    dev_free(it.pw);
    dev_free(it.evoff);
    dev_free(it.evitems);
    dev_free(it.scan_tmp);
    dev_free(it.itemslot);
    dev_free(it.evflag);
    dev_free(it.chunks);
    dev_free(it.bricks);
    dev_free(it.tiles);
    dev_free(it.bwmax);
    dev_free(it.gflag);
    dev_free(it.item_recs);
    dev_free(it.cnt);
    dev_free(it.off_d);
    dev_free(it.tabs);
    it = ItemSet();
}

// The lists no longer describe the loaded events; their buffers stay for
// the next build.
void invalidate_items(ItemSet &it) {
    it.n_chunks = it.n_bricks = it.n_slots = 0;
    it.n_items = it.n_all_bricks = 0;
    it.item_bytes = 0;
    it.h_chunks.clear();
    it.h_bricks.clear();
}

// Destroy the instantiated iteration graphs (they hold the buffer addresses
// and launch sizes of the current batch, and its kernel sequence).
void drop_graphs_only(lmtof_ctx *c) {
    for (auto &kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        for (hipEvent_t e : kv.second.ev) (void)hipEventDestroy(e);
    }
    c->graphs.clear();
}

// ... and mark the brick lists stale.  Device buffers are kept.
void drop_graphs(lmtof_ctx *c) {
    drop_graphs_only(c);
    invalidate_items(c->items);
}

void drop_regions(lmtof_ctx *c) {
    c->regions.clear();
    c->probs_dirty = true;
}

// No events loaded any more; the event store and permutation buffers stay
// for the next load (lmtof_destroy frees them).
void drop_events(lmtof_ctx *c) {
    c->n_events = 0;
    c->has_image = false;
    drop_regions(c);
    drop_graphs(c);
    c->probs_dirty = true;
}

// Make (store, perm), taken from the spare buffers, the current events; the
// previous current buffers become the spares.
void install_events(lmtof_ctx *c) {
    std::swap(c->d_events, c->sc_events.p);
    std::swap(c->events_cap, c->sc_events.cap);
    void *pp = c->d_perm;
    c->d_perm = static_cast<int64_t *>(c->sc_perm.p);
    c->sc_perm.p = pp;
    std::swap(c->perm_cap, c->sc_perm.cap);
}

// Free the buffers kept for the next load (a served request loads once).
void release_load_scratch(lmtof_ctx *c) {
    for (Scratch *sc : {&c->sc_events, &c->sc_perm, &c->sc_keys, &c->sc_hist, &c->sc_tmp, &c->sc_err, &c->sc_inner,
                        &c->sc_raw})
        scratch_free(*sc);
}

double sigma_mm(const lmtof_geometry &g) {
    return (g.c_mm_per_ps * g.tof_fwhm_ps / 2.0) / (2.0 * std::sqrt(2.0 * std::log(2.0)));
}

// Kernel-side description of a grid (whole volume or a z-slab of it).
Problem make_problem(const lmtof_ctx *c, int z_lo, int nz, float *x, float *b, const float *s) {
    const lmtof_geometry &g = c->g;
    Problem P{};
    P.packed = c->stored_packed;
    P.tof = g.tof_fwhm_ps > 0 ? 1 : 0;
    P.nx = g.nx;
    P.ny = g.ny;
    P.nz = nz;
    const double oz = g.z0 + z_lo * g.vz;
    P.ox = (float)g.x0;
    P.oy = (float)g.y0;
    P.oz = (float)oz;
    P.hx = (float)(g.x0 + g.nx * g.vx);
    P.hy = (float)(g.y0 + g.ny * g.vy);
    P.hz = (float)(oz + nz * g.vz);
    P.vx = (float)g.vx;
    P.vy = (float)g.vy;
    P.vz = (float)g.vz;
    P.ivx = (float)(1.0 / g.vx);
    P.ivy = (float)(1.0 / g.vy);
    P.ivz = (float)(1.0 / g.vz);
    P.half_c = (float)(g.c_mm_per_ps / 2.0);
    if (P.tof) {
        const double sg = sigma_mm(g);
        P.inv_sig_sqrt2 = (float)(1.0 / (sg * std::sqrt(2.0)));
        P.k_sigma = (float)(g.tof_trunc_sigmas * sg);
        P.norm = (float)(1.0 / (2.0 * std::erf(g.tof_trunc_sigmas / std::sqrt(2.0))));
    }
    P.lut = c->d_lut;
    P.lin = c->d_lin;
    if (P.tof) {
        const double h = 2.0 * g.tof_trunc_sigmas / (kLutN - 1);
        P.lut_a = (float)(1.0 / (sigma_mm(g) * h));
        P.lut_b = (float)((kLutN - 1) / 2) + 12582912.0f;  // centre node + 1.5 2^23, exact
        const double hl = 2.0 * g.tof_trunc_sigmas / kLinN;
        P.lin_a = (float)(1.0 / (sigma_mm(g) * hl));
        P.lin_b = (float)((kLinN - 1) / 2) + 12582912.0f;  // centre cell + 1.5 2^23, exact
    }
    P.a_max = P.tof ? 1.0f : (float)std::sqrt(g.vx * g.vx + g.vy * g.vy + g.vz * g.vz);
    P.nbx = (g.nx + kBrickX - 1) / kBrickX;
    P.nby = (g.ny + kBrickY - 1) / kBrickY;
    P.nbz = (nz + kBrickZ - 1) / kBrickZ;
    P.nbx4 = (g.nx + 3) / 4;
    P.nby4 = (g.ny + 3) / 4;
    P.nbz4 = (nz + 3) / 4;
    P.xfx = 0;
    while ((1 << P.xfx) < P.nbx4) ++P.xfx;
    P.xfy = 0;
    while ((1 << P.xfy) < P.nby4) ++P.xfy;
    P.x = x;
    P.b = b;
    P.s = s;
    return P;
}

// Kernel-CDF table for truncation K: node k at u_k = -K + k h (sigma units),
// h = 2K / (n - 1), holds Phi(u_k), Phi'(u_k) h and Phi''(u_k) h^2 / 2 with
// Phi(u) = erf(u / sqrt 2) / (2 erf(K / sqrt 2)) (so a piece's weight is a
// difference of two values) and Phi'' = -u Phi'.  Evaluated in FP64.  Node
// k sits at entry k + 1; entries 0 and n + 1 repeat the end values, flat.
int ensure_lut(lmtof_ctx *c) {
    const double K = c->g.tof_trunc_sigmas;
    if (c->d_lut && c->lut_k == K) return LMTOF_OK;
    std::vector<float4> tab(kLutN + 2);
    const double h = 2.0 * K / (kLutN - 1), den = std::erf(K / std::sqrt(2.0));
    for (int k = 0; k < kLutN; ++k) {
        const double u = -K + k * h;
        const double phi = std::exp(-0.5 * u * u) / (std::sqrt(2.0 * M_PI) * den);
        tab[k + 1] = make_float4((float)(std::erf(u / std::sqrt(2.0)) / (2.0 * den)), (float)(phi * h),
                                 (float)(-u * phi * h * h / 2.0), 0.0f);
    }
    tab[0] = make_float4(tab[1].x, 0.0f, 0.0f, 0.0f);
    tab[kLutN + 1] = make_float4(tab[kLutN].x, 0.0f, 0.0f, 0.0f);
    // Piecewise-linear table: cell j spans [-K + j hl, -K + (j + 1) hl],
    // hl = 2K / kLinN; it holds the chord's value at the cell's middle and
    // the CDF difference over the cell, so CDF(t) ~ mid + f diff with f the
    // offset from the middle in cells, in [-1/2, 1/2]: continuous and
    // non-decreasing, |error| <= hl^2 max|Phi''| / 8 (~6.5e-8 at K = 3).
    // The pads repeat the end values with no slope.
    std::vector<float2> lin(kLinN + 2);
    const double hl = 2.0 * K / kLinN;
    auto cdf = [&](double u) { return std::erf(u / std::sqrt(2.0)) / (2.0 * den); };
    for (int j = 0; j < kLinN; ++j) {
        const double a = cdf(-K + j * hl), b = cdf(-K + (j + 1) * hl);
        lin[j + 1] = make_float2((float)(0.5 * (a + b)), (float)(b - a));
    }
    lin[0] = make_float2((float)cdf(-K), 0.0f);
    lin[kLinN + 1] = make_float2((float)cdf(K), 0.0f);
    if (!c->d_lut) {
        int rc = dev_alloc(c, &c->d_lut, kLutN + 2);
        if (rc) return rc;
    }
    if (!c->d_lin) {
        int rc = dev_alloc(c, &c->d_lin, kLinN + 2);
        if (rc) return rc;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_lut, tab.data(), sizeof(float4) * (kLutN + 2), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_lin, lin.data(), sizeof(float2) * (kLinN + 2), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->lut_k = K;
    return LMTOF_OK;
}

void launch_shape(const lmtof_ctx *c, int &block, int &ept) {
    block = kForwardBlock;
    ept = c->opt_ept > 0 ? c->opt_ept : kDefaultEpt;
}

// Upload a problem table (assigning chunk ranges) to *d (reallocated as needed).
// Lay out the problems' blocked image copies back to back in xb (n_xblk
// 4^3 blocks of 64 floats in total; xb may be NULL to only count them).
int64_t assign_xblocks(std::vector<Problem> &ps, float *xb) {
    int64_t n = 0;
    for (auto &P : ps) {
        P.xblk_begin = n;
        P.xb = xb ? xb + 64 * n : nullptr;
        n += xblocks(P);
    }
    return n;
}

int upload_problems(lmtof_ctx *c, std::vector<Problem> &ps, int block, int ept, Problem **d, int64_t &n_chunks,
                    int64_t &n_vchunks) {
    const int64_t ce = project_chunk_events(block, ept), cv = update_chunk_voxels();
    n_chunks = 0;
    n_vchunks = 0;
    int64_t nb = 0;
    for (auto &P : ps) {
        // the forward pass addresses a problem's blocked copy with 32-bit byte offsets
        if (xblocks(P) * 256 > 0xffffffffLL)
            return fail(c, LMTOF_EUNSUPPORTED, "grid too large: its blocked image copy exceeds 4 GiB");
        P.chunk_begin = n_chunks;
        P.vchunk_begin = n_vchunks;
        P.brick_base = (int32_t)nb;
        nb += (int64_t)P.nbx * P.nby * P.nbz;
        n_chunks += (P.n_events + ce - 1) / ce;
        n_vchunks += ((int64_t)P.nx * P.ny * P.nz + cv - 1) / cv;
    }
    if (n_chunks > 0x7fffffffLL) return fail(c, LMTOF_EUNSUPPORTED, "too many projector blocks (%lld)", (long long)n_chunks);
    if (nb > 0x7fffffffLL) return fail(c, LMTOF_EUNSUPPORTED, "too many bricks (%lld)", (long long)nb);
    if (!*d) {
        int rc = dev_alloc(c, d, kMaxProblems);
        if (rc) return rc;
    }
    HIPCHK(c, hipMemcpyAsync(*d, ps.data(), sizeof(Problem) * ps.size(), hipMemcpyHostToDevice, c->stream));
    return LMTOF_OK;
}

// Brick item lists for an uploaded problem batch: count pieces per brick,
// lay the lists out by brick and fill them on the GPU; then cut each list
// into chunks of at most C items (C grows with the total so there are
// ~8k chunks) and order the chunks largest first.  The chunk table is a
// launch schedule built on the host from the per-brick counts.
// Keep *p if it holds n elements already, else reallocate it.
template <class T>
int reserve(lmtof_ctx *c, T **p, size_t &cap, size_t n) {
    if (*p && cap >= n) return LMTOF_OK;
    dev_free(*p);
    cap = 0;
    int rc = dev_alloc(c, p, n);
    if (!rc) cap = std::max<size_t>(n, 1);
    return rc;
}

int build_items(lmtof_ctx *c, std::vector<Problem> &ps, Problem *d_probs, int64_t n_chunks, int ept,
                ItemSet &it) {
    // Every array is rebuilt in place and only reallocated when it has to
    // grow.  Until the build completes the set holds no lists.
    invalidate_items(it);
    uint64_t nb = 0;
    for (const auto &P : ps) nb += (uint64_t)P.nbx * P.nby * P.nbz;
    if (nb * kItemClasses >= 0xffffffffULL)
        return fail(c, LMTOF_EUNSUPPORTED, "%llu bricks of 16^3 voxels: too many for 32-bit (brick, class) keys",
                    (unsigned long long)nb);
    const uint64_t nk = nb * kItemClasses;  // (brick, item class) keys
    // per-event item offsets over the stored events the problems cover
    int64_t ne = 0;
    for (const auto &P : ps) ne = std::max<int64_t>(ne, P.ev_offset + P.n_events);
    Launch L;
    L.stream = c->stream;
    int rc;
    if ((rc = reserve(c, &it.cnt, it.cnt_cap, nk + 1)) ||
        (rc = reserve(c, &it.tabs, it.tabs_cap, (size_t)brick_item_tab_words(n_chunks))) ||
        (rc = reserve(c, &it.off_d, it.off_cap, nk + 1)) || (rc = reserve(c, &it.bwmax, it.bwmax_cap, nb)) ||
        (rc = reserve(c, &it.gflag, it.gflag_cap, ps.size())) ||
        (rc = reserve(c, &it.evoff, it.evoff_cap, (size_t)ne + 1)) ||
        (rc = reserve(c, &it.evflag, it.evflag_cap, (size_t)ne + 1)) ||
        (rc = reserve(c, &it.scan_tmp, it.scan_cap, (size_t)scan_tmp_elems(ne + 1))))
        return rc;
    for (auto &P : ps) {
        P.evoff = it.evoff + P.ev_offset;
        P.evflag = it.evflag + P.ev_offset;
        P.runs = it.tabs + P.chunk_begin * kTabWords;
        P.bwmax = it.bwmax + P.brick_base;
        P.gflag = it.gflag + (&P - ps.data());
    }
    std::vector<uint32_t> hk(nk);
    hipError_t he = hipMemcpyAsync(d_probs, ps.data(), sizeof(Problem) * ps.size(), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(it.cnt, 0, sizeof(uint32_t) * (nk + 1), c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(it.evoff, 0, sizeof(uint32_t) * ((size_t)ne + 1), c->stream);
    if (he == hipSuccess)
        he = launch_brick_items(L, d_probs, (int)ps.size(), n_chunks, ept, it.cnt, nullptr, 0, it.tabs);
    // each event's item count -> the first entry of its positions
    if (he == hipSuccess) he = launch_exclusive_scan(L, it.evoff, ne + 1, it.scan_tmp);
    if (he == hipSuccess) he = hipMemcpyAsync(hk.data(), it.cnt, sizeof(uint32_t) * nk, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return fail(c, LMTOF_EHIP, "brick item count: %s", hipGetErrorString(he));
    // a brick's items are its class ranges back to back
    std::vector<uint32_t> offk(nk + 1), h(nb), off(nb + 1);
    uint64_t tot = 0;
    for (uint64_t k = 0; k < nk; ++k) {
        if (k % kItemClasses == 0) {
            off[k / kItemClasses] = (uint32_t)std::min<uint64_t>(tot, 0xffffffffULL);
            h[k / kItemClasses] = 0;
        }
        offk[k] = (uint32_t)std::min<uint64_t>(tot, 0xffffffffULL);
        tot += hk[k];
        h[k / kItemClasses] += hk[k];
    }
    if (tot > 0xffffffffULL) return fail(c, LMTOF_EUNSUPPORTED, "more than 2^32-1 brick items");
    offk[nk] = (uint32_t)tot;
    off[nb] = (uint32_t)tot;
    const uint64_t D = (uint64_t)c->opt_bchunks;
    const uint64_t C = std::max<uint64_t>(2048, (tot + D - 1) / D);
    std::vector<uint4> chunks, bricks;
    uint32_t slot = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        if (!h[b]) continue;
        const uint32_t nch = (uint32_t)((h[b] + C - 1) / C);
        const uint32_t bi = (uint32_t)bricks.size();
        bricks.push_back(make_uint4((uint32_t)b, slot, slot + nch, h[b]));
        for (uint32_t q = 0; q < nch; ++q) {
            const uint32_t k0 = off[b] + (uint32_t)((uint64_t)h[b] * q / nch);
            const uint32_t k1 = off[b] + (uint32_t)((uint64_t)h[b] * (q + 1) / nch);
            chunks.push_back(make_uint4(bi, k0, k1, slot + q));
        }
        slot += nch;
    }
    std::stable_sort(chunks.begin(), chunks.end(),
                     [](const uint4 &a, const uint4 &b) { return (a.z - a.y) > (b.z - b.y); });
    if ((rc = reserve(c, &it.pw, it.pw_cap, tot)) || (rc = reserve(c, &it.evitems, it.evitems_cap, tot)) ||
        (rc = reserve(c, &it.itemslot, it.itemslot_cap, tot)) ||
        (rc = reserve(c, &it.chunks, it.chunks_cap, chunks.size())) ||
        (rc = reserve(c, &it.bricks, it.bricks_cap, bricks.size())) ||
        (rc = reserve(c, &it.tiles, it.tiles_cap, (size_t)slot * kBrickVox)) ||
        (rc = reserve(c, &it.item_recs, it.item_recs_cap, (size_t)tot * kItemRecBytes)))
        return rc;
    for (auto &P : ps) {
        P.pw = it.pw;
        P.itemslot = it.itemslot;
        P.n_items = (uint32_t)tot;
        P.evitems = it.evitems;
        P.tiles = it.tiles;
        P.rec_a = reinterpret_cast<const float4 *>(it.item_recs);
        P.rec_b = reinterpret_cast<const float4 *>(it.item_recs + (size_t)tot * 16);
    }
    he = hipMemcpyAsync(d_probs, ps.data(), sizeof(Problem) * ps.size(), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(it.off_d, offk.data(), sizeof(uint32_t) * (nk + 1), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess && !chunks.empty())
        he = hipMemcpyAsync(it.chunks, chunks.data(), sizeof(uint4) * chunks.size(), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess && !bricks.empty())
        he = hipMemcpyAsync(it.bricks, bricks.data(), sizeof(uint4) * bricks.size(), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(it.cnt, it.off_d, sizeof(uint32_t) * (nk + 1), hipMemcpyDeviceToDevice, c->stream);
    if (he == hipSuccess)
        he = launch_brick_items(L, d_probs, (int)ps.size(), n_chunks, ept, it.cnt, it.off_d + 1, 1, it.tabs);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return fail(c, LMTOF_EHIP, "brick item fill: %s", hipGetErrorString(he));
    it.n_chunks = (uint32_t)chunks.size();
    it.n_bricks = (uint32_t)bricks.size();
    it.n_slots = slot;
    it.n_items = tot;
    it.n_all_bricks = nb;
    it.item_bytes = (size_t)tot * kItemRecBytes;
    it.h_chunks = std::move(chunks);
    it.h_bricks = std::move(bricks);
    return LMTOF_OK;
}

// Back projection of each problem's weights P.rw into its b (as graph nodes
// after *prev, or on the stream).  In a graph, ev_a and ev_b (if given) are
// recorded right before and right after the brick kernel, to time it alone.
int add_back(lmtof_ctx *c, Launch L, const Problem *d_probs, int np, const ItemSet &it, hipGraphNode_t *prev,
             hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr) {
    const bool tof = c->g.tof_fwhm_ps > 0;
    hipGraphNode_t node = nullptr;
    if (L.graph) {
        L.deps = prev;
        L.n_deps = 1;
        L.node = &node;
    }
    auto record = [&](hipEvent_t ev) -> int {
        if (!L.graph || !ev) return LMTOF_OK;
        hipGraphNode_t n = nullptr;
        HIPCHK(c, hipGraphAddEventRecordNode(&n, L.graph, prev, 1, ev));
        *prev = n;
        L.deps = prev;
        return LMTOF_OK;
    };
    int rc;
    if ((rc = record(ev_a))) return rc;
    HIPCHK(c, launch_back_chunks(L, tof, d_probs, np, it.chunks, it.n_chunks, it.bricks));
    if (L.graph && it.n_chunks) {
        *prev = node;
        L.deps = prev;
    }
    if ((rc = record(ev_b))) return rc;
    HIPCHK(c, launch_reduce_tiles(L, d_probs, np, it.bricks, it.n_bricks));
    if (L.graph && it.n_bricks) *prev = node;
    return LMTOF_OK;
}

int ensure_rw(lmtof_ctx *c) {
    if ((size_t)c->n_events <= c->rw_cap) return LMTOF_OK;
    dev_free(c->d_rw);
    c->rw_cap = 0;
    int rc = dev_alloc(c, &c->d_rw, c->n_events);
    if (rc) return rc;
    c->rw_cap = c->n_events;
    return LMTOF_OK;
}

// (Re)build the batch the iteration runs: the whole volume, or one problem per region.
int ensure_problems(lmtof_ctx *c) {
    if (!c->probs_dirty) return LMTOF_OK;
    drop_graphs(c);
    int rc0 = ensure_lut(c);
    if (rc0) return rc0;
    if ((rc0 = ensure_rw(c))) return rc0;
    std::vector<Problem> ps;
    const size_t esz = c->stored_packed ? 16 : 32;
    if (c->regions.empty()) {
        Problem P = make_problem(c, 0, c->g.nz, c->d_x, c->d_b, c->d_s);
        P.events = c->d_events;
        P.n_events = c->n_events;
        P.ev_offset = 0;
        P.rw = c->d_rw;
        ps.push_back(P);
    } else {
        for (auto &r : c->regions) {
            Problem P = make_problem(c, r.z_lo, r.nz, r.x, r.b, r.s);
            P.events = (const char *)c->d_events + esz * r.ev_offset;
            P.n_events = r.n_events;
            P.ev_offset = r.ev_offset;
            P.rw = c->d_rw + r.ev_offset;
            ps.push_back(P);
        }
    }
    int block, ept;
    launch_shape(c, block, ept);
    const int64_t nxb = assign_xblocks(ps, nullptr);
    int rc = reserve(c, &c->d_xb, c->xb_cap, (size_t)nxb * 64);
    if (rc) return rc;
    // padding blocks of the blocked copies stay 0 (the relayout skips them)
    HIPCHK(c, hipMemsetAsync(c->d_xb, 0, sizeof(float) * 64 * (size_t)nxb, c->stream));
    c->n_xblk = assign_xblocks(ps, c->d_xb);
    if ((rc = upload_problems(c, ps, block, ept, &c->d_probs, c->n_chunks, c->n_vchunks))) return rc;
    if ((rc = build_items(c, ps, c->d_probs, c->n_chunks, ept, c->items))) return rc;
    c->probs = ps;
    c->ept_used = ept;
    if (c->has_evw) {
        // the ratio weights in stored order, applied where the ratios are
        // written to the items
        if ((rc = reserve(c, &c->d_evw, c->evw_stored_cap, (size_t)c->n_events))) return rc;
        Launch Lw;
        Lw.stream = c->stream;
        HIPCHK(c, launch_gather_by_perm(Lw, c->d_evw_caller, c->d_perm, c->n_events, c->d_evw));
        for (auto &P : ps) P.evw = c->d_evw + P.ev_offset;
        HIPCHK(c, hipMemcpyAsync(c->d_probs, ps.data(), sizeof(Problem) * ps.size(), hipMemcpyHostToDevice, c->stream));
        c->probs = ps;
    }
    if ((size_t)c->n_chunks > c->part_cap) {
        dev_free(c->d_part_neff);
        dev_free(c->d_part_ll);
        c->part_cap = 0;
        if ((rc = dev_alloc(c, &c->d_part_neff, c->n_chunks))) return rc;
        if ((rc = dev_alloc(c, &c->d_part_ll, c->n_chunks))) return rc;
        c->part_cap = c->n_chunks;
    }
    if ((size_t)c->n_vchunks > c->vpart_cap) {
        dev_free(c->d_part_old);
        dev_free(c->d_part_new);
        c->vpart_cap = 0;
        if ((rc = dev_alloc(c, &c->d_part_old, c->n_vchunks))) return rc;
        if ((rc = dev_alloc(c, &c->d_part_new, c->n_vchunks))) return rc;
        c->vpart_cap = c->n_vchunks;
    }
    c->probs_dirty = false;
    return LMTOF_OK;
}

int ensure_stats(lmtof_ctx *c, size_t n) {
    if (n <= c->stats_cap) return LMTOF_OK;
    dev_free(c->d_stats);
    c->stats_cap = 0;
    int rc = dev_alloc(c, &c->d_stats, n);
    if (rc) return rc;
    c->stats_cap = n;
    return LMTOF_OK;
}

// Forward stage of an MLEM iteration over the batch (graph nodes after
// *prev, or on the stream): the brick-owned forward pass and the combine
// pass (ratios written to the items), or the event-parallel pass and the
// pass that writes its ratios to the items.  ev_mid (graphs only) is
// recorded between the two.
int add_forward(lmtof_ctx *c, Launch L, const Problem *d_probs, int np, int64_t n_chunks, int64_t n_xblk,
                const ItemSet &it, int ept, int *part_neff, double *part_ll, hipGraphNode_t *prev,
                hipEvent_t ev_mid = nullptr) {
    const bool tof = c->g.tof_fwhm_ps > 0;
    hipGraphNode_t node = nullptr;
    auto chain = [&]() {
        if (L.graph && node) *prev = node;
        L.deps = prev;
        node = nullptr;
    };
    if (L.graph) {
        L.deps = prev;
        L.n_deps = 1;
        L.node = &node;
    }
    if (c->opt_forward == LMTOF_FORWARD_BRICKS) {
        HIPCHK(c, launch_forward_items(L, tof, d_probs, np, it.chunks, it.n_chunks, it.bricks));
        chain();
    } else {
        HIPCHK(c, launch_block_image(L, d_probs, np, n_xblk));
        chain();
        HIPCHK(c, launch_forward(L, tof, d_probs, np, n_chunks, ept, 0, part_neff, part_ll));
        chain();
    }
    HIPCHK(c, launch_clear_bwmax(L, d_probs, np, (int64_t)it.n_all_bricks));
    chain();
    if (L.graph && ev_mid) {
        hipGraphNode_t n = nullptr;
        HIPCHK(c, hipGraphAddEventRecordNode(&n, L.graph, prev, 1, ev_mid));
        *prev = n;
        L.deps = prev;
    }
    HIPCHK(c, launch_combine(L, d_probs, np, n_chunks, ept,
                             c->opt_forward == LMTOF_FORWARD_BRICKS ? kCombineRatio : kCombineWeights, part_neff,
                             part_ll));
    chain();
    HIPCHK(c, launch_brick_wmax(L, d_probs, np, it.chunks, it.n_chunks, it.bricks));
    chain();
    return LMTOF_OK;
}

// n_iter MLEM iterations as one explicit HIP graph.  Per iteration: event
// record, forward kernel, event record, combine, event record, brick
// scales, event record, brick back projection, event record, tile
// reduction, event record, update, finalize (stats of iteration k into
// slot k), [median sieve], event record.
int build_graph(lmtof_ctx *c, int n_iter, GraphEntry &ge) {
    const int np = (int)c->probs.size();
    HIPCHK(c, hipGraphCreate(&ge.graph, 0));
    ge.ev.assign(kEventsPerIter * n_iter, nullptr);
    for (auto &e : ge.ev) HIPCHK(c, hipEventCreate(&e));
    hipGraphNode_t prev = nullptr;
    bool have_prev = false;
    auto record = [&](hipEvent_t ev) -> int {
        hipGraphNode_t n = nullptr;
        HIPCHK(c, hipGraphAddEventRecordNode(&n, ge.graph, have_prev ? &prev : nullptr, have_prev ? 1 : 0, ev));
        prev = n;
        have_prev = true;
        return LMTOF_OK;
    };
    for (int k = 0; k < n_iter; ++k) {
        int rc;
        hipEvent_t *e = &ge.ev[(size_t)kEventsPerIter * k];
        if ((rc = record(e[0]))) return rc;
        Launch L;
        L.graph = ge.graph;
        if ((rc = add_forward(c, L, c->d_probs, np, c->n_chunks, c->n_xblk, c->items, c->ept_used, c->d_part_neff,
                              c->d_part_ll, &prev, e[1])))
            return rc;
        if ((rc = record(e[2]))) return rc;
        if ((rc = add_back(c, L, c->d_probs, np, c->items, &prev, e[3], e[4])))
            return rc;
        if ((rc = record(e[5]))) return rc;
        hipGraphNode_t node = nullptr;
        L.deps = &prev;
        L.n_deps = 1;
        L.node = &node;
        HIPCHK(c, launch_update(L, c->d_probs, np, c->n_vchunks, c->d_part_old, c->d_part_new));
        if (node) prev = node;
        L.deps = &prev;
        node = nullptr;
        HIPCHK(c, launch_finalize(L, c->d_probs, np, c->n_chunks, c->n_vchunks, c->d_part_neff, c->d_part_ll,
                                  c->d_part_old, c->d_part_new, c->d_stats, k));
        if (node) prev = node;
        if (c->opt_median) {
            // median sieve of each problem's image, through its (cleared) b
            for (const auto &P : c->probs) {
                L.deps = &prev;
                node = nullptr;
                HIPCHK(c, launch_median3(L, P.x, P.b, P.nx, P.ny, P.nz));
                if (node) prev = node;
                L.deps = &prev;
                node = nullptr;
                HIPCHK(c, launch_take_clear(L, P.x, P.b, (int64_t)P.nx * P.ny * P.nz));
                if (node) prev = node;
            }
        }
        if ((rc = record(e[6]))) return rc;
    }
    HIPCHK(c, hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
    return LMTOF_OK;
}

int copy_in(lmtof_ctx *c, void *dst, const void *src, size_t bytes, int mem) {
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, mem == LMTOF_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                             c->stream));
    return LMTOF_OK;
}

int copy_out(lmtof_ctx *c, void *dst, const void *src, size_t bytes, int mem) {
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, mem == LMTOF_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LMTOF_OK;
}

bool valid_mem(int mem) { return mem == LMTOF_MEM_HOST || mem == LMTOF_MEM_DEVICE; }

int check_geometry(lmtof_ctx *c, const lmtof_geometry &g) {
    auto fin = [](double v) { return std::isfinite(v); };
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) return fail(c, LMTOF_EINVAL, "grid size must be >= 1 per axis");
    if ((int64_t)g.nx * g.ny * g.nz > 0x7fffffffLL) return fail(c, LMTOF_EINVAL, "grid has more than 2^31-1 voxels");
    if (g.reserved0 != 0) return fail(c, LMTOF_EINVAL, "reserved0 must be 0");
    if (!(g.vx > 0 && g.vy > 0 && g.vz > 0 && fin(g.vx) && fin(g.vy) && fin(g.vz)))
        return fail(c, LMTOF_EINVAL, "voxel sizes must be finite and > 0");
    if (!(fin(g.x0) && fin(g.y0) && fin(g.z0))) return fail(c, LMTOF_EINVAL, "grid corner must be finite");
    if (!(g.scanner_radius > 0 && g.scanner_half_length > 0 && fin(g.scanner_radius) && fin(g.scanner_half_length)))
        return fail(c, LMTOF_EINVAL, "scanner radius and half length must be finite and > 0");
    if (!(g.max_axial_angle_deg >= 0 && g.max_axial_angle_deg < 90))
        return fail(c, LMTOF_EINVAL, "max_axial_angle_deg must be in [0, 90)");
    if (!fin(g.tof_fwhm_ps)) return fail(c, LMTOF_EINVAL, "tof_fwhm_ps must be finite");
    if (!(g.tof_trunc_sigmas >= 0 && g.tof_trunc_sigmas <= 10))
        return fail(c, LMTOF_EINVAL, "tof_trunc_sigmas must be in [0, 10] (0 = default 3)");
    if (!(g.c_mm_per_ps >= 0 && fin(g.c_mm_per_ps))) return fail(c, LMTOF_EINVAL, "c_mm_per_ps must be >= 0");
    // grid inside the scanner cylinder
    const double R = g.scanner_radius, H = g.scanner_half_length;
    const double xs[2] = {g.x0, g.x0 + g.nx * g.vx}, ys[2] = {g.y0, g.y0 + g.ny * g.vy};
    for (double x : xs)
        for (double y : ys)
            if (std::hypot(x, y) > R * (1 + 1e-12))
                return fail(c, LMTOF_EINVAL, "grid corner (%g, %g) lies outside the scanner radius %g", x, y, R);
    if (g.z0 < -H * (1 + 1e-12) || g.z0 + g.nz * g.vz > H * (1 + 1e-12))
        return fail(c, LMTOF_EINVAL, "grid z range lies outside the scanner (|z| <= %g)", H);
    return LMTOF_OK;
}

KeyGeom key_geom(const lmtof_ctx *c, bool sort, const std::vector<Region> &regions) {
    const lmtof_geometry &g = c->g;
    KeyGeom k{};
    k.ox = (float)g.x0;
    k.oy = (float)g.y0;
    k.oz = (float)g.z0;
    // direction bins: 4 azimuth x 2 elevation (finer bins made the walks no
    // faster and the combine pass slower; coarser ones, or one bin, put
    // more events on each sort key, whose atomics then contend at load)
    k.n_phi = 4;
    k.n_lam = 2;
    k.sort = sort ? 1 : 0;
    k.tof = g.tof_fwhm_ps > 0;
    k.half_c = (float)(g.c_mm_per_ps / 2.0);
    k.bx_inv = (float)(1.0 / (kBrickX * g.vx));
    k.by_inv = (float)(1.0 / (kBrickY * g.vy));
    k.bz_inv = (float)(1.0 / (kBrickZ * g.vz));
    k.ncx = (g.nx + kBrickX - 1) / kBrickX;
    k.ncy = (g.ny + kBrickY - 1) / kBrickY;
    int nzb = g.nz;
    if (!regions.empty()) {
        nzb = 0;
        for (const auto &r : regions) nzb = std::max(nzb, r.nz);
    }
    k.ncz = (nzb + kBrickZ - 1) / kBrickZ;
    // sub-cells of about the requested cell size, fewer if the key space grows too large
    auto nsub = [&](double brick_mm) { return std::max(1, std::min(16, (int)std::lround(brick_mm / c->opt_cell_mm))); };
    k.nsx = nsub(kBrickX * g.vx);
    k.nsy = nsub(kBrickY * g.vy);
    k.nsz = nsub(kBrickZ * g.vz);
    const double nr = std::max<size_t>(1, regions.size());
    while ((double)k.ncx * k.ncy * k.ncz * k.n_phi * k.n_lam * k.nsx * k.nsy * k.nsz * nr > (double)(1 << 26)) {
        if (k.nsx * k.nsy * k.nsz > 1) {
            k.nsx = std::max(1, k.nsx / 2);
            k.nsy = std::max(1, k.nsy / 2);
            k.nsz = std::max(1, k.nsz / 2);
        } else {
            k.n_phi = std::max(1, k.n_phi / 2);
            k.n_lam = std::max(1, k.n_lam / 2);
            if (k.n_phi == 1 && k.n_lam == 1) break;
        }
    }
    k.n_regions = (int)regions.size();
    for (size_t r = 0; r < regions.size(); ++r) {
        k.region_z[r] = (float)(g.z0 + regions[r].core_lo * g.vz);
        k.region_z0[r] = (float)(g.z0 + regions[r].z_lo * g.vz);
    }
    if (!regions.empty()) k.region_z[regions.size()] = (float)(g.z0 + regions.back().core_hi * g.vz);
    return k;
}

// Device bytes a prepared context holds (events, permutation, per-event
// weights, brick lists and tiles, images, partials).
int64_t ctx_device_bytes(const lmtof_ctx *c) {
    const ItemSet &it = c->items;
    int64_t b = (int64_t)(c->events_cap + c->perm_cap) + (int64_t)c->rw_cap * 4 + 3 * 4 * (int64_t)c->img_cap;
    for (const Scratch *sc : {&c->sc_events, &c->sc_perm, &c->sc_keys, &c->sc_hist, &c->sc_tmp, &c->sc_err,
                              &c->sc_inner, &c->sc_reg, &c->sc_raw})
        b += (int64_t)sc->cap;
    b += (int64_t)c->reg_cap;
    b += (int64_t)(it.pw_cap + it.evitems_cap + it.evoff_cap + it.scan_cap) * 4 + (int64_t)it.itemslot_cap * 2 +
         (int64_t)it.evflag_cap + (int64_t)it.item_recs_cap +
         (int64_t)it.tiles_cap * 8;
    b += (int64_t)(it.chunks_cap + it.bricks_cap) * 16;
    b += (int64_t)(it.bwmax_cap + it.gflag_cap + it.cnt_cap + it.off_cap + it.tabs_cap) * 4;
    b += (int64_t)(c->evw_cap + c->evw_stored_cap) * 4;
    b += (int64_t)c->part_cap * 12 + (int64_t)c->vpart_cap * 16 + (kLutN + 2) * 16 + (kLinN + 2) * 8 + (int64_t)c->xb_cap * 4;
    return b;
}

// Footprint the pool reserves for a request: stored events, permutation,
// weights, ~ (1 + 1.7 * window / brick edge) brick items per event (walk
// record, weight, position) plus tiles, three images, and the transient ingest
// buffers (raw copy, keys, sort histogram).
int64_t request_bytes_estimate(const lmtof_request &q) {
    const lmtof_geometry &g = q.geometry;
    const int64_t V = (int64_t)g.nx * g.ny * g.nz;
    const int64_t N = q.n_events;
    const double c = g.c_mm_per_ps > 0 ? g.c_mm_per_ps : kDefaultC;
    const double K = g.tof_trunc_sigmas > 0 ? g.tof_trunc_sigmas : 3.0;
    const double vmin = std::min(g.vx, std::min(g.vy, g.vz));
    double win;
    if (g.tof_fwhm_ps > 0)
        win = 2.0 * K * (c * g.tof_fwhm_ps / 2.0) / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    else
        win = std::sqrt(std::pow(g.nx * g.vx, 2) + std::pow(g.ny * g.vy, 2) + std::pow(g.nz * g.vz, 2));
    const double ipe = 1.3 * (1.0 + 1.7 * win / (kBrickX * vmin));
    const int64_t items = (int64_t)(N * ipe);
    const int64_t esz = q.storage ? 16 : 32;
    auto pow2 = [](int64_t n) {
        int64_t q2 = 1;
        while (q2 < n) q2 <<= 1;
        return q2;
    };
    const int64_t xbv = pow2((g.nx + 3) / 4) * pow2((g.ny + 3) / 4) * ((g.nz + 3) / 4) * 64;  // blocked copy of x
    // per event: store, permutation, weight, item offset, flag; per item:
    // walk record, weight, position in its event's list, combine slot;
    // x, b, s, blocked x
    int64_t b = N * (esz + 8 + 4 + 4 + 1) + items * (10 + kItemRecBytes) + 3 * 4 * V + 4 * xbv;
    b += (items / 2048 + 1 + V / kBrickVox + 1) * (int64_t)kBrickVox * 8 / 4;  // tiles
    const int64_t nbr = (int64_t)((g.nx + kBrickX - 1) / kBrickX) * ((g.ny + kBrickY - 1) / kBrickY) *
                        ((g.nz + kBrickZ - 1) / kBrickZ);
    b += nbr * (4 + 4 * kItemClasses * 2);  // per brick: maximum; builder counters and offsets
    // the forward chunks' key tables, then run rows (kTabWords words per
    // chunk of kForwardBlock x kDefaultEpt events), kept for the iterations
    b += (N + kForwardBlock * kDefaultEpt - 1) / (kForwardBlock * kDefaultEpt) * kTabWords * 4;
    // transients of the ingest
    b += N * (q.mem == LMTOF_MEM_HOST ? 28 : 0) + N * (esz + 8 + 4);
    return b + (64 << 20);
}

}  // namespace

// =====================================================================  C ABI
extern "C" {

int lmtof_create(lmtof_ctx **out, int hip_device, void *hip_stream) {
    if (!out) {
        g_create_err = "out is NULL";
        return LMTOF_EINVAL;
    }
    *out = nullptr;
    try {
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess || ndev < 1) {
            g_create_err = std::string("no HIP device: ") + hipGetErrorString(e);
            return LMTOF_EHIP;
        }
        if (hip_device < 0 || hip_device >= ndev) {
            g_create_err = "hip_device out of range";
            return LMTOF_EINVAL;
        }
        e = hipSetDevice(hip_device);
        if (e != hipSuccess) {
            g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(e);
            return LMTOF_EHIP;
        }
        if (hip_device >= kMaxDevices) {
            g_create_err = "hip_device beyond the supported device count";
            return LMTOF_EUNSUPPORTED;
        }
        {
            // this device's copy of the allocation-free entry point's scratch
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            if (!g_scratch_ptr[hip_device]) {
                void *p = nullptr;
                e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
                if (e != hipSuccess || !p) {
                    g_create_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                    return LMTOF_EHIP;
                }
                g_scratch_ptr[hip_device] = static_cast<float *>(p);
            }
        }
        lmtof_ctx *c = new lmtof_ctx();
        c->device = hip_device;
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                delete c;
                g_create_err = std::string("hipStreamCreate: ") + hipGetErrorString(e);
                return LMTOF_EHIP;
            }
            c->own_stream = true;
        }
        *out = c;
        g_create_err.clear();
        return LMTOF_OK;
    } catch (...) {
        g_create_err = "host allocation failed";
        return LMTOF_ENOMEM;
    }
}

int lmtof_destroy(lmtof_ctx *c) {
    if (!c) return LMTOF_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_events(c);
    free_items(c->items);
    dev_free(c->d_events);
    dev_free(c->d_perm);
    dev_free(c->reg_buf);
    scratch_free(c->sc_reg);
    dev_free(c->d_s);
    dev_free(c->d_x);
    dev_free(c->d_b);
    dev_free(c->d_xb);
    release_load_scratch(c);
    dev_free(c->d_probs);
    dev_free(c->d_part_neff);
    dev_free(c->d_part_ll);
    dev_free(c->d_part_old);
    dev_free(c->d_part_new);
    dev_free(c->d_stats);
    dev_free(c->d_scratch);
    dev_free(c->d_rw);
    dev_free(c->d_evw);
    dev_free(c->d_evw_caller);
    dev_free(c->d_lut);
    dev_free(c->d_lin);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LMTOF_OK;
}

const char *lmtof_last_error(const lmtof_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int lmtof_check_geometry(const lmtof_geometry *gin, char *msg, int64_t msg_len) {
    lmtof_ctx tmp;
    int rc = LMTOF_EINVAL;
    if (!gin) {
        tmp.err = "geometry is NULL";
    } else {
        lmtof_geometry g = *gin;
        if (g.tof_trunc_sigmas == 0) g.tof_trunc_sigmas = 3.0;
        if (g.c_mm_per_ps == 0) g.c_mm_per_ps = kDefaultC;
        rc = check_geometry(&tmp, g);
    }
    if (msg && msg_len > 0) {
        const std::string &m = rc == LMTOF_OK ? std::string() : tmp.err;
        const size_t k = std::min<size_t>(m.size(), (size_t)msg_len - 1);
        memcpy(msg, m.data(), k);
        msg[k] = 0;
    }
    return rc;
}

int lmtof_set_option(lmtof_ctx *c, int key, int64_t v) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    switch (key) {
    case LMTOF_OPT_STORAGE:
        if (v != 0 && v != 1) return fail(c, LMTOF_EINVAL, "storage must be 0 (plain) or 1 (packed)");
        c->opt_storage = (int)v;
        return LMTOF_OK;
    case LMTOF_OPT_SORT:
        if (v != 0 && v != 1) return fail(c, LMTOF_EINVAL, "sort must be 0 or 1");
        c->opt_sort = (int)v;
        return LMTOF_OK;
    case LMTOF_OPT_SENS_NPHI:
        if (v < 4 || v > 4096) return fail(c, LMTOF_EINVAL, "sensitivity azimuth nodes must be in [4, 4096]");
        c->opt_nphi = (int)v;
        return LMTOF_OK;
    case LMTOF_OPT_EVENTS_PER_THREAD:
        if (v < 0 || v > 16) return fail(c, LMTOF_EINVAL, "events per thread must be in [0, 16]");
        c->opt_ept = (int)v;
        c->probs_dirty = true;
        return LMTOF_OK;
    case LMTOF_OPT_SORT_CELL_MM:
        if (v < 1 || v > 10000) return fail(c, LMTOF_EINVAL, "sort cell must be in [1, 10000] mm");
        c->opt_cell_mm = (double)v;
        return LMTOF_OK;
    case LMTOF_OPT_MEDIAN_SIEVE:
        if (v != 0 && v != 1) return fail(c, LMTOF_EINVAL, "median sieve must be 0 or 1");
        if ((int)v != c->opt_median) drop_graphs_only(c);  // the brick lists stay
        c->opt_median = (int)v;
        return LMTOF_OK;
    case LMTOF_OPT_BRICK_CHUNKS:
        if (v < 256 || v > 65536) return fail(c, LMTOF_EINVAL, "brick chunks must be in [256, 65536]");
        if ((int)v != c->opt_bchunks) c->probs_dirty = true;
        c->opt_bchunks = (int)v;
        return LMTOF_OK;
    case LMTOF_OPT_FORWARD:
        if (v != LMTOF_FORWARD_BRICKS && v != LMTOF_FORWARD_EVENTS)
            return fail(c, LMTOF_EINVAL, "forward projector must be LMTOF_FORWARD_BRICKS or LMTOF_FORWARD_EVENTS");
        if ((int)v != c->opt_forward) drop_graphs_only(c);  // the brick lists stay
        c->opt_forward = (int)v;
        return LMTOF_OK;
    default:
        return fail(c, LMTOF_EINVAL, "unknown option %d", key);
    }
}

int lmtof_get_option(const lmtof_ctx *c, int key, int64_t *v) {
    if (!c || !v) return LMTOF_EINVAL;
    switch (key) {
    case LMTOF_OPT_STORAGE: *v = c->opt_storage; return LMTOF_OK;
    case LMTOF_OPT_SORT: *v = c->opt_sort; return LMTOF_OK;
    case LMTOF_OPT_SENS_NPHI: *v = c->opt_nphi; return LMTOF_OK;
    case LMTOF_OPT_EVENTS_PER_THREAD: *v = c->opt_ept > 0 ? c->opt_ept : kDefaultEpt; return LMTOF_OK;
    case LMTOF_OPT_SORT_CELL_MM: *v = (int64_t)c->opt_cell_mm; return LMTOF_OK;
    case LMTOF_OPT_MEDIAN_SIEVE: *v = c->opt_median; return LMTOF_OK;
    case LMTOF_OPT_FORWARD: *v = c->opt_forward; return LMTOF_OK;
    case LMTOF_OPT_BRICK_CHUNKS: *v = c->opt_bchunks; return LMTOF_OK;
    default: return LMTOF_EINVAL;
    }
}

int lmtof_set_geometry(lmtof_ctx *c, const lmtof_geometry *gin) {
    if (!c) return LMTOF_EINVAL;
    if (!gin) return fail(c, LMTOF_EINVAL, "geometry is NULL");
    c->err.clear();
    lmtof_geometry g = *gin;
    if (g.tof_trunc_sigmas == 0) g.tof_trunc_sigmas = 3.0;
    if (g.c_mm_per_ps == 0) g.c_mm_per_ps = kDefaultC;
    int rc = check_geometry(c, g);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    try {
        const int64_t V = (int64_t)g.nx * g.ny * g.nz;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if ((size_t)V > c->img_cap) {
            // grow: the new images are allocated before the old ones go
            float *s = nullptr, *x = nullptr, *b = nullptr;
            if ((rc = dev_alloc(c, &s, V))) return rc;
            if ((rc = dev_alloc(c, &x, V))) { dev_free(s); return rc; }
            if ((rc = dev_alloc(c, &b, V))) { dev_free(s); dev_free(x); return rc; }
            dev_free(c->d_s);
            dev_free(c->d_x);
            dev_free(c->d_b);
            c->d_s = s;
            c->d_x = x;
            c->d_b = b;
            c->img_cap = (size_t)V;
        }
        drop_events(c);
        c->g = g;
        c->V = V;
        c->has_geom = true;
        c->has_sens = false;
        c->has_image = false;
        c->probs_dirty = true;
        Launch L;
        L.stream = c->stream;
        HIPCHK(c, launch_fill(L, c->d_b, V, 0.0f));
        HIPCHK(c, launch_fill(L, c->d_x, V, 0.0f));
        HIPCHK(c, launch_fill(L, c->d_s, V, 0.0f));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LMTOF_OK;
    } catch (...) {
        return fail(c, LMTOF_ENOMEM, "host allocation failed");
    }
}

int lmtof_load_events(lmtof_ctx *c, const void *ev, int64_t n, int format, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_geom) return fail(c, LMTOF_ESTATE, "set the geometry before loading events");
    if (!ev) return fail(c, LMTOF_EINVAL, "events pointer is NULL");
    if (n < 1 || n > (int64_t)0xffffffffLL) return fail(c, LMTOF_EINVAL, "event count must be in [1, 2^32-1]");
    if (format != LMTOF_FMT_F32X7 && format != LMTOF_FMT_PACKED16) return fail(c, LMTOF_EINVAL, "unknown format %d", format);
    if (!valid_mem(mem)) return fail(c, LMTOF_EINVAL, "unknown memory kind %d", mem);
    HIPCHK(c, hipSetDevice(c->device));
    const size_t raw_sz = format == LMTOF_FMT_F32X7 ? 28 : 16;
    const int packed = c->opt_storage;
    const size_t st_sz = packed ? 16 : 32;
    Launch L;
    L.stream = c->stream;
    int rc;
    void *raw = nullptr;
    char *store = nullptr;
    int64_t *perm = nullptr;
    uint32_t *keys = nullptr, *hist = nullptr, *tmp = nullptr, *err = nullptr;
    auto cleanup = [&]() { (void)hipStreamSynchronize(c->stream); };
    if (mem == LMTOF_MEM_HOST) {
        if ((rc = take(c, c->sc_raw, (char **)&raw, raw_sz * n))) return rc;
        if ((rc = copy_in(c, raw, ev, raw_sz * n, LMTOF_MEM_HOST))) { cleanup(); return rc; }
    } else {
        raw = const_cast<void *>(ev);
    }
    // the current events stay valid until the new ones are complete
    if ((rc = take(c, c->sc_events, &store, st_sz * n)) || (rc = take(c, c->sc_perm, &perm, n)) ||
        (rc = take(c, c->sc_err, &err, 1))) {
        cleanup();
        return rc;
    }
    hipError_t he = hipMemsetAsync(err, 0, sizeof(uint32_t), c->stream);
    const bool sort = c->opt_sort != 0;
    // events are loaded unsplit; lmtof_set_regions re-sorts by region
    KeyGeom kg = key_geom(c, sort, std::vector<Region>());
    uint32_t nkeys = key_count(kg);
    if (he == hipSuccess && sort) {
        if ((rc = take(c, c->sc_keys, &keys, n)) || (rc = take(c, c->sc_hist, &hist, nkeys)) ||
            (rc = take(c, c->sc_tmp, &tmp, scan_tmp_elems(nkeys)))) {
            cleanup();
            return rc;
        }
        he = hipMemsetAsync(hist, 0, sizeof(uint32_t) * nkeys, c->stream);
    }
    if (he == hipSuccess) he = launch_ingest_keys(L, raw, format, n, kg, packed, sort ? keys : nullptr, hist, err);
    if (he == hipSuccess && sort) he = launch_exclusive_scan(L, hist, nkeys, tmp);
    uint32_t herr = 0;
    if (he == hipSuccess) he = hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) {
        cleanup();
        return fail(c, LMTOF_EHIP, "event ingest: %s", hipGetErrorString(he));
    }
    if (herr) {
        cleanup();
        std::string why;
        if (herr & 1) why += " non-finite value;";
        if (herr & 2) why += " coincident endpoints;";
        if (herr & 4) why += " coordinate outside int16 range at 0.1 mm;";
        if (herr & 8) why += " dt outside the binary16 range;";
        return fail(c, LMTOF_EINVAL, "invalid events:%s", why.c_str());
    }
    he = launch_scatter_events(L, raw, format, n, sort ? keys : nullptr, sort ? hist : nullptr, packed, store, perm);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) {
        cleanup();
        return fail(c, LMTOF_EHIP, "event scatter: %s", hipGetErrorString(he));
    }
    c->has_image = false;
    drop_regions(c);
    drop_graphs(c);
    install_events(c);
    c->has_evw = false;  // weights belong to the previous events
    c->n_events = n;
    c->stored_packed = packed;
    c->probs_dirty = true;
    cleanup();
    return LMTOF_OK;
}

int lmtof_num_events(const lmtof_ctx *c, int64_t *n) {
    if (!c || !n) return LMTOF_EINVAL;
    *n = c->n_events;
    return LMTOF_OK;
}

int lmtof_read_packed_events(lmtof_ctx *c, void *out, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events || !c->stored_packed) return fail(c, LMTOF_ESTATE, "no packed events are loaded");
    if (!out || n != c->n_events || !valid_mem(mem)) return fail(c, LMTOF_EINVAL, "need n = %lld and a buffer", (long long)c->n_events);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    uint4 *tmp = nullptr;
    int rc;
    if (mem == LMTOF_MEM_HOST && (rc = dev_alloc(c, &tmp, n))) return rc;
    uint4 *dst = mem == LMTOF_MEM_HOST ? tmp : (uint4 *)out;
    hipError_t he = launch_unpermute_packed(L, (const uint4 *)c->d_events, c->d_perm, n, dst);
    if (he != hipSuccess) { dev_free(tmp); return fail(c, LMTOF_EHIP, "unpermute: %s", hipGetErrorString(he)); }
    rc = mem == LMTOF_MEM_HOST ? copy_out(c, out, tmp, 16 * n, LMTOF_MEM_HOST)
                               : (hipStreamSynchronize(c->stream) == hipSuccess ? LMTOF_OK : LMTOF_EHIP);
    dev_free(tmp);
    return rc;
}

int lmtof_compute_sensitivity(lmtof_ctx *c) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_geom) return fail(c, LMTOF_ESTATE, "set the geometry first");
    HIPCHK(c, hipSetDevice(c->device));
    const lmtof_geometry &g = c->g;
    SensGeom sg{};
    sg.nx = g.nx;
    sg.ny = g.ny;
    sg.nz = g.nz;
    sg.n_phi = c->opt_nphi;
    sg.ox = g.x0;
    sg.oy = g.y0;
    sg.oz = g.z0;
    sg.vx = g.vx;
    sg.vy = g.vy;
    sg.vz = g.vz;
    sg.R = g.scanner_radius;
    sg.H = g.scanner_half_length;
    sg.tan_lmax = g.max_axial_angle_deg > 0 ? std::tan(g.max_axial_angle_deg * M_PI / 180.0) : 0.0;
    Launch L;
    L.stream = c->stream;
    HIPCHK(c, launch_sensitivity(L, sg, c->d_s));
    const int64_t plane = (int64_t)g.nx * g.ny;
    for (auto &r : c->regions) HIPCHK(c, launch_copy_slab(L, c->d_s, plane, r.z_lo, r.nz, r.s));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_sens = true;
    c->has_image = false;
    return LMTOF_OK;
}

int lmtof_read_sensitivity(lmtof_ctx *c, float *out, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_sens) return fail(c, LMTOF_ESTATE, "no sensitivity yet");
    if (!out || n != c->V || !valid_mem(mem)) return fail(c, LMTOF_EINVAL, "need n = %lld floats", (long long)c->V);
    HIPCHK(c, hipSetDevice(c->device));
    return copy_out(c, out, c->d_s, sizeof(float) * n, mem);
}

int lmtof_set_sensitivity(lmtof_ctx *c, const float *s, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_geom) return fail(c, LMTOF_ESTATE, "set the geometry first");
    if (!s || n != c->V || !valid_mem(mem)) return fail(c, LMTOF_EINVAL, "need n = %lld floats", (long long)c->V);
    if (mem == LMTOF_MEM_HOST)
        for (int64_t j = 0; j < n; ++j)
            if (!(s[j] >= 0.0f) || !std::isfinite(s[j])) return fail(c, LMTOF_EINVAL, "sensitivity must be finite and >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = copy_in(c, c->d_s, s, sizeof(float) * n, mem);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_sens = true;
    c->has_image = false;
    drop_regions(c);
    return LMTOF_OK;
}

int lmtof_set_image(lmtof_ctx *c, const float *x0, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events || !c->has_sens) return fail(c, LMTOF_ESTATE, "load events and compute the sensitivity first");
    if (x0 && (n != c->V || !valid_mem(mem))) return fail(c, LMTOF_EINVAL, "need n = %lld floats", (long long)c->V);
    if (x0 && mem == LMTOF_MEM_HOST)
        for (int64_t j = 0; j < n; ++j)
            if (!(x0[j] >= 0.0f) || !std::isfinite(x0[j])) return fail(c, LMTOF_EINVAL, "image must be finite and >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = ensure_problems(c);
    if (rc) return rc;
    if (!c->d_scratch && (rc = dev_alloc(c, &c->d_scratch, 1025))) return rc;
    Launch L;
    L.stream = c->stream;
    for (size_t p = 0; p < c->probs.size(); ++p) {
        const Problem &P = c->probs[p];
        const int64_t Vp = (int64_t)P.nx * P.ny * P.nz;
        if (x0) {
            const int z_lo = c->regions.empty() ? 0 : c->regions[p].z_lo;
            const float *src = x0 + (int64_t)z_lo * P.nx * P.ny;
            if ((rc = copy_in(c, P.x, src, sizeof(float) * Vp, mem))) return rc;
        } else {
            HIPCHK(c, launch_sum_positive(L, P.s, Vp, c->d_scratch, 1024, c->d_scratch + 1024));
            HIPCHK(c, launch_uniform_image(L, P.s, Vp, c->d_scratch + 1024, (double)P.n_events, P.x));
        }
        HIPCHK(c, launch_fill(L, P.b, Vp, 0.0f));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_image = true;
    c->iter_count = 0;
    return LMTOF_OK;
}

int lmtof_read_image(lmtof_ctx *c, float *out, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_image) return fail(c, LMTOF_ESTATE, "no image yet");
    if (!out || n != c->V || !valid_mem(mem)) return fail(c, LMTOF_EINVAL, "need n = %lld floats", (long long)c->V);
    HIPCHK(c, hipSetDevice(c->device));
    if (c->regions.empty()) return copy_out(c, out, c->d_x, sizeof(float) * n, mem);
    // Section 2.5: the region images, each at its z offset, are summed into one volume
    Launch L;
    L.stream = c->stream;
    const int64_t plane = (int64_t)c->g.nx * c->g.ny;
    HIPCHK(c, launch_fill(L, c->d_x, c->V, 0.0f));
    for (auto &r : c->regions) HIPCHK(c, launch_add_slab(L, r.x, plane, r.z_lo, r.nz, c->d_x));
    return copy_out(c, out, c->d_x, sizeof(float) * n, mem);
}

int lmtof_iterate(lmtof_ctx *c, int n_iter, lmtof_iter_stats *stats) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_image) return fail(c, LMTOF_ESTATE, "set the image (lmtof_set_image) first");
    if (n_iter < 1 || n_iter > 10000) return fail(c, LMTOF_EINVAL, "n_iter must be in [1, 10000]");
    HIPCHK(c, hipSetDevice(c->device));
    try {
        int rc = ensure_problems(c);
        if (rc) return rc;
        const int np = (int)c->probs.size();
        if ((rc = ensure_stats(c, (size_t)n_iter * np))) return rc;
        auto it = c->graphs.find(n_iter);
        if (it == c->graphs.end()) {
            GraphEntry ge;
            rc = build_graph(c, n_iter, ge);
            if (rc) {
                if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
                if (ge.graph) (void)hipGraphDestroy(ge.graph);
                for (hipEvent_t e : ge.ev) if (e) (void)hipEventDestroy(e);
                return rc;
            }
            it = c->graphs.emplace(n_iter, ge).first;
        }
        HIPCHK(c, hipGraphLaunch(it->second.exec, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<DevStats> hs((size_t)n_iter * np);
        HIPCHK(c, hipMemcpy(hs.data(), c->d_stats, sizeof(DevStats) * hs.size(), hipMemcpyDeviceToHost));
        if (stats) {
            for (int k = 0; k < n_iter; ++k) {
                lmtof_iter_stats &o = stats[k];
                memset(&o, 0, sizeof o);
                o.iter = c->iter_count + k;
                double sx = 0, sxo = 0, slf = 0;
                int64_t ne = 0;
                for (int p = 0; p < np; ++p) {
                    const DevStats &d = hs[(size_t)k * np + p];
                    ne += d.n_eff;
                    sx += d.sum_sx;
                    sxo += d.sum_sx_old;
                    slf += d.sum_logf;
                }
                o.n_eff = ne;
                o.sum_sx = sx;
                o.loglik = slf - sxo;
                const auto &ev = it->second.ev;
                const hipEvent_t *e = &ev[(size_t)kEventsPerIter * k];
                auto span = [&](int a, int b) {
                    float t = 0;
                    return hipEventElapsedTime(&t, e[a], e[b]) == hipSuccess ? t : 0.0f;
                };
                o.ms = span(0, 6);
                o.forward_ms = span(0, 2);
                o.forward_kernel_ms = span(0, 1);
                o.back_ms = span(2, 5);
                o.back_kernel_ms = span(3, 4);
                o.update_ms = span(5, 6);
                o.project_ms = o.forward_ms + o.back_ms;
                (void)hipGetLastError();
            }
        }
        c->iter_count += n_iter;
        return LMTOF_OK;
    } catch (...) {
        return fail(c, LMTOF_ENOMEM, "host allocation failed");
    }
}

// f (caller order) = A x over the loaded events, with the TOF kernel if tof,
// else plain chord lengths (the LOR inside the grid); exp(A x) if acf.
static int forward_events(lmtof_ctx *c, const float *x, int64_t nx_, float *f, int64_t nf, int mem, bool tof,
                          bool acf) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (!x || !f || nx_ != c->V || nf != c->n_events || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need x of %lld floats and f of %lld floats", (long long)c->V, (long long)c->n_events);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    float *dx = nullptr, *fs = nullptr, *fc = nullptr, *xb = nullptr;
    Problem *dp = nullptr;
    ItemSet its;
    int rc = LMTOF_OK;
    auto done = [&](int r) {
        (void)hipStreamSynchronize(c->stream);
        if (mem == LMTOF_MEM_HOST) { dev_free(dx); dev_free(fc); }
        dev_free(fs);
        dev_free(xb);
        dev_free(dp);
        free_items(its);
        return r;
    };
    if (mem == LMTOF_MEM_HOST) {
        if ((rc = dev_alloc(c, &dx, c->V)) || (rc = dev_alloc(c, &fc, c->n_events))) return done(rc);
        if ((rc = copy_in(c, dx, x, sizeof(float) * c->V, LMTOF_MEM_HOST))) return done(rc);
    } else {
        dx = const_cast<float *>(x);
        fc = f;
    }
    if ((rc = dev_alloc(c, &fs, c->n_events)) || (rc = ensure_lut(c))) return done(rc);
    std::vector<Problem> ps{make_problem(c, 0, c->g.nz, dx, nullptr, nullptr)};
    if (!tof) ps[0].tof = 0;
    ps[0].events = c->d_events;
    ps[0].n_events = c->n_events;
    ps[0].rw = fs;
    int block, ept;
    launch_shape(c, block, ept);
    int64_t nch, nvch;
    hipError_t he = hipSuccess;
    if (tof && c->opt_forward == LMTOF_FORWARD_BRICKS) {
        // the MLEM iteration's projector: brick lists for this one problem
        if ((rc = upload_problems(c, ps, block, ept, &dp, nch, nvch)) || (rc = build_items(c, ps, dp, nch, ept, its)))
            return done(rc);
        he = launch_forward_items(L, true, dp, 1, its.chunks, its.n_chunks, its.bricks);
        if (he == hipSuccess) he = launch_combine(L, dp, 1, nch, ept, kCombineF, nullptr, nullptr);
    } else {
        const int64_t nxb = assign_xblocks(ps, nullptr);
        if ((rc = dev_alloc(c, &xb, nxb * 64))) return done(rc);
        assign_xblocks(ps, xb);
        if ((rc = upload_problems(c, ps, block, ept, &dp, nch, nvch))) return done(rc);
        he = hipMemsetAsync(xb, 0, sizeof(float) * 64 * (size_t)nxb, c->stream);
        if (he == hipSuccess) he = launch_block_image(L, dp, 1, nxb);
        if (he == hipSuccess) he = launch_forward(L, tof, dp, 1, nch, ept, 1, nullptr, nullptr);
    }
    if (he == hipSuccess && acf) he = launch_exp(L, fs, c->n_events);
    if (he == hipSuccess) he = launch_scatter_by_perm(L, fs, c->d_perm, c->n_events, fc);
    if (he != hipSuccess) return done(fail(c, LMTOF_EHIP, "forward projection: %s", hipGetErrorString(he)));
    if (mem == LMTOF_MEM_HOST) rc = copy_out(c, f, fc, sizeof(float) * c->n_events, LMTOF_MEM_HOST);
    else if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(c, LMTOF_EHIP, "forward projection failed");
    return done(rc);
}

int lmtof_forward_project(lmtof_ctx *c, const float *x, int64_t nx_, float *f, int64_t nf, int mem) {
    if (!c) return LMTOF_EINVAL;
    return forward_events(c, x, nx_, f, nf, mem, c->g.tof_fwhm_ps > 0, false);
}

int lmtof_attenuation_factors(lmtof_ctx *c, const float *mu, int64_t n_mu, float *acf, int64_t n_acf, int mem) {
    if (!c) return LMTOF_EINVAL;
    return forward_events(c, mu, n_mu, acf, n_acf, mem, false, true);
}

int lmtof_set_event_weights(lmtof_ctx *c, const float *w, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!w) {
        if (c->has_evw) c->probs_dirty = true;
        c->has_evw = false;
        return LMTOF_OK;
    }
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (n != c->n_events || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need %lld weights", (long long)c->n_events);
    HIPCHK(c, hipSetDevice(c->device));
    int rc = reserve(c, &c->d_evw_caller, c->evw_cap, (size_t)n);
    if (rc) return rc;
    if ((rc = copy_in(c, c->d_evw_caller, w, sizeof(float) * (size_t)n, mem))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_evw = true;
    c->probs_dirty = true;  // stored-order copy and the iteration graph follow
    return LMTOF_OK;
}

int lmtof_median_filter(lmtof_ctx *c, const float *x, int64_t nx_, float *y, int64_t ny_, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_geom) return fail(c, LMTOF_ESTATE, "set the geometry first");
    if (!x || !y || nx_ != c->V || ny_ != c->V || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need x and y of %lld floats", (long long)c->V);
    if (x == y) return fail(c, LMTOF_EINVAL, "x and y must not be the same array");
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    float *dx = nullptr, *dy = nullptr;
    int rc = LMTOF_OK;
    auto done = [&](int r) {
        (void)hipStreamSynchronize(c->stream);
        if (mem == LMTOF_MEM_HOST) {
            dev_free(dx);
            dev_free(dy);
        }
        return r;
    };
    if (mem == LMTOF_MEM_HOST) {
        if ((rc = dev_alloc(c, &dx, c->V)) || (rc = dev_alloc(c, &dy, c->V))) return done(rc);
        if ((rc = copy_in(c, dx, x, sizeof(float) * c->V, LMTOF_MEM_HOST))) return done(rc);
    } else {
        dx = const_cast<float *>(x);
        dy = y;
    }
    const hipError_t he = launch_median3(L, dx, dy, c->g.nx, c->g.ny, c->g.nz);
    if (he != hipSuccess) return done(fail(c, LMTOF_EHIP, "median filter: %s", hipGetErrorString(he)));
    if (mem == LMTOF_MEM_HOST) rc = copy_out(c, y, dy, sizeof(float) * c->V, LMTOF_MEM_HOST);
    else if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(c, LMTOF_EHIP, "median filter failed");
    return done(rc);
}

// The sampled projector's geometry: sample positions and Gaussian weights
// (FP64, normalised to sum 1, then rounded).
static SampledGeom sampled_geom(const lmtof_ctx *c) {
    const lmtof_geometry &g = c->g;
    SampledGeom G{};
    G.ox = (float)g.x0;
    G.oy = (float)g.y0;
    G.oz = (float)g.z0;
    G.ivx = (float)(1.0 / g.vx);
    G.ivy = (float)(1.0 / g.vy);
    G.ivz = (float)(1.0 / g.vz);
    G.nx = g.nx;
    G.ny = g.ny;
    G.nz = g.nz;
    G.half_c = (float)(g.c_mm_per_ps / 2.0);
    const double sg = sigma_mm(g), K = g.tof_trunc_sigmas, step = 2.0 * K * sg / kSampledN;
    G.t_lo = (float)(-K * sg);
    G.step = (float)step;
    double w[kSampledN], sum = 0.0;
    for (int k = 0; k < kSampledN; ++k) {
        const double t = -K * sg + (k + 0.5) * step;
        w[k] = std::exp(-0.5 * (t / sg) * (t / sg));
        sum += w[k];
    }
    for (int k = 0; k < kSampledN; ++k) G.w[k] = (float)(w[k] / sum);
    return G;
}

// Sampled forward (r == NULL: out = f over events, caller order) or back
// projection (out = b over voxels) of the loaded events.
static int sampled_project(lmtof_ctx *c, const float *in, int64_t n_in, float *out, int64_t n_out, int mem,
                           bool back) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (!(c->g.tof_fwhm_ps > 0)) return fail(c, LMTOF_EUNSUPPORTED, "the sampled projector needs TOF events");
    const int64_t want_in = back ? c->n_events : c->V, want_out = back ? c->V : c->n_events;
    if (!in || !out || n_in != want_in || n_out != want_out || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need %lld inputs and %lld outputs", (long long)want_in, (long long)want_out);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    float *din = nullptr, *dout = nullptr, *tmp = nullptr;
    int rc = LMTOF_OK;
    auto done = [&](int r) {
        (void)hipStreamSynchronize(c->stream);
        if (mem == LMTOF_MEM_HOST) {
            dev_free(din);
            dev_free(dout);
        }
        dev_free(tmp);
        return r;
    };
    if (mem == LMTOF_MEM_HOST) {
        if ((rc = dev_alloc(c, &din, want_in)) || (rc = dev_alloc(c, &dout, want_out))) return done(rc);
        if ((rc = copy_in(c, din, in, sizeof(float) * want_in, LMTOF_MEM_HOST))) return done(rc);
    } else {
        din = const_cast<float *>(in);
        dout = out;
    }
    if ((rc = dev_alloc(c, &tmp, c->n_events))) return done(rc);
    const SampledGeom G = sampled_geom(c);
    const bool packed = c->stored_packed != 0;
    hipError_t he;
    if (back) {
        he = launch_gather_by_perm(L, din, c->d_perm, c->n_events, tmp);
        if (he == hipSuccess) he = launch_fill(L, dout, c->V, 0.0f);
        if (he == hipSuccess) he = launch_sampled(L, c->d_events, packed, c->n_events, G, nullptr, nullptr, tmp, dout);
    } else {
        he = launch_sampled(L, c->d_events, packed, c->n_events, G, din, tmp, nullptr, nullptr);
        if (he == hipSuccess) he = launch_scatter_by_perm(L, tmp, c->d_perm, c->n_events, dout);
    }
    if (he != hipSuccess) return done(fail(c, LMTOF_EHIP, "sampled projector: %s", hipGetErrorString(he)));
    if (mem == LMTOF_MEM_HOST) rc = copy_out(c, out, dout, sizeof(float) * want_out, LMTOF_MEM_HOST);
    else if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(c, LMTOF_EHIP, "sampled projector failed");
    return done(rc);
}

int lmtof_sampled_forward_project(lmtof_ctx *c, const float *x, int64_t nx_, float *f, int64_t nf, int mem) {
    return sampled_project(c, x, nx_, f, nf, mem, false);
}

int lmtof_sampled_forward_project_noalloc(lmtof_ctx *c, const float *x, int64_t nx_, float *f, int64_t nf) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (!(c->g.tof_fwhm_ps > 0)) return fail(c, LMTOF_EUNSUPPORTED, "the sampled projector needs TOF events");
    if (!x || !f || nx_ != c->V || nf != c->n_events)
        return fail(c, LMTOF_EINVAL, "need x of %lld floats and f of %lld floats", (long long)c->V,
                    (long long)c->n_events);
    if (c->n_events > kNoAllocMaxEvents)
        return fail(c, LMTOF_EINVAL, "%lld events loaded: the allocation-free projection takes at most %lld",
                    (long long)c->n_events, (long long)kNoAllocMaxEvents);
    float *tmp = g_scratch_ptr[c->device];  // set by lmtof_create for this device
    if (!tmp) return fail(c, LMTOF_ESTATE, "no scratch address for device %d", c->device);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    const SampledGeom G = sampled_geom(c);
    hipError_t he = launch_sampled(L, c->d_events, c->stored_packed != 0, c->n_events, G, x, tmp, nullptr, nullptr);
    if (he == hipSuccess) he = launch_scatter_by_perm(L, tmp, c->d_perm, c->n_events, f);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return fail(c, LMTOF_EHIP, "sampled projector: %s", hipGetErrorString(he));
    return LMTOF_OK;
}

int lmtof_sampled_back_project(lmtof_ctx *c, const float *r, int64_t nr, float *b, int64_t nb, int mem) {
    return sampled_project(c, r, nr, b, nb, mem, true);
}

int lmtof_tof_keep(lmtof_ctx *c, const uint8_t *mask, int64_t nmask, uint8_t *keep, int64_t nkeep, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (!(c->g.tof_fwhm_ps > 0)) return fail(c, LMTOF_EUNSUPPORTED, "TOF scatter rejection needs TOF events");
    if (!mask || !keep || nmask != c->V || nkeep != c->n_events || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need a mask of %lld bytes and keep of %lld bytes", (long long)c->V,
                    (long long)c->n_events);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    uint8_t *dm = nullptr, *dk = nullptr;
    Problem *dp = nullptr;
    int rc = LMTOF_OK;
    auto done = [&](int r) {
        (void)hipStreamSynchronize(c->stream);
        if (mem == LMTOF_MEM_HOST) {
            dev_free(dm);
            dev_free(dk);
        }
        dev_free(dp);
        return r;
    };
    if (mem == LMTOF_MEM_HOST) {
        if ((rc = dev_alloc(c, &dm, c->V)) || (rc = dev_alloc(c, &dk, c->n_events))) return done(rc);
        if ((rc = copy_in(c, dm, mask, (size_t)c->V, LMTOF_MEM_HOST))) return done(rc);
    } else {
        dm = const_cast<uint8_t *>(mask);
        dk = keep;
    }
    // two-sided 95 % interval of the annihilation point along the LOR
    const double half = kTofRejectZ * sigma_mm(c->g);
    std::vector<Problem> ps{make_problem(c, 0, c->g.nz, nullptr, nullptr, nullptr)};
    ps[0].events = c->d_events;
    ps[0].n_events = c->n_events;
    ps[0].k_sigma = std::max(ps[0].k_sigma, (float)half * 1.001f);
    int block, ept;
    launch_shape(c, block, ept);
    int64_t nch, nvch;
    if ((rc = upload_problems(c, ps, block, ept, &dp, nch, nvch))) return done(rc);
    const hipError_t he = launch_tof_keep(L, dp, c->stored_packed != 0, c->n_events, (float)half, dm, c->d_perm, dk);
    if (he != hipSuccess) return done(fail(c, LMTOF_EHIP, "TOF scatter rejection: %s", hipGetErrorString(he)));
    if (mem == LMTOF_MEM_HOST) rc = copy_out(c, keep, dk, (size_t)c->n_events, LMTOF_MEM_HOST);
    else if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(c, LMTOF_EHIP, "TOF scatter rejection failed");
    return done(rc);
}

int lmtof_back_project(lmtof_ctx *c, const float *w, int64_t nw, float *b, int64_t nb, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (!w || !b || nw != c->n_events || nb != c->V || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need w of %lld floats and b of %lld floats", (long long)c->n_events, (long long)c->V);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    float *dw = nullptr, *ws = nullptr, *db = nullptr;
    Problem *dp = nullptr;
    ItemSet its;
    int rc = LMTOF_OK;
    auto done = [&](int r) {
        (void)hipStreamSynchronize(c->stream);
        if (mem == LMTOF_MEM_HOST) { dev_free(dw); dev_free(db); }
        dev_free(ws);
        dev_free(dp);
        free_items(its);
        return r;
    };
    if (mem == LMTOF_MEM_HOST) {
        if ((rc = dev_alloc(c, &dw, c->n_events)) || (rc = dev_alloc(c, &db, c->V))) return done(rc);
        if ((rc = copy_in(c, dw, w, sizeof(float) * c->n_events, LMTOF_MEM_HOST))) return done(rc);
    } else {
        dw = const_cast<float *>(w);
        db = b;
    }
    if ((rc = dev_alloc(c, &ws, c->n_events)) || (rc = ensure_lut(c))) return done(rc);
    std::vector<Problem> ps{make_problem(c, 0, c->g.nz, nullptr, db, nullptr)};
    ps[0].events = c->d_events;
    ps[0].n_events = c->n_events;
    ps[0].rw = ws;
    int block, ept;
    launch_shape(c, block, ept);
    int64_t nch, nvch;
    if ((rc = upload_problems(c, ps, block, ept, &dp, nch, nvch))) return done(rc);
    if ((rc = build_items(c, ps, dp, nch, ept, its))) return done(rc);
    hipError_t he = launch_gather_by_perm(L, dw, c->d_perm, c->n_events, ws);
    if (he == hipSuccess) he = launch_fill(L, db, c->V, 0.0f);
    // each event's weight onto its items, and each brick's largest |w|
    if (he == hipSuccess) he = launch_clear_bwmax(L, dp, 1, (int64_t)its.n_all_bricks);
    if (he == hipSuccess) he = launch_combine(L, dp, 1, nch, ept, kCombineWeights, nullptr, nullptr);
    if (he == hipSuccess) he = launch_brick_wmax(L, dp, 1, its.chunks, its.n_chunks, its.bricks);
    if (he != hipSuccess) return done(fail(c, LMTOF_EHIP, "back projection: %s", hipGetErrorString(he)));
    if ((rc = add_back(c, L, dp, 1, its, nullptr))) return done(rc);
    if (mem == LMTOF_MEM_HOST) rc = copy_out(c, b, db, sizeof(float) * c->V, LMTOF_MEM_HOST);
    else if (hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(c, LMTOF_EHIP, "back projection failed");
    return done(rc);
}

int lmtof_autotune(lmtof_ctx *c, int use_cache, lmtof_tune_result *out) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->has_image) return fail(c, LMTOF_ESTATE, "set the image (lmtof_set_image) first");
    HIPCHK(c, hipSetDevice(c->device));
    lmtof_tune_result res{};
    // cache key: device architecture, grid, voxel, TOF FWHM, storage,
    // regions, event count to a power of two
    std::string key;
    {
        hipDeviceProp_t prop{};
        HIPCHK(c, hipGetDeviceProperties(&prop, c->device));
        char buf[512];
        int l2n = 0;
        while ((int64_t(1) << (l2n + 1)) <= c->n_events) ++l2n;
        snprintf(buf, sizeof buf, "%s|%d,%d,%d|%.6g,%.6g,%.6g|%.6g|%d|%zu|%d", prop.gcnArchName, c->g.nx, c->g.ny,
                 c->g.nz, c->g.vx, c->g.vy, c->g.vz, c->g.tof_fwhm_ps, c->opt_storage, c->regions.size(), l2n);
        key = buf;
    }
    const int saved_fwd = c->opt_forward, saved_ept = c->opt_ept, saved_bch = c->opt_bchunks;
    auto restore = [&](int rc) {
        c->opt_forward = saved_fwd;
        c->opt_ept = saved_ept;
        c->opt_bchunks = saved_bch;
        c->probs_dirty = true;
        drop_graphs_only(c);
        return rc;
    };
    // apply a configuration: options, brick lists, b cleared
    auto apply = [&](int fwd, int ept, int bch) -> int {
        if (ept != (c->opt_ept > 0 ? c->opt_ept : kDefaultEpt) || bch != c->opt_bchunks) c->probs_dirty = true;
        c->opt_forward = fwd;
        c->opt_ept = ept;
        c->opt_bchunks = bch;
        drop_graphs_only(c);
        int rc = ensure_problems(c);
        if (rc) return rc;
        Launch L;
        L.stream = c->stream;
        for (const auto &P : c->probs)
            HIPCHK(c, launch_fill(L, P.b, (int64_t)P.nx * P.ny * P.nz, 0.0f));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LMTOF_OK;
    };
    bool hit = false;
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            res = it->second;
            hit = true;
        }
    }
    if (hit) {
        int rc = apply(res.forward, res.events_per_thread, res.brick_chunks);
        if (rc) return restore(rc);
        res.n_candidates = 0;
        res.cached = 1;
        if (out) *out = res;
        return LMTOF_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&](int rc) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return rc;
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return cleanup(restore(fail(c, LMTOF_EHIP, "event creation failed")));
    // time one candidate: build its lists, then the fastest of three passes
    // after a warm-up; cur_build is the build time of the lists now built
    float cur_build = 0.0f;
    c->probs_dirty = true;  // the first candidate builds (and times) its lists
    auto timeit = [&](int fwd, int ept, int bch, float &score) -> int {
        const auto b0 = std::chrono::steady_clock::now();
        const bool rebuild = ept != (c->opt_ept > 0 ? c->opt_ept : kDefaultEpt) || bch != c->opt_bchunks ||
                             c->probs_dirty;
        int rc = apply(fwd, ept, bch);
        if (rc) return rc;
        if (rebuild)
            cur_build = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - b0).count();
        const int np = (int)c->probs.size();
        Launch L;
        L.stream = c->stream;
        float t = 0.0f;
        for (int rep = 0; rep < 4; ++rep) {
            HIPCHK(c, hipEventRecord(e0, c->stream));
            if ((rc = add_forward(c, L, c->d_probs, np, c->n_chunks, c->n_xblk, c->items, c->ept_used,
                                  c->d_part_neff, c->d_part_ll, nullptr)))
                return rc;
            if ((rc = add_back(c, L, c->d_probs, np, c->items, nullptr))) return rc;
            float tr = 0.0f;
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&tr, e0, e1) != hipSuccess)
                return fail(c, LMTOF_EHIP, "autotune timing failed");
            if (rep == 1 || (rep > 1 && tr < t)) t = tr;
        }
        if (res.n_candidates < LMTOF_TUNE_MAX_CANDIDATES) {
            lmtof_tune_candidate &q = res.cand[res.n_candidates++];
            q.forward = fwd;
            q.events_per_thread = ept;
            q.brick_chunks = bch;
            q.pass_ms = t;
            q.build_ms = cur_build;
        }
        // the brick lists are built once per reconstruction: a tenth of
        // their build time is charged to each pass (~10 iterations)
        score = t + cur_build / kAutotuneIters;
        return LMTOF_OK;
    };
    int best_f = LMTOF_FORWARD_BRICKS, best_e = kDefaultEpt, best_b = kDefaultBrickChunks;
    float best = 0.0f;
    int rc = timeit(best_f, best_e, best_b, best);
    if (rc) return cleanup(restore(rc));
    // a change must beat the incumbent by more than 1 % (closer is within
    // the run-to-run spread of one timing)
    auto consider = [&](int f, int e, int b) -> int {
        float sc = 0.0f;
        int r = timeit(f, e, b, sc);
        if (r) return r;
        if (sc < 0.99f * best) {
            best = sc;
            best_f = f;
            best_e = e;
            best_b = b;
        }
        return LMTOF_OK;
    };
    for (int e : {1, 2, 8})
        if ((rc = consider(best_f, e, best_b))) return cleanup(restore(rc));
    for (int b : {4096, 16384})
        if ((rc = consider(best_f, best_e, b))) return cleanup(restore(rc));
    if ((rc = consider(LMTOF_FORWARD_EVENTS, best_e, best_b))) return cleanup(restore(rc));
    if ((rc = apply(best_f, best_e, best_b))) return cleanup(restore(rc));
    res.forward = best_f;
    res.events_per_thread = best_e;
    res.brick_chunks = best_b;
    res.cached = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = res;
    }
    if (out) *out = res;
    return cleanup(LMTOF_OK);
}

int lmtof_count_segments(lmtof_ctx *c, int64_t *visited, int64_t *weighted) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events) return fail(c, LMTOF_ESTATE, "load events first");
    if (!visited || !weighted) return fail(c, LMTOF_EINVAL, "output pointers are NULL");
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    Problem *dp = nullptr;
    unsigned long long *part = nullptr;
    std::vector<Problem> ps{make_problem(c, 0, c->g.nz, nullptr, nullptr, nullptr)};
    ps[0].events = c->d_events;
    ps[0].n_events = c->n_events;
    int block, ept;
    launch_shape(c, block, ept);
    int64_t nch, nvch;
    int rc = ensure_lut(c);
    if (!rc) ps[0] = make_problem(c, 0, c->g.nz, nullptr, nullptr, nullptr);
    ps[0].events = c->d_events;
    ps[0].n_events = c->n_events;
    if (!rc) rc = upload_problems(c, ps, block, ept, &dp, nch, nvch);
    if (!rc) rc = dev_alloc(c, &part, 2 * nch);
    std::vector<unsigned long long> h;
    if (!rc) {
        hipError_t he = launch_count_pieces(L, c->g.tof_fwhm_ps > 0, dp, 1, nch, ept, part);
        if (he == hipSuccess) {
            h.resize(2 * nch);
            he = hipMemcpyAsync(h.data(), part, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                                c->stream);
        }
        if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
        if (he != hipSuccess) rc = fail(c, LMTOF_EHIP, "segment count: %s", hipGetErrorString(he));
    }
    (void)hipStreamSynchronize(c->stream);
    dev_free(dp);
    dev_free(part);
    if (rc) return rc;
    unsigned long long a = 0, b = 0;
    for (int64_t k = 0; k < nch; ++k) {
        a += h[2 * k];
        b += h[2 * k + 1];
    }
    *visited = (int64_t)a;
    *weighted = (int64_t)b;
    return LMTOF_OK;
}

int lmtof_set_regions(lmtof_ctx *c, const int32_t *zb, int n, int margin) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->n_events || !c->has_sens) return fail(c, LMTOF_ESTATE, "load events and compute the sensitivity first");
    const lmtof_geometry &g = c->g;
    if (!(g.tof_fwhm_ps > 0)) return fail(c, LMTOF_EUNSUPPORTED, "the TOF-assisted data division needs TOF data");
    if (!zb || n < 1 || n > kMaxProblems) return fail(c, LMTOF_EINVAL, "n_regions must be in [1, %d]", kMaxProblems);
    if (zb[0] < 0 || zb[n] > g.nz) return fail(c, LMTOF_EINVAL, "z_bounds must lie within [0, nz = %d]", g.nz);
    for (int k = 0; k < n; ++k)
        if (zb[k + 1] <= zb[k]) return fail(c, LMTOF_EINVAL, "z_bounds must be strictly increasing");
    if (margin < 0) {
        const double sg = sigma_mm(g);
        const double sl = g.max_axial_angle_deg > 0 ? std::sin(g.max_axial_angle_deg * M_PI / 180.0) : 1.0;
        margin = (int)std::ceil(g.tof_trunc_sigmas * sg * sl / g.vz - 1e-9) + (int)std::ceil(6.0 / g.vz - 1e-9);
    }
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<Region> regs(n);
    for (int k = 0; k < n; ++k) {
        regs[k].core_lo = zb[k];
        regs[k].core_hi = zb[k + 1];
        regs[k].z_lo = std::max(0, zb[k] - margin);
        regs[k].nz = std::min(g.nz, zb[k + 1] + margin) - regs[k].z_lo;
    }
    const int64_t N = c->n_events;
    const size_t esz = c->stored_packed ? 16 : 32;
    KeyGeom kg = key_geom(c, c->opt_sort != 0, regs);
    const uint32_t nkeys = key_count(kg), kpr = nkeys / (uint32_t)n;
    Launch L;
    L.stream = c->stream;
    uint32_t *keys = nullptr, *hist = nullptr, *tmp = nullptr, *err = nullptr;
    int64_t *inner = nullptr, *perm = nullptr;
    char *store = nullptr;
    const int64_t plane = (int64_t)g.nx * g.ny;
    auto cleanup = [&](int rc) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
    };
    int rc;
    if ((rc = take(c, c->sc_keys, &keys, N)) || (rc = take(c, c->sc_hist, &hist, nkeys)) ||
        (rc = take(c, c->sc_tmp, &tmp, scan_tmp_elems(nkeys))) || (rc = take(c, c->sc_err, &err, 1)) ||
        (rc = take(c, c->sc_inner, &inner, N)) || (rc = take(c, c->sc_perm, &perm, N)) ||
        (rc = take(c, c->sc_events, &store, esz * N)))
        return cleanup(rc);
    int64_t reg_vox = 0;
    for (auto &r : regs) reg_vox += plane * r.nz;
    float *rbuf = nullptr;
    if ((rc = take(c, c->sc_reg, &rbuf, 3 * (size_t)reg_vox))) return cleanup(rc);
    for (auto &r : regs) {
        const int64_t Vr = plane * r.nz;
        r.x = rbuf;
        r.b = rbuf + Vr;
        r.s = rbuf + 2 * Vr;
        rbuf += 3 * Vr;
    }
    const int fmt = c->stored_packed ? 1 : 2;
    hipError_t he = hipMemsetAsync(hist, 0, sizeof(uint32_t) * nkeys, c->stream);
    if (he == hipSuccess) he = hipMemsetAsync(err, 0, sizeof(uint32_t), c->stream);
    if (he == hipSuccess) he = launch_ingest_keys(L, c->d_events, fmt, N, kg, 0, keys, hist, err);
    if (he == hipSuccess) he = launch_exclusive_scan(L, hist, nkeys, tmp);
    std::vector<uint32_t> starts(n, 0);
    for (int k = 0; k < n && he == hipSuccess; ++k)
        he = hipMemcpyAsync(&starts[k], hist + (size_t)k * kpr, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess)
        he = launch_scatter_events(L, c->d_events, fmt, N, keys, hist, c->stored_packed, store, inner);
    if (he == hipSuccess) he = launch_compose_perm(L, c->d_perm, inner, N, perm);
    for (auto &r : regs) {
        if (he != hipSuccess) break;
        he = launch_copy_slab(L, c->d_s, plane, r.z_lo, r.nz, r.s);
        if (he == hipSuccess) he = launch_fill(L, r.b, plane * r.nz, 0.0f);
        if (he == hipSuccess) he = launch_fill(L, r.x, plane * r.nz, 0.0f);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return cleanup(fail(c, LMTOF_EHIP, "region split: %s", hipGetErrorString(he)));
    for (int k = 0; k < n; ++k) {
        regs[k].ev_offset = starts[k];
        regs[k].n_events = (k + 1 < n ? (int64_t)starts[k + 1] : N) - (int64_t)starts[k];
    }
    // install: new event order, new permutation, region buffers
    drop_regions(c);
    drop_graphs(c);
    install_events(c);
    c->regions = regs;
    {
        void *old = c->reg_buf;
        c->reg_buf = static_cast<float *>(c->sc_reg.p);
        c->sc_reg.p = old;
        std::swap(c->reg_cap, c->sc_reg.cap);
    }
    c->margin_used = margin;
    c->has_image = false;
    c->probs_dirty = true;
    return cleanup(LMTOF_OK);
}

int lmtof_region_info(const lmtof_ctx *c, int k, int32_t *out4, int64_t *n_events) {
    if (!c || !out4 || !n_events) return LMTOF_EINVAL;
    if (k < 0 || k >= (int)c->regions.size()) return LMTOF_EINVAL;
    const Region &r = c->regions[k];
    out4[0] = r.z_lo;
    out4[1] = r.nz;
    out4[2] = r.core_lo;
    out4[3] = r.core_hi;
    *n_events = r.n_events;
    return LMTOF_OK;
}

int lmtof_event_regions(lmtof_ctx *c, int32_t *region, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (c->regions.empty()) return fail(c, LMTOF_ESTATE, "no region split (lmtof_set_regions) yet");
    if (!region || n != c->n_events || !valid_mem(mem))
        return fail(c, LMTOF_EINVAL, "need n = %lld int32 entries", (long long)c->n_events);
    HIPCHK(c, hipSetDevice(c->device));
    Launch L;
    L.stream = c->stream;
    int32_t *dst = region;
    int rc;
    if (mem == LMTOF_MEM_HOST) {
        // staged through the spare event store (not in use between loads)
        if ((rc = take(c, c->sc_events, &dst, (size_t)n))) return rc;
    }
    for (size_t k = 0; k < c->regions.size(); ++k)
        HIPCHK(c, launch_fill_by_perm(L, c->d_perm + c->regions[k].ev_offset, c->regions[k].n_events, (int32_t)k, dst));
    if (mem == LMTOF_MEM_HOST) return copy_out(c, region, dst, sizeof(int32_t) * (size_t)n, LMTOF_MEM_HOST);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LMTOF_OK;
}

int lmtof_read_region_image(lmtof_ctx *c, int k, float *out, int64_t n, int mem) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (c->regions.empty() || !c->has_image) return fail(c, LMTOF_ESTATE, "no region images yet");
    if (k < 0 || k >= (int)c->regions.size()) return fail(c, LMTOF_EINVAL, "region %d out of range", k);
    const Region &r = c->regions[k];
    const int64_t Vr = (int64_t)c->g.nx * c->g.ny * r.nz;
    if (!out || n != Vr || !valid_mem(mem)) return fail(c, LMTOF_EINVAL, "need n = %lld floats", (long long)Vr);
    HIPCHK(c, hipSetDevice(c->device));
    return copy_out(c, out, r.x, sizeof(float) * n, mem);
}

int lmtof_clear_regions(lmtof_ctx *c) {
    if (!c) return LMTOF_EINVAL;
    c->err.clear();
    if (!c->regions.empty()) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        drop_regions(c);
        drop_graphs(c);
        c->has_image = false;
    }
    return LMTOF_OK;
}

}  // extern "C"

// ==================================================================== serving

struct PoolReq {
    int64_t id = 0;
    lmtof_ctx *ctx = nullptr;
    int n_iter = 0, done = 0;
    int64_t bytes = 0;
};

// A request handed to the preparation thread (its footprint is reserved).
struct PrepJob {
    int64_t id = 0;
    lmtof_ctx *ctx = nullptr;
    lmtof_request q{};
    int64_t bytes = 0;
};

struct lmtof_pool {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int64_t budget = 0, used = 0, next_id = 1;
    std::vector<PoolReq> active;
    std::map<int64_t, PoolReq> finished;
    // Background preparation: one thread, its own stream.  mu guards used,
    // jobs, preparing, prepared and failed (the thread touches nothing else
    // of the pool); the calling thread owns everything else.
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    hipStream_t prep_stream = nullptr;
    std::deque<PrepJob> jobs;
    std::map<int64_t, bool> preparing;  // id -> TOF, from submit until the thread is done with it
    std::vector<PoolReq> prepared;      // ready to join the batch
    std::map<int64_t, std::pair<int, std::string>> failed;
    // contexts of released requests, kept with their device buffers for the
    // next admissions (a new request reuses one instead of allocating);
    // their bytes count against the budget and they are destroyed when an
    // admission needs the room
    std::vector<lmtof_ctx *> spare;
    // current batch
    bool dirty = true;
    std::vector<Problem> batch;
    Problem *d_probs = nullptr;
    size_t probs_cap = 0;
    uint4 *d_chunks = nullptr, *d_bricks = nullptr;
    size_t chunks_cap = 0, bricks_cap = 0;
    uint32_t n_bchunks = 0, n_bbricks = 0;
    int64_t n_chunks = 0, n_vchunks = 0;
    int *part_neff = nullptr;
    double *part_ll = nullptr, *part_old = nullptr, *part_new = nullptr;
    int64_t n_xblk = 0, n_all_bricks = 0;
    size_t part_cap = 0, vpart_cap = 0;
    DevStats *d_stats = nullptr;
    size_t stats_cap = 0;
    int ept = kDefaultEpt;
};

namespace {

int pfail(lmtof_pool *p, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (p) p->err = buf;
    return code;
}

#define PHIP(p, expr)                                                                                  \
    do {                                                                                               \
        hipError_t e__ = (expr);                                                                       \
        if (e__ != hipSuccess) return pfail((p), LMTOF_EHIP, "%s: %s", #expr, hipGetErrorString(e__)); \
    } while (0)

template <class T>
int pool_grow(lmtof_pool *p, T **ptr, size_t &cap, size_t n) {
    if (n <= cap && *ptr) return LMTOF_OK;
    dev_free(*ptr);
    cap = 0;
    if (hipMalloc((void **)ptr, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return pfail(p, LMTOF_ENOMEM, "pool batch allocation failed");
    }
    cap = n;
    return LMTOF_OK;
}

// Ingest, bucketing, sensitivity, start image and brick lists of a request
// on its context (on the context's stream), then wait for them.
int prepare_request(lmtof_ctx *c, const lmtof_request &q) {
    int rc;
    if ((rc = lmtof_set_option(c, LMTOF_OPT_STORAGE, q.storage)) || (rc = lmtof_set_geometry(c, &q.geometry)) ||
        (rc = lmtof_load_events(c, q.events, q.n_events, q.format, q.mem)) || (rc = lmtof_compute_sensitivity(c)) ||
        (rc = lmtof_set_image(c, nullptr, 0, LMTOF_MEM_HOST)))
        return rc;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, LMTOF_EHIP, "request preparation failed");
    return LMTOF_OK;
}

// The preparation thread: takes queued requests in order and prepares each
// on the pool's second stream while the calling thread steps the batch.
void pool_worker(lmtof_pool *p) {
    (void)hipSetDevice(p->device);
    for (;;) {
        PrepJob j;
        {
            std::unique_lock<std::mutex> lk(p->mu);
            p->cv.wait(lk, [&] { return p->stop || !p->jobs.empty(); });
            if (p->jobs.empty()) return;  // stop requested and nothing queued
            j = p->jobs.front();
            p->jobs.pop_front();
        }
        int rc = prepare_request(j.ctx, j.q);
        std::string msg = rc ? std::string(lmtof_last_error(j.ctx)) : std::string();
        if (!rc && j.ctx->ept_used != p->ept) {  // run lists and item slots index the forward chunks of this launch shape
            rc = LMTOF_EUNSUPPORTED;
            msg = "request prepared with a different launch shape";
        }
        const int64_t held = rc ? 0 : std::max(j.bytes, ctx_device_bytes(j.ctx));
        {
            std::lock_guard<std::mutex> lk(p->mu);
            p->preparing.erase(j.id);
            p->used += held - j.bytes;
            if (rc) {
                p->failed[j.id] = {rc, msg};
            } else {
                PoolReq r;
                r.id = j.id;
                r.ctx = j.ctx;
                r.n_iter = j.q.n_iter;
                r.bytes = held;
                p->prepared.push_back(r);
            }
        }
        if (rc) lmtof_destroy(j.ctx);
    }
}

// Batch = every active request's problem; chunk ids, brick ids and update
// chunks renumbered across the batch; brick chunks of all requests merged
// largest first.
int pool_build_batch(lmtof_pool *p) {
    p->batch.clear();
    std::vector<uint4> chunks, bricks;
    int64_t nch = 0, nvch = 0, nb = 0, nxb = 0;
    const int64_t ce = project_chunk_events(kForwardBlock, p->ept), cv = update_chunk_voxels();
    for (auto &r : p->active) {
        Problem P = r.ctx->probs[0];  // its blocked image copy stays the request's own (P.xb)
        P.chunk_begin = nch;
        P.vchunk_begin = nvch;
        P.brick_base = (int32_t)nb;
        P.xblk_begin = nxb;
        nxb += xblocks(P);
        nch += (P.n_events + ce - 1) / ce;
        nvch += ((int64_t)P.nx * P.ny * P.nz + cv - 1) / cv;
        const uint32_t bt = (uint32_t)bricks.size();
        for (uint4 q : r.ctx->items.h_chunks) chunks.push_back(make_uint4(q.x + bt, q.y, q.z, q.w));
        for (uint4 q : r.ctx->items.h_bricks) bricks.push_back(make_uint4(q.x + (uint32_t)nb, q.y, q.z, q.w));
        nb += (int64_t)P.nbx * P.nby * P.nbz;
        p->batch.push_back(P);
    }
    if (nch > 0x7fffffffLL || nb > 0x7fffffffLL) return pfail(p, LMTOF_EUNSUPPORTED, "batch too large");
    std::stable_sort(chunks.begin(), chunks.end(),
                     [](const uint4 &a, const uint4 &b) { return (a.z - a.y) > (b.z - b.y); });
    const size_t np = p->batch.size();
    int rc;
    if ((rc = pool_grow(p, &p->d_probs, p->probs_cap, np)) || (rc = pool_grow(p, &p->d_chunks, p->chunks_cap, chunks.size())) ||
        (rc = pool_grow(p, &p->d_bricks, p->bricks_cap, bricks.size())) ||
        (rc = pool_grow(p, &p->d_stats, p->stats_cap, np)))
        return rc;
    if ((size_t)nch > p->part_cap) {
        size_t c0 = p->part_cap, c1 = p->part_cap;
        if ((rc = pool_grow(p, &p->part_neff, c0, nch)) || (rc = pool_grow(p, &p->part_ll, c1, nch))) return rc;
        p->part_cap = nch;
    }
    if ((size_t)nvch > p->vpart_cap) {
        size_t c0 = p->vpart_cap, c1 = p->vpart_cap;
        if ((rc = pool_grow(p, &p->part_old, c0, nvch)) || (rc = pool_grow(p, &p->part_new, c1, nvch))) return rc;
        p->vpart_cap = nvch;
    }
    PHIP(p, hipMemcpyAsync(p->d_probs, p->batch.data(), sizeof(Problem) * np, hipMemcpyHostToDevice, p->stream));
    if (!chunks.empty())
        PHIP(p, hipMemcpyAsync(p->d_chunks, chunks.data(), sizeof(uint4) * chunks.size(), hipMemcpyHostToDevice, p->stream));
    if (!bricks.empty())
        PHIP(p, hipMemcpyAsync(p->d_bricks, bricks.data(), sizeof(uint4) * bricks.size(), hipMemcpyHostToDevice, p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    p->n_bchunks = (uint32_t)chunks.size();
    p->n_bbricks = (uint32_t)bricks.size();
    p->n_chunks = nch;
    p->n_vchunks = nvch;
    p->n_xblk = nxb;
    p->n_all_bricks = nb;
    p->dirty = false;
    return LMTOF_OK;
}

}  // namespace

extern "C" {

int lmtof_pool_create(lmtof_pool **out, int hip_device, void *hip_stream, int64_t budget) {
    if (!out) return LMTOF_EINVAL;
    *out = nullptr;
    if (budget <= 0) {
        g_create_err = "HBM budget must be > 0";
        return LMTOF_EINVAL;
    }
    try {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
            (void)hipGetLastError();
            g_create_err = "no such HIP device";
            return ndev < 1 ? LMTOF_EHIP : LMTOF_EINVAL;
        }
        if (hipSetDevice(hip_device) != hipSuccess) {
            g_create_err = "hipSetDevice failed";
            return LMTOF_EHIP;
        }
        lmtof_pool *p = new lmtof_pool();
        p->device = hip_device;
        p->budget = budget;
        if (hip_stream) {
            p->stream = (hipStream_t)hip_stream;
        } else {
            if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
                delete p;
                g_create_err = "hipStreamCreate failed";
                return LMTOF_EHIP;
            }
            p->own_stream = true;
        }
        *out = p;
        return LMTOF_OK;
    } catch (...) {
        g_create_err = "host allocation failed";
        return LMTOF_ENOMEM;
    }
}

int lmtof_pool_destroy(lmtof_pool *p) {
    if (!p) return LMTOF_OK;
    (void)hipSetDevice(p->device);
    if (p->worker.joinable()) {
        // drop the queued preparations, let the running one finish
        std::deque<PrepJob> queued;
        {
            std::lock_guard<std::mutex> lk(p->mu);
            queued.swap(p->jobs);
            p->stop = true;
        }
        p->cv.notify_all();
        p->worker.join();
        for (auto &j : queued) lmtof_destroy(j.ctx);
    }
    for (auto &r : p->prepared) lmtof_destroy(r.ctx);
    if (p->prep_stream) (void)hipStreamDestroy(p->prep_stream);
    (void)hipStreamSynchronize(p->stream);
    for (auto &r : p->active) lmtof_destroy(r.ctx);
    for (auto &kv : p->finished) lmtof_destroy(kv.second.ctx);
    for (lmtof_ctx *c : p->spare) lmtof_destroy(c);
    dev_free(p->d_probs);
    dev_free(p->d_chunks);
    dev_free(p->d_bricks);
    dev_free(p->part_neff);
    dev_free(p->part_ll);
    dev_free(p->part_old);
    dev_free(p->part_new);
    dev_free(p->d_stats);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return LMTOF_OK;
}

const char *lmtof_pool_last_error(const lmtof_pool *p) { return p ? p->err.c_str() : g_create_err.c_str(); }

int lmtof_pool_request_bytes(const lmtof_request *q, int64_t *bytes) {
    if (!q || !bytes || q->n_events < 1) return LMTOF_EINVAL;
    *bytes = request_bytes_estimate(*q);
    return LMTOF_OK;
}

int lmtof_pool_submit(lmtof_pool *p, const lmtof_request *q, int64_t *id) {
    if (!p) return LMTOF_EINVAL;
    p->err.clear();
    if (!q || !id) return pfail(p, LMTOF_EINVAL, "request or id pointer is NULL");
    if (q->n_iter < 1 || q->n_iter > 10000) return pfail(p, LMTOF_EINVAL, "n_iter must be in [1, 10000]");
    if (q->storage != 0 && q->storage != 1) return pfail(p, LMTOF_EINVAL, "storage must be 0 or 1");
    if (q->n_events < 1) return pfail(p, LMTOF_EINVAL, "n_events must be >= 1");
    if ((q->flags & ~LMTOF_REQ_BACKGROUND) || q->reserved0 != 0)
        return pfail(p, LMTOF_EINVAL, "unknown request flags");
    const bool background = (q->flags & LMTOF_REQ_BACKGROUND) != 0;
    const bool tof = q->geometry.tof_fwhm_ps > 0;
    std::unique_lock<std::mutex> lk(p->mu);
    bool mixed = false;
    for (auto &r : p->active) mixed = mixed || (r.ctx->g.tof_fwhm_ps > 0) != tof;
    for (auto &r : p->prepared) mixed = mixed || (r.ctx->g.tof_fwhm_ps > 0) != tof;
    for (auto &kv : p->preparing) mixed = mixed || kv.second != tof;
    if (mixed) return pfail(p, LMTOF_EAGAIN, "TOF and non-TOF requests are not batched together; retry when drained");
    const int64_t est = request_bytes_estimate(*q);
    if (est > p->budget) return pfail(p, LMTOF_ENOMEM, "request needs ~%lld bytes, over the %lld-byte budget",
                                      (long long)est, (long long)p->budget);
    if (p->used + est > p->budget)
        return pfail(p, LMTOF_EAGAIN, "request needs ~%lld bytes, %lld free now", (long long)est,
                     (long long)(p->budget - p->used));
    // Reuse a released request's context: the smallest one that already
    // holds the estimate within the budget, else the largest (it grows).
    // Other spares are destroyed while the pool's total would exceed it.
    int pick = -1;
    {
        int64_t best = 0;
        for (size_t k = 0; k < p->spare.size(); ++k) {
            const int64_t b = ctx_device_bytes(p->spare[k]);
            if (b >= est && p->used + b <= p->budget && (pick < 0 || b < best)) { pick = (int)k; best = b; }
        }
        if (pick < 0)
            for (size_t k = 0; k < p->spare.size(); ++k) {
                const int64_t b = ctx_device_bytes(p->spare[k]);
                if (b < est && (pick < 0 || b > best)) { pick = (int)k; best = b; }
            }
    }
    lmtof_ctx *c = nullptr;
    if (pick >= 0) {
        c = p->spare[pick];
        p->spare.erase(p->spare.begin() + pick);
    }
    for (;;) {
        int64_t rest = 0;
        size_t big = 0;
        for (size_t k = 0; k < p->spare.size(); ++k) {
            const int64_t b = ctx_device_bytes(p->spare[k]);
            rest += b;
            if (b > ctx_device_bytes(p->spare[big])) big = k;
        }
        if (p->spare.empty() || p->used + std::max(est, c ? ctx_device_bytes(c) : 0) + rest <= p->budget) break;
        lmtof_destroy(p->spare[big]);
        p->spare.erase(p->spare.begin() + big);
    }
    int rc;
    if (background && !p->prep_stream) {
        hipError_t e = hipStreamCreateWithFlags(&p->prep_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            p->prep_stream = nullptr;
            if (c) p->spare.push_back(c);
            return pfail(p, LMTOF_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
        }
    }
    hipStream_t st = background ? p->prep_stream : p->stream;
    if (!c && (rc = lmtof_create(&c, p->device, st))) return pfail(p, rc, "%s", lmtof_last_error(nullptr));
    c->stream = st;  // (a reused context may come from the other stream)
    if (background) {
        if (!p->worker.joinable()) {
            try {
                p->worker = std::thread(pool_worker, p);
            } catch (...) {
                p->spare.push_back(c);
                return pfail(p, LMTOF_ENOMEM, "could not start the preparation thread");
            }
        }
        PrepJob j;
        j.id = p->next_id++;
        j.ctx = c;
        j.q = *q;
        j.bytes = est;
        p->used += est;
        p->preparing[j.id] = tof;
        p->jobs.push_back(j);
        lk.unlock();
        p->cv.notify_one();
        *id = j.id;
        return LMTOF_OK;
    }
    lk.unlock();
    if ((rc = prepare_request(c, *q))) {
        std::string m = lmtof_last_error(c);
        lmtof_destroy(c);
        return pfail(p, rc, "%s", m.c_str());
    }
    if (c->ept_used != p->ept) {  // run lists and item slots index the forward chunks of this launch shape
        lmtof_destroy(c);
        return pfail(p, LMTOF_EUNSUPPORTED, "request prepared with a different launch shape");
    }
    PoolReq r;
    r.id = p->next_id++;
    r.ctx = c;
    r.n_iter = q->n_iter;
    r.bytes = std::max(est, ctx_device_bytes(c));
    lk.lock();
    p->used += r.bytes;
    p->active.push_back(r);
    p->dirty = true;
    *id = r.id;
    return LMTOF_OK;
}

int lmtof_pool_step(lmtof_pool *p, int *n_active) {
    if (!p) return LMTOF_EINVAL;
    p->err.clear();
    {
        // requests whose background preparation has finished join now
        std::lock_guard<std::mutex> lk(p->mu);
        for (auto &r : p->prepared) {
            r.ctx->stream = p->stream;
            p->active.push_back(r);
            p->dirty = true;
        }
        p->prepared.clear();
    }
    if (n_active) *n_active = (int)p->active.size();
    if (p->active.empty()) return LMTOF_OK;
    PHIP(p, hipSetDevice(p->device));
    int rc;
    if (p->dirty && (rc = pool_build_batch(p))) return rc;
    const int np = (int)p->batch.size();
    const bool tof = p->batch[0].tof != 0;  // submit keeps a batch all-TOF or all-non-TOF
    Launch L;
    L.stream = p->stream;
    PHIP(p, launch_forward_items(L, tof, p->d_probs, np, p->d_chunks, p->n_bchunks, p->d_bricks));
    PHIP(p, launch_clear_bwmax(L, p->d_probs, np, p->n_all_bricks));
    PHIP(p, launch_combine(L, p->d_probs, np, p->n_chunks, p->ept, kCombineRatio, p->part_neff, p->part_ll));
    PHIP(p, launch_brick_wmax(L, p->d_probs, np, p->d_chunks, p->n_bchunks, p->d_bricks));
    PHIP(p, launch_back_chunks(L, tof, p->d_probs, np, p->d_chunks, p->n_bchunks, p->d_bricks));
    PHIP(p, launch_reduce_tiles(L, p->d_probs, np, p->d_bricks, p->n_bbricks));
    PHIP(p, launch_update(L, p->d_probs, np, p->n_vchunks, p->part_old, p->part_new));
    PHIP(p, launch_finalize(L, p->d_probs, np, p->n_chunks, p->n_vchunks, p->part_neff, p->part_ll, p->part_old,
                            p->part_new, p->d_stats, 0));
    PHIP(p, hipStreamSynchronize(p->stream));
    std::vector<PoolReq> still;
    for (auto &r : p->active) {
        r.done += 1;
        r.ctx->iter_count += 1;
        if (r.done >= r.n_iter) {
            p->finished[r.id] = r;
            p->dirty = true;
        } else {
            still.push_back(r);
        }
    }
    p->active.swap(still);
    return LMTOF_OK;
}

int lmtof_pool_poll(lmtof_pool *p, int64_t id, int *done, float *out, int64_t n, int mem) {
    if (!p) return LMTOF_EINVAL;
    p->err.clear();
    if (!done) return pfail(p, LMTOF_EINVAL, "done pointer is NULL");
    *done = 0;
    auto it = p->finished.find(id);
    if (it == p->finished.end()) {
        for (auto &r : p->active)
            if (r.id == id) return LMTOF_OK;
        std::lock_guard<std::mutex> lk(p->mu);
        auto f = p->failed.find(id);
        if (f != p->failed.end()) {
            const int code = f->second.first;
            const std::string m = f->second.second;
            p->failed.erase(f);
            return pfail(p, code, "request %lld: %s", (long long)id, m.c_str());
        }
        if (p->preparing.count(id)) return LMTOF_OK;
        for (auto &r : p->prepared)
            if (r.id == id) return LMTOF_OK;
        return pfail(p, LMTOF_EINVAL, "unknown request id %lld", (long long)id);
    }
    lmtof_ctx *c = it->second.ctx;
    if (out) {
        int rc = lmtof_read_image(c, out, n, mem);
        if (rc) return pfail(p, rc, "%s", lmtof_last_error(c));
    }
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->used -= it->second.bytes;
    }
    p->spare.push_back(c);
    p->finished.erase(it);
    *done = 1;
    return LMTOF_OK;
}

int lmtof_pool_info(const lmtof_pool *p, int64_t *used, int64_t *budget, int *n_active, int *n_finished) {
    if (!p) return LMTOF_EINVAL;
    if (used) {
        std::lock_guard<std::mutex> lk(const_cast<lmtof_pool *>(p)->mu);
        *used = p->used;
    }
    if (budget) *budget = p->budget;
    if (n_active) *n_active = (int)p->active.size();
    if (n_finished) *n_finished = (int)p->finished.size();
    return LMTOF_OK;
}

}  // extern "C"

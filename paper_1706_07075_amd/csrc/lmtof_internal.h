// Internal declarations shared by the HIP sources of liblmtof.so.
// Not part of the public ABI (include/lmtof.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lmtof {

// One MLEM problem as the kernels see it: a voxel grid, its images and a
// contiguous range of stored events.  A whole-volume reconstruction is one
// problem; the TOF-assisted data division runs one problem per body region.
// Kernel-CDF table nodes, brick shape and launch shapes of the projector.
constexpr int kLutN = 1025;  // odd: the centre of the window is a node
// Cells of the brick projectors' piecewise-linear CDF table (odd: the
// centre of the window is the middle of a cell).
constexpr int kLinN = 4095;
constexpr int kBrickX = 16, kBrickY = 16, kBrickZ = 16;
constexpr int kBrickVox = kBrickX * kBrickY * kBrickZ;
// Brick items are grouped by their voxel-plane crossings in the brick
// (longest first), so that a wavefront's lanes walk similar lengths.
constexpr int kItemClasses = 12;
// Bytes of one brick item's walk record (two float4 and one uint2).
constexpr int kItemRecBytes = 32;
constexpr int kForwardBlock = 256;
constexpr int kBackBlock = 1024;

struct Problem {
    const void *events;   // stored events of this problem (plain: 2 x float4; packed: 1 x uint4)
    int64_t n_events;
    int64_t ev_offset;    // stored index of this problem's first event (per-event arrays)
    int64_t chunk_begin;  // first projector chunk of this problem (chunk ids are global)
    int64_t vchunk_begin; // first update chunk of this problem
    float *x;             // image (nx*ny*nz)
    float *b;             // back-projection accumulator, zero between iterations
    const float *s;       // sensitivity
    float *rw;            // per event of this problem: 1 / f or f (event-parallel forward), or a caller's weight
    const float *evw;     // per event of this problem: ratio weight (attenuation correction), or NULL
    // Brick items (the pieces of the events' windows inside 16^3-voxel
    // bricks), at positions the chunks index: per item its forward partial
    // sum of a x over the piece, replaced by its event's back-projection
    // weight before the back projection reads it
    float *pw;
    uint32_t n_items;     // items of the item set this problem's positions index
    // item positions of each event, in the order its window crosses the
    // bricks: evitems[evoff[i] .. evoff[i + 1]) for problem-local event i
    const uint32_t *evoff;
    const uint32_t *evitems;
    // How the combine pass reaches a forward chunk's items with coalesced
    // accesses.  runs + chunk * kTabWords (chunk counted from this
    // problem's first): a header (number of runs, items in runs) and a row
    // per run of consecutive positions the chunk's events fill (one run per
    // (brick, item class) key: first position, length | brick slot << 16 |
    // owner << 31, prefix of the lengths, problem-local brick).  itemslot,
    // in run order from the chunk's first evitems index (evoff of its first
    // event): each run item's index in the chunk's items in event-major
    // order (its event's evoff minus the chunk's first, plus its ordinal);
    // written for chunks of at most kRunItems items.  Per event: 1 if any
    // of its items was placed outside the runs (the combine pass then
    // reaches all of them through evitems).
    const uint32_t *runs;
    const uint16_t *itemslot;
    const uint8_t *evflag;
    // per item, its walk inside the brick, precomputed when the lists are
    // built: (A_x, A_y, A_z, B_x), (B_y, B_z, k_x | k_y << 16, k_z | local
    // voxel << 16 | entry face << 28) with k the first plane index minus the
    // anchor; the item's piece of the window follows from the entry face and
    // the brick's far faces
    const float4 *rec_a;
    const float4 *rec_b;
    unsigned long long *tiles;  // 64-bit fixed-point chunk tiles, indexed by tile slot
    // per problem-local brick: the largest exponent field of |w| over its
    // items this iteration, as that power of two's FP32 bits (an unsigned
    // max; cleared before the combine pass, which sets it), which fixes the
    // brick's fixed-point scale
    uint32_t *bwmax;
    // set (non-zero) by the combine pass when it wrote some item's weight
    // outside the runs, whose maximum it then leaves to launch_brick_wmax
    uint32_t *gflag;
    int32_t packed;
    int32_t tof;
    int32_t nx, ny, nz;
    float ox, oy, oz;     // grid corner (mm)
    float hx, hy, hz;     // far corner (mm)
    float vx, vy, vz;     // voxel size (mm)
    float ivx, ivy, ivz;  // 1 / voxel size
    float half_c;         // c / 2 (mm/ps): TOF centre shift per ps of dt
    float inv_sig_sqrt2;  // 1 / (sigma sqrt 2), sigma in mm
    float k_sigma;        // truncation half-width K sigma (mm)
    float norm;           // 1 / (2 erf(K / sqrt 2)): makes the full kernel sum to 1
    const float4 *lut;    // kernel-CDF table: a pad entry, kLutN nodes over [-K, K] sigma, a pad entry
    float lut_a, lut_b;   // node position of t (mm): t * lut_a + (kLutN - 1) / 2; lut_b = (kLutN - 1) / 2 + 1.5 2^23
    // Piecewise-linear kernel CDF of the brick projectors: a pad entry,
    // kLinN cells over [-K, K] sigma as (CDF at the cell's middle on the
    // chord, CDF difference over the cell), a pad entry.  Cell of t (mm):
    // the nearest integer to t * lin_a + (kLinN - 1) / 2; lin_b =
    // (kLinN - 1) / 2 + 1.5 2^23.
    const float2 *lin;
    float lin_a, lin_b;
    float a_max;          // bound on one piece weight (TOF: 1, the kernel mass; else the voxel diagonal)
    int32_t brick_base;   // global id of this problem's first brick
    int32_t nbx, nby, nbz;// bricks per axis
    // Forward-pass copy of x in 4x4x4-voxel blocks, x fastest inside a
    // block, so that the gathers of a wavefront's near-parallel rays fall on
    // a few 64-byte sectors.  Element index = (block << 6) | (iz & 3) << 4 |
    // (iy & 3) << 2 | (ix & 3), block = bz << (xfx + xfy) | by << xfx | bx:
    // each block coordinate has a bit field of its own (x and y fields
    // padded to powers of two; padding blocks hold 0), so a one-voxel step
    // along an axis is an add within that axis's bits.
    float *xb;
    int64_t xblk_begin;   // first block of this problem in the relayout launch
    int32_t nbx4, nby4, nbz4;  // 4^3 blocks per axis holding voxels
    int32_t xfx, xfy;     // widths of the bx and by fields
};

// Blocks (of 64 floats) of a problem's blocked copy, padding included.
__host__ __device__ inline int64_t xblocks(const Problem &P) { return (int64_t)P.nbz4 << (P.xfx + P.xfy); }

constexpr int kMaxProblems = 64;

// Where a kernel goes: straight onto a stream, or as a node of an explicit
// HIP graph after `deps` (the new node is written to *node).
struct Launch {
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t n_deps = 0;
    hipGraphNode_t *node = nullptr;
};

inline hipError_t do_launch(const Launch &L, const void *func, dim3 grid, dim3 block, size_t shmem, void **args) {
    if (grid.x == 0) return hipSuccess;
    if (!L.graph) {
        hipError_t e = hipLaunchKernel(func, grid, block, args, shmem, L.stream);
        return e != hipSuccess ? e : hipGetLastError();
    }
    hipKernelNodeParams p{};
    p.blockDim = block;
    p.gridDim = grid;
    p.func = const_cast<void *>(func);
    p.kernelParams = args;
    p.sharedMemBytes = (unsigned)shmem;
    p.extra = nullptr;
    return hipGraphAddKernelNode(L.node, L.graph, L.deps, L.n_deps, &p);
}

// ---- projector (project.hip)
int64_t project_chunk_events(int block, int ept);
// Event-parallel forward projection per event into P.rw, gathering from
// the blocked image copy P.xb; mode 0: 1 / f (0 if f <= 0) and per-chunk
// partials (n_eff, sum log f); mode 1: f.
hipError_t launch_forward(const Launch &L, bool tof, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept,
                          int mode, int *part_neff, double *part_ll);
// Brick-owned forward projection: every brick chunk (see the back
// projection) stages its brick of P.x in LDS and writes each item's partial
// sum of a x to P.pw.
hipError_t launch_forward_items(const Launch &L, bool tof, const Problem *d_probs, int n_probs, const uint4 *chunks,
                                uint32_t n_chunks, const uint4 *bricks);
// Per event (forward chunks of the launch shape of launch_forward), over
// its items' positions evitems[evoff[i] .. evoff[i + 1]):
//   kCombineRatio: f = sum of the items' partials P.pw; w = 1 / f (0 if
//     f <= 0), times P.evw[i] if set, written back to every item of the
//     event; per-chunk partials as launch_forward mode 0;
//   kCombineF: P.rw[i] = f;
//   kCombineWeights: w = P.rw[i], times P.evw[i] if set, written to every
//     item of the event.
// With kCombineRatio and kCombineWeights, P.bwmax (cleared first by
// launch_clear_bwmax) receives each brick's largest exponent of |w| (as
// that power of two's float bits) over the items the pass reached by runs;
// launch_brick_wmax then adds the items reached through evitems, if there
// were any (P.gflag).
enum { kCombineRatio = 0, kCombineF = 1, kCombineWeights = 2 };
hipError_t launch_combine(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept, int mode,
                          int *part_neff, double *part_ll);
// P.bwmax <- 0 for every brick of every problem (n_bricks in all), and
// P.gflag <- 0.
hipError_t launch_clear_bwmax(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_bricks);
// After the combine pass, if P.gflag is set: P.bwmax of each brick chunk's
// brick <- max(itself, the largest exponent of |w| over the chunk's items).  A chunk of
// a problem whose flag is clear returns at once.
hipError_t launch_brick_wmax(const Launch &L, const Problem *d_probs, int n_probs, const uint4 *chunks,
                             uint32_t n_chunks, const uint4 *bricks);
// Back projection by brick chunks.  Brick table entry (global brick id,
// first tile slot, end tile slot, items in the brick); chunk (brick table
// index, first item, end item, tile slot) over the items of the brick's
// problem with their weights P.pw, each brick's fixed-point scale from
// P.bwmax.  launch_back_chunks, then launch_reduce_tiles (which writes
// every voxel of the listed bricks of P.b).
hipError_t launch_back_chunks(const Launch &L, bool tof, const Problem *d_probs, int n_probs, const uint4 *chunks,
                              uint32_t n_chunks, const uint4 *bricks);
hipError_t launch_reduce_tiles(const Launch &L, const Problem *d_probs, int n_probs, const uint4 *bricks,
                               uint32_t n_bricks);
// Brick item lists, keyed by global brick * kItemClasses + item class.
// fill == 0 counts pieces per key into ctr and each event's pieces into
// P.evoff[i]; else writes every piece's walk record at position ctr[key]++
// (never past end[key]), the position to P.evitems[P.evoff[i] + k] for the
// event's k-th piece, the item's combine slot, the event's flag and the
// chunk's run list.  Same launch shape as the forward pass (its chunks are
// the combine pass's chunks).  tabs (brick_item_tab_words(n_chunks) words)
// carries each block's key table from the counting launch to the filling
// one, which replaces it with the run list.
hipError_t launch_brick_items(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept,
                              uint32_t *ctr, const uint32_t *end, int fill, uint32_t *tabs);
// Words of one forward chunk's table: the builder's (key, count) pairs of
// its LDS hash table (count pass), then a 4-word header and 4 words per run
// (fill pass).
constexpr int kTabHead = 4;
constexpr int64_t kTabWords = kTabHead + 4 * 1024;
int64_t brick_item_tab_words(int64_t n_chunks);
// part[2c] = voxel pieces visited by chunk c, part[2c+1] = pieces with non-zero weight.
hipError_t launch_count_pieces(const Launch &L, bool tof, const Problem *d_probs, int n_probs, int64_t n_chunks,
                               int ept, unsigned long long *part);

// TOF scatter rejection of the one problem at d_probs (n_events stored
// events): keep[perm[i]] = 1 if event i's LOR within half_width mm of its TOF
// centre passes through a voxel with mask != 0 (P.k_sigma >= half_width).
hipError_t launch_tof_keep(const Launch &L, const Problem *d_probs, bool packed, int64_t n_events, float half_width,
                          const uint8_t *mask, const int64_t *perm, uint8_t *keep);

// ---- the paper's sampled TOF projector (sampled.hip)
constexpr int kSampledN = 32;  // samples per event
struct SampledGeom {
    float ox, oy, oz, ivx, ivy, ivz;  // grid corner (mm) and inverse voxel sizes
    int nx, ny, nz;
    float half_c;       // c / 2 (mm/ps)
    float t_lo, step;   // sample k at t_lo + (k + 1/2) step (mm from the TOF centre)
    float w[kSampledN]; // weights, summing to 1
};
// Forward (r == NULL): f[i] = sum_k w_k x[voxel of sample k], per stored
// event.  Back (r != NULL): b[voxel] += w_k r[i] (b accumulated, FP32 atomics).
hipError_t launch_sampled(const Launch &L, const void *events, bool packed, int64_t n, const SampledGeom &G,
                          const float *x, float *f, const float *r, float *b);

// ---- median sieve (median.hip)
// y = 3x3x3 median of x (nx * ny * nz voxels, x fastest), 0 outside the grid; y != x.
hipError_t launch_median3(const Launch &L, const float *x, float *y, int nx, int ny, int nz);
// x <- t, t <- 0 over n voxels.
hipError_t launch_take_clear(const Launch &L, float *x, float *t, int64_t n);

// xb <- x in 4^3 blocks for every problem (n_xblk blocks in total).
hipError_t launch_block_image(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_xblk);

// ---- update and reductions (update.hip)
int64_t update_chunk_voxels();
hipError_t launch_update(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_vchunks, double *part_old,
                         double *part_new);

struct DevStats {
    int64_t n_eff;
    double sum_sx;      // sum s x after the update
    double sum_sx_old;  // sum s x before the update
    double sum_logf;    // sum over events with f > 0 of log f
};
// One block per problem: reduce the projector and update partials into
// stats[iter * n_probs + p].  n_chunks / n_vchunks: totals over all problems.
hipError_t launch_finalize(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks,
                           int64_t n_vchunks, const int *part_neff, const double *part_ll, const double *part_old,
                           const double *part_new, DevStats *stats, int iter);

hipError_t launch_sum_positive(const Launch &L, const float *s, int64_t n, double *partials, int n_part,
                               double *out);
hipError_t launch_uniform_image(const Launch &L, const float *s, int64_t n, const double *sum, double n_events,
                                float *x);
hipError_t launch_fill(const Launch &L, float *p, int64_t n, float v);
// a[i] *= w[i]; a[i] = exp(a[i]) (i < n).
hipError_t launch_mul(const Launch &L, float *a, const float *w, int64_t n);
hipError_t launch_exp(const Launch &L, float *a, int64_t n);
// dst[i] = src[z_lo * nx * ny + i] for a z-slab of nzs slices.
hipError_t launch_copy_slab(const Launch &L, const float *src, int64_t plane, int z_lo, int nzs, float *dst);
// dst[z_lo * plane + i] += src[i] for i < plane * nzs.
hipError_t launch_add_slab(const Launch &L, const float *src, int64_t plane, int z_lo, int nzs, float *dst);

// ---- sensitivity (sens.hip)
struct SensGeom {
    int32_t nx, ny, nz, n_phi;
    double ox, oy, oz, vx, vy, vz;
    double R, H, tan_lmax;  // tan_lmax <= 0: no cut
    // symmetries of the voxel-centre lattice that the acceptance shares
    // (set by the launcher): mirror in x, in y, in z, and the x <-> y swap
    int32_t sym_x, sym_y, sym_z, sym_xy;
};
hipError_t launch_sensitivity(const Launch &L, const SensGeom &g, float *s);

// ---- event ingest: validation, packing, bucketing sort (events.hip)
struct KeyGeom {
    int32_t ncx, ncy, ncz;  // bricks per axis holding TOF centres
    int32_t nsx, nsy, nsz;  // sub-cells per brick and axis
    int32_t n_phi, n_lam;   // direction bins (azimuth over [0, pi), elevation)
    int32_t n_regions;      // 0: no region split
    int32_t sort;           // 0: key = region only (keeps caller order inside a region)
    int32_t tof;
    float ox, oy, oz;       // grid corner (mm)
    float bx_inv, by_inv, bz_inv;  // 1 / brick edge (mm)
    float half_c;
    float region_z[kMaxProblems + 1];   // core bounds in mm (n_regions + 1 values)
    float region_z0[kMaxProblems];      // z of each region sub-volume's first plane (mm)
};
uint32_t key_count(const KeyGeom &g);
// Pass 1: validate raw events, compute keys, histogram them.
// err bits: 1 non-finite, 2 coincident endpoints, 4 int16 overflow (check_pack), 8 dt beyond binary16.
hipError_t launch_ingest_keys(const Launch &L, const void *raw, int fmt, int64_t n, const KeyGeom &g,
                              int check_pack, uint32_t *keys, uint32_t *hist, uint32_t *err);
// In-place exclusive scan of n counters; tmp needs scan_tmp_elems(n) entries.
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_exclusive_scan(const Launch &L, uint32_t *data, int64_t n, uint32_t *tmp);
// Pass 2: place every event at cursor[key]++ in the stored format; perm[pos] = caller index.
hipError_t launch_scatter_events(const Launch &L, const void *raw, int fmt, int64_t n, const uint32_t *keys,
                                 uint32_t *cursor, int store_packed, void *store, int64_t *perm);
hipError_t launch_gather_by_perm(const Launch &L, const float *src_caller, const int64_t *perm, int64_t n,
                                 float *dst_stored);
hipError_t launch_scatter_by_perm(const Launch &L, const float *src_stored, const int64_t *perm, int64_t n,
                                  float *dst_caller);
// dst_caller[perm[i]] = value for i < n.
hipError_t launch_fill_by_perm(const Launch &L, const int64_t *perm, int64_t n, int32_t value, int32_t *dst_caller);
// out[i] = outer[inner[i]] (compose two permutations).
hipError_t launch_compose_perm(const Launch &L, const int64_t *outer, const int64_t *inner, int64_t n,
                               int64_t *out);
hipError_t launch_unpermute_packed(const Launch &L, const uint4 *store, const int64_t *perm, int64_t n, uint4 *out);

}  // namespace lmtof

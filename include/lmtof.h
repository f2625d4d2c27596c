/*
 * lmtof — list-mode TOF-weighted MLEM on AMD Instinct MI355X (gfx950).
 *
 * C ABI of liblmtof.so.  All arguments are plain pointers and sizes; no C++
 * or framework types cross this boundary.
 *
 * Problem (arXiv 1706.07075, Sections 2.3-2.5): reconstruct the activity
 * image of a single-bed, long-axial-field-of-view cylindrical PET scanner
 * from list-mode coincidences, each a pair of detection points plus a
 * time-of-flight difference, with MLEM whose system model weights every
 * event's line of response by a Gaussian TOF kernel normalised to one.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: LMTOF_OK (0) or a negative LMTOF_E* code.  No C++ exception
 *   or abort crosses the ABI.  On error the context is left valid and
 *   unchanged (except that lmtof_last_error() holds the message).
 * Units: millimetres and picoseconds.  Frame: origin at the scanner centre,
 *   z along the scanner axis.
 * Images: float32, x fastest: index ix + nx * (iy + ny * iz).
 * Events: caller's order; outputs indexed per event (forward projections,
 *   back-projection weights) use the caller's order too, whatever internal
 *   order the library keeps.
 * Memory kinds: `mem` = LMTOF_MEM_HOST (pageable or pinned host memory) or
 *   LMTOF_MEM_DEVICE (device memory on the context's GPU).  Inputs are
 *   copied into buffers the library owns; the caller may free its buffers
 *   when the call returns.  Device inputs must be ready (their producers
 *   synchronised) when passed.  Outputs go to caller-provided buffers.
 * Streams: all work of a context runs on its stream; calls that return data
 *   to the caller synchronise that stream before returning.
 * Threads: a context is used by one host thread at a time.
 */
#ifndef LMTOF_H
#define LMTOF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define LMTOF_OK 0
#define LMTOF_EINVAL -1       /* bad argument, geometry, non-finite event, int16 overflow */
#define LMTOF_ESTATE -2       /* call made in the wrong order (e.g. iterate before load) */
#define LMTOF_ENOMEM -3       /* device allocation failed or over the memory budget */
#define LMTOF_EHIP -4         /* HIP runtime error (message kept) */
#define LMTOF_EUNSUPPORTED -5 /* valid request the library does not handle */
#define LMTOF_EAGAIN -6       /* pool: request does not fit right now; retry later */

/* --------------------------------------------------- event input formats */
/* 7 x float32 per event: P1.x P1.y P1.z P2.x P2.y P2.z (mm), dt = t1 - t2 (ps),
 * where t1 is the detection time at P1.  dt > 0 puts the TOF centre nearer P2. */
#define LMTOF_FMT_F32X7 0
/* 8 x int16 per event (16 bytes): q[0..5] = P1.xyz, P2.xyz in 0.1 mm quanta
 * (scanner-centred), q[6] = dt as IEEE binary16 bits (ps), q[7] = spare (0). */
#define LMTOF_FMT_PACKED16 1

/* ------------------------------------------------------------ memory kinds */
#define LMTOF_MEM_HOST 0
#define LMTOF_MEM_DEVICE 1

/* ----------------------------------------------------------------- options */
/* Internal event storage: 0 = plain float32 (32 B/event), 1 = packed
 * (16 B/event: int16 endpoints at 0.1 mm, binary16 dt; float32 input is
 * rounded half-to-even on the GPU).  Takes effect at the next load.  Default 0. */
#define LMTOF_OPT_STORAGE 1
/* Reorder events at load by (16^3-voxel brick holding the TOF centre,
 * direction bin, sub-cell of the brick) so that neighbouring GPU lanes trace
 * nearby, near-parallel rays and each brick's events form a few long runs.
 * 0/1, default 1. */
#define LMTOF_OPT_SORT 2
/* Azimuth nodes of the sensitivity quadrature.  Default 2048. */
#define LMTOF_OPT_SENS_NPHI 3
/* Events per forward chunk, over 256: 1..16, 0 = library default (4).  A
 * forward chunk (256 x value events, in stored order) is the unit of the
 * event-parallel forward pass, of the brick-list builder's key tables and
 * of the combine pass, which handles a chunk of at most 2048 events and
 * 8192 brick items through LDS and larger ones through each event's item
 * list (slower).  Takes effect when the brick lists are next built. */
#define LMTOF_OPT_EVENTS_PER_THREAD 5
/* Approximate edge of the sort key's sub-cells inside a brick, in mm
 * (default 16: 4 x 4 x 4 sub-cells of a brick of 4 mm voxels). */
#define LMTOF_OPT_SORT_CELL_MM 6
/* Median sieve between iterations (Section 2.4): after each iteration's
 * update, every image voxel is replaced by the median of its 3 x 3 x 3
 * neighbourhood, voxels outside the image (the grid, or a region's
 * sub-volume) counting as 0 (see lmtof_median_filter).  The iteration's
 * statistics describe the EM step before the sieve, which breaks the EM
 * normalisation sum_j s_j x_j = n_eff.  0/1, default 0.  Takes effect at the
 * next lmtof_iterate. */
#define LMTOF_OPT_MEDIAN_SIEVE 8

/* Forward projector of the MLEM iteration and of lmtof_forward_project with
 * TOF (Section 2.4: f_i = sum_j a_ij x_j; both give the same a_ij):
 * LMTOF_FORWARD_BRICKS (default): brick-owned.  Every event's window is cut
 *   into pieces per 16^3-voxel brick at load; a workgroup stages one brick
 *   of the image in LDS and adds up its pieces' a_ij x_j, and a second pass
 *   sums each event's pieces in the order its window crosses the bricks.
 * LMTOF_FORWARD_EVENTS: event-parallel, one GPU lane per event walking its
 *   whole window, the image read from global memory.
 * The iteration's back projection is brick-owned either way.  Takes effect
 * at the next call that projects. */
#define LMTOF_OPT_FORWARD 9
#define LMTOF_FORWARD_BRICKS 0
#define LMTOF_FORWARD_EVENTS 1
/* Workgroups of the brick projectors: a problem batch's brick items are cut
 * into chunks of max(2048, items / value) items (a brick's list into at
 * least one chunk).  256..65536, default 8192.  Takes effect when the brick
 * lists are next built (next load, region split or image set). */
#define LMTOF_OPT_BRICK_CHUNKS 10

/* ------------------------------------------------------------------ types */
typedef struct lmtof_ctx lmtof_ctx;

/* Reconstruction geometry.  The voxel grid must lie inside the scanner
 * cylinder (transaxial corners within the radius, z within the half length). */
typedef struct {
    int32_t nx, ny, nz;         /* voxels per axis, >= 1 */
    int32_t reserved0;          /* must be 0 */
    double vx, vy, vz;          /* voxel size (mm), > 0 */
    double x0, y0, z0;          /* grid corner (mm): voxel (0,0,0) spans [x0, x0+vx) ... */
    double scanner_radius;      /* barrel radius R (mm) */
    double scanner_half_length; /* barrel half length H (mm) */
    double max_axial_angle_deg; /* acceptance cut on the LOR elevation; 0 = none */
    double tof_fwhm_ps;         /* coincidence time resolution (FWHM, ps); <= 0: non-TOF */
    double tof_trunc_sigmas;    /* kernel truncation K (sigmas); 0 = default 3 */
    double c_mm_per_ps;         /* speed of light; 0 = default 0.299792458 */
} lmtof_geometry;

/* Per-iteration statistics (iteration k maps image x^k to x^{k+1}). */
typedef struct {
    int32_t iter;     /* k, counted from the last lmtof_set_image */
    int32_t reserved0;
    int64_t n_eff;    /* events with forward projection (A x^k)_i > 0 */
    double sum_sx;    /* sum_j s_j x^{k+1}_j, FP64 (equals n_eff up to rounding) */
    double loglik;    /* sum_i log (A x^k)_i - sum_j s_j x^k_j over n_eff events */
    float ms;         /* wall time of the iteration on the GPU (ms) */
    float project_ms; /* of which: forward + back projection (ms) */
    float forward_ms; /* forward stage: projection, ratios written to the brick items (ms) */
    float back_ms;    /* back projection stage: brick scales, brick kernel, tile reduction (ms) */
    float back_kernel_ms; /* of which the brick back projection kernel alone (ms) */
    float update_ms;  /* image update and statistics (ms) */
    float forward_kernel_ms; /* of forward_ms, the forward projection kernel alone (ms) */
} lmtof_iter_stats;

/* ------------------------------------------------------------- lifecycle */
/* Create a context on HIP device `hip_device`.  `hip_stream` is a
 * hipStream_t to run on, or NULL to let the library create its own
 * (default priority).  *out receives the context. */
int lmtof_create(lmtof_ctx **out, int hip_device, void *hip_stream);
/* Free every device buffer, graph and stream the context owns.  NULL is a no-op. */
int lmtof_destroy(lmtof_ctx *ctx);
/* Message of the last failing call on ctx ("" if none).  Valid until the
 * next call on ctx.  With ctx == NULL: message of the last failed create. */
const char *lmtof_last_error(const lmtof_ctx *ctx);
/* Set an LMTOF_OPT_* option.  EINVAL for an unknown key or value. */
int lmtof_set_option(lmtof_ctx *ctx, int key, int64_t value);
int lmtof_get_option(const lmtof_ctx *ctx, int key, int64_t *value);

/* -------------------------------------------------------------- geometry */
/* Host-only validation of a geometry, without a context or a GPU: returns
 * LMTOF_OK, or LMTOF_EINVAL with the reason copied (NUL-terminated,
 * truncated) into msg[0..msg_len-1] when msg is non-NULL. */
int lmtof_check_geometry(const lmtof_geometry *g, char *msg, int64_t msg_len);
/* Section 2 (Materials and Methods): a voxelised image volume inside a
 * single-bed cylindrical scanner; Section 2.3: Gaussian TOF kernel of the
 * given FWHM.  Validates and stores the geometry.  Drops loaded events,
 * sensitivity and image (they depend on it). */
int lmtof_set_geometry(lmtof_ctx *ctx, const lmtof_geometry *g);

/* ---------------------------------------------------------------- events */
/* Load n >= 1 list-mode events (Section 1: list-mode processing, one event
 * at a time, of the whole axial field of view) in `format` from `ev`
 * (host or device memory per `mem`).  Every coordinate and dt must be
 * finite (EINVAL otherwise); with packed storage every coordinate must fit
 * int16 at 0.1 mm (EINVAL otherwise).  Replaces previously loaded events
 * and resets the image.  Needs a geometry (ESTATE). */
int lmtof_load_events(lmtof_ctx *ctx, const void *ev, int64_t n, int format, int mem);
/* Number of loaded events. */
int lmtof_num_events(const lmtof_ctx *ctx, int64_t *n);
/* Copy the stored packed records (LMTOF_FMT_PACKED16 layout, caller's
 * order) to `out` (n x 16 bytes).  ESTATE unless storage is packed. */
int lmtof_read_packed_events(lmtof_ctx *ctx, void *out, int64_t n, int mem);

/* ----------------------------------------------------------- sensitivity */
/* Section 2.4 ("sensitive matrix"): s_j = probability that an isotropic
 * back-to-back photon pair emitted at the centre of voxel j is detected,
 * i.e. both ends meet the barrel within |z| <= H with elevation inside the
 * axial acceptance cut (Section 2.1.2, 45 degrees).  Azimuth quadrature with
 * LMTOF_OPT_SENS_NPHI midpoint nodes, FP64 accumulation, stored float32.
 * Needs a geometry (ESTATE). */
int lmtof_compute_sensitivity(lmtof_ctx *ctx);
/* Copy s (n = nx*ny*nz floats) out, or set it from the caller. */
int lmtof_read_sensitivity(lmtof_ctx *ctx, float *out, int64_t n, int mem);
int lmtof_set_sensitivity(lmtof_ctx *ctx, const float *s, int64_t n, int mem);

/* --------------------------------------------------------------- image */
/* The image MLEM starts from (Section 2.4, the iteration's x^0; the paper
 * feeds it with a starting back projection, Section 3.5.4, read here as the
 * uniform image of the same total, which keeps sum_j s_j x_j = N from the
 * first iteration on).  Sets x^0 (n = nx*ny*nz floats, >= 0, finite), or
 * with x0 == NULL the uniform start x^0_j = N / sum_{s>0} s for s_j > 0,
 * else 0 (sum in FP64).  Resets the iteration counter.  Needs events and
 * sensitivity (ESTATE). */
int lmtof_set_image(lmtof_ctx *ctx, const float *x0, int64_t n, int mem);
/* Copy the current MLEM image x^k (Section 2.4; n = nx*ny*nz floats, x
 * fastest) out; with a region split (Section 2.5) the region images summed
 * at their z offsets. */
int lmtof_read_image(lmtof_ctx *ctx, float *out, int64_t n, int mem);

/* ------------------------------------------------------------ iterations */
/* Section 2.4: run n_iter >= 1 list-mode MLEM iterations with the TOF
 * kernel: f_i = sum_j a_ij x_j; b_j = sum_{i: f_i > 0} a_ij / f_i;
 * x_j <- x_j b_j / s_j (0 where s_j = 0).  a_ij is the truncated (+-K sigma),
 * renormalised Gaussian TOF kernel integrated over the piece of event i's
 * line inside voxel j (Siddon traversal); non-TOF geometry: the piece
 * length.  The n_iter iterations are replayed from one HIP graph.  If stats
 * is non-NULL it receives n_iter entries.  Needs an image (ESTATE). */
int lmtof_iterate(lmtof_ctx *ctx, int n_iter, lmtof_iter_stats *stats);

/* One configuration the autotuner timed. */
typedef struct {
    int32_t forward;           /* LMTOF_FORWARD_* */
    int32_t events_per_thread; /* LMTOF_OPT_EVENTS_PER_THREAD */
    int32_t brick_chunks;      /* LMTOF_OPT_BRICK_CHUNKS */
    int32_t reserved0;
    float pass_ms;             /* one projector pass (forward stage + back stage), fastest of three */
    float build_ms;            /* building its brick lists (host wall time) */
} lmtof_tune_candidate;

#define LMTOF_TUNE_MAX_CANDIDATES 16

typedef struct {
    int32_t forward;           /* chosen configuration, now set as the options */
    int32_t events_per_thread;
    int32_t brick_chunks;
    int32_t n_candidates;      /* entries of cand (0 when taken from the cache) */
    int32_t cached;            /* 1: found in the cache, nothing timed */
    int32_t reserved0;
    lmtof_tune_candidate cand[LMTOF_TUNE_MAX_CANDIDATES];
} lmtof_tune_result;

/* Launch autotuner (the batched launch of Section 2.5 made to fit the
 * device).  Times one projector pass over the loaded events and current
 * batch (whole volume or regions) per candidate, each the fastest of three
 * after a warm-up pass, and scores it as that time plus a tenth of the time
 * its brick lists took to build (once per reconstruction of ~10
 * iterations).  The search is coordinate-wise from the defaults (brick
 * forward projector, 4 events per thread, 8192 brick chunks): events per
 * thread over {1, 2, 4, 8}, then brick chunks over {4096, 8192, 16384},
 * then the forward projector over {bricks, events}; a change is kept only
 * if it beats the incumbent by more than 1 %.  The winner is set as the
 * options and its brick lists are built.  Results are cached for the
 * process, keyed by (device architecture, grid, voxel size, TOF FWHM,
 * storage format, number of regions, event count rounded to a power of
 * two); with use_cache != 0 a cached configuration is applied without
 * timing.  The image is not changed; the back projection accumulator is
 * cleared afterwards.  *out (may be NULL) receives the result.  Needs an
 * image (ESTATE). */
int lmtof_autotune(lmtof_ctx *ctx, int use_cache, lmtof_tune_result *out);

/* --------------------------------------------------- projector (testing) */
/* Forward projection of Section 2.4's MLEM, f_i = sum_j a_ij x_j with the
 * TOF-weighted a_ij of lmtof_iterate (Section 2.3's kernel integrated over
 * each voxel piece), of image x (nx*ny*nz floats) for every loaded event,
 * f in the caller's event order (n_events floats).  x and f live in `mem`.
 * Needs events (ESTATE). */
int lmtof_forward_project(lmtof_ctx *ctx, const float *x, int64_t nx_, float *f, int64_t nf, int mem);
/* Median sieve of Section 2.4, applied once: y_j = median of x over the
 * 3 x 3 x 3 block of voxels around j, voxels outside the grid counting as 0
 * (the paper gives neither the neighbourhood nor the border rule: this is
 * the reading used).  With 27 values the median is the 14th smallest, an
 * element of x: exact.  x and y (nx*ny*nz floats each, x fastest, distinct
 * arrays) live in `mem`.  Needs a geometry (ESTATE); EINVAL for wrong sizes
 * or x == y. */
int lmtof_median_filter(lmtof_ctx *ctx, const float *x, int64_t nx_, float *y, int64_t ny_, int mem);

/* TOF scatter rejection of Section 2.2 (a pre-pass: filter the events, then
 * load the kept ones).  For every loaded event, keep[k] (k the event's index
 * in the caller's order of the last load) = 1 if the stretch of its LOR
 * within 1.959964 sigma of its TOF centre (the two-sided 95 % interval of
 * the annihilation point), cut by the grid box, passes a piece of positive
 * length through a body voxel, else 0.  The body outline is mask: one byte
 * per voxel of the grid (x fastest, non-zero = body), e.g. from a CT.  mask
 * (nx*ny*nz bytes) and keep (n_events bytes) live in `mem`.  Needs loaded
 * events (ESTATE) and TOF (EUNSUPPORTED otherwise). */
int lmtof_tof_keep(lmtof_ctx *ctx, const uint8_t *mask, int64_t n_mask, uint8_t *keep, int64_t n_keep, int mem);

/* Attenuation correction on the LOR (Section 2.4).  The paper weights each
 * event in the forward model instead of attenuating the sensitivity; its
 * wording is read as the correction factor 1 / P_survive.
 * lmtof_attenuation_factors: acf[k] = exp(line integral of mu along event
 * k's whole LOR inside the grid), k in the caller's order of the last load;
 * mu (nx*ny*nz floats, 1/mm, x fastest) and acf (n_events floats) live in
 * `mem`.  Needs loaded events (ESTATE).
 * lmtof_set_event_weights: w[k] (caller order, n_events floats in `mem`)
 * multiplies event k's ratio in every following iteration: x <- x / s *
 * A^T (w / A x).  Then sum_j s_j x_j after an iteration equals the sum of w
 * over the events with (A x)_i > 0, and the log-likelihood stays
 * unweighted.  w = NULL drops the weights; loading events drops them too.
 * Needs loaded events (ESTATE); EINVAL for a wrong count. */
int lmtof_attenuation_factors(lmtof_ctx *ctx, const float *mu, int64_t n_mu, float *acf, int64_t n_acf, int mem);
int lmtof_set_event_weights(lmtof_ctx *ctx, const float *w, int64_t n, int mem);

/* The paper's own TOF projector (Section 2.3), for comparison with the
 * exact-integral projector above: each loaded event is sampled at 32 points
 * spaced equally along its LOR over [-K sigma, K sigma] around the TOF
 * centre (midpoints of 32 equal steps; K = tof_trunc_sigmas), weighted by
 * the Gaussian density there with the 32 weights summing to 1, each point
 * reading (forward) or adding into (back) the voxel that holds it; points
 * outside the grid are dropped.  Forward: f (n_events, caller order) from x
 * (nx*ny*nz).  Back: b (nx*ny*nz, overwritten) from r (n_events, caller
 * order); FP32 atomics, so b is not bit-reproducible.  Arrays in `mem`.
 * Needs loaded TOF events (ESTATE / EUNSUPPORTED). */
int lmtof_sampled_forward_project(lmtof_ctx *ctx, const float *x, int64_t nx_, float *f, int64_t nf, int mem);
int lmtof_sampled_back_project(lmtof_ctx *ctx, const float *r, int64_t nr, float *b, int64_t nb, int mem);
/* lmtof_sampled_forward_project for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same f, bit for bit, with x
 * and f in device memory (no `mem` argument), and no allocation or free of
 * any kind during the call.  The projections in stored event order live in
 * a fixed device buffer of the library, one per GPU, that holds at most
 * 4194304 (2^22) events: EINVAL if more events are loaded.  That buffer is
 * shared by every context on the GPU and keeps the last call's contents:
 * calls that overlap on one GPU (several host threads or streams) race and
 * must be serialised by the caller.  Synchronises the context's stream
 * before returning.  Needs loaded TOF events (ESTATE / EUNSUPPORTED). */
int lmtof_sampled_forward_project_noalloc(lmtof_ctx *ctx, const float *x, int64_t nx_, float *f, int64_t nf);
/* Back projection of Section 2.4's MLEM (the transpose of the forward
 * projection above), b_j = sum_i a_ij w_i of per-event weights w (caller's
 * order, n_events floats) into b (nx*ny*nz floats, overwritten).  Sums are
 * exact 64-bit fixed point: b does not depend on event order. */
int lmtof_back_project(lmtof_ctx *ctx, const float *w, int64_t nw, float *b, int64_t nb, int mem);

/* Diagnostic: total voxel pieces the loaded events' rays visit inside their
 * windows (*visited; each costs one image gather in the forward pass) and
 * how many have non-zero weight (*weighted; each costs one atomic add in the
 * back pass).  Needs events (ESTATE). */
int lmtof_count_segments(lmtof_ctx *ctx, int64_t *visited, int64_t *weighted);

/* ------------------------------------------------------------- regions */
/* Section 2.5, TOF-assisted data division: split the field of view into
 * n_regions (1..64) axial core slabs given by n_regions+1 strictly
 * increasing slice indices 0 <= z_bounds[0] < ... < z_bounds[n] <= nz.
 * Each event goes to the core holding its TOF centre's z (clamped to the
 * first/last core).  Needs TOF (EUNSUPPORTED otherwise).  Region
 * k is an independent MLEM problem on the sub-volume core_k widened by
 * margin_slices on both sides (clamped to the grid); a negative margin asks
 * for the default ceil(K sigma sin(lambda_max) / vz) + ceil(6 mm / vz).
 * All regions iterate together in one batched launch per iteration.
 * Needs events and sensitivity (ESTATE). */
int lmtof_set_regions(lmtof_ctx *ctx, const int32_t *z_bounds, int n_regions, int margin_slices);
/* Region k's sub-volume: out4[0] = first slice, out4[1] = slices,
 * out4[2] = core first slice, out4[3] = core end slice; *n_events = events. */
int lmtof_region_info(const lmtof_ctx *ctx, int k, int32_t *out4, int64_t *n_events);
/* Section 2.5: the region each loaded event was assigned to by
 * lmtof_set_regions (its TOF centre's core), region[i] in [0, n_regions)
 * for event i in the caller's order of the last lmtof_load_events.  n must
 * equal the number of loaded events; region is caller-owned (n int32 in
 * `mem`).  ESTATE without a region split. */
int lmtof_event_regions(lmtof_ctx *ctx, int32_t *region, int64_t n, int mem);
/* Region k's current image (nx*ny*slices floats). */
int lmtof_read_region_image(lmtof_ctx *ctx, int k, float *out, int64_t n, int mem);
/* Drop the region split (back to one whole-volume problem). */
int lmtof_clear_regions(lmtof_ctx *ctx);

/* --------------------------------------------------------------- serving */
/* Continuous-batching reconstruction server on one GPU (not in the paper; it
 * serves many list-mode reconstructions at once).  A pool admits requests
 * while their estimated device footprint fits its HBM budget; each step runs
 * ONE batched MLEM iteration over every active request (each at its own
 * iteration index, all in the same kernel launches); requests join and
 * leave at step boundaries, keeping events and images resident meanwhile.
 * A request's result does not depend on which other requests share its
 * steps (every kernel is order-independent for a given request). */
typedef struct lmtof_pool lmtof_pool;

typedef struct {
    lmtof_geometry geometry;
    const void *events;  /* n_events records in `format`, in `mem` */
    int64_t n_events;
    int32_t format;      /* LMTOF_FMT_* */
    int32_t mem;         /* LMTOF_MEM_* */
    int32_t n_iter;      /* MLEM iterations, >= 1 */
    int32_t storage;     /* 0 plain, 1 packed */
    int32_t flags;       /* 0 or LMTOF_REQ_BACKGROUND */
    int32_t reserved0;   /* must be 0 */
} lmtof_request;

/* Request flag: prepare the request in the background (see
 * lmtof_pool_submit), so that running requests keep stepping meanwhile. */
#define LMTOF_REQ_BACKGROUND 1

/* Create a pool on `hip_device` (stream as in lmtof_create) with an HBM
 * budget in bytes for resident requests (> 0). */
int lmtof_pool_create(lmtof_pool **out, int hip_device, void *hip_stream, int64_t hbm_budget_bytes);
int lmtof_pool_destroy(lmtof_pool *pool);
const char *lmtof_pool_last_error(const lmtof_pool *pool);
/* Estimated device footprint (bytes) the pool reserves for a request. */
int lmtof_pool_request_bytes(const lmtof_request *req, int64_t *bytes);
/* Validate, copy and prepare (ingest, bucketing, sensitivity, start image,
 * brick lists) a request; *id receives its handle.  LMTOF_EAGAIN (nothing
 * done) if its footprint does not fit the budget next to the resident and
 * preparing requests now, or if it is TOF and those requests are not (or
 * the reverse: a batch is all-TOF or all-non-TOF); LMTOF_ENOMEM if it can
 * never fit.
 * Without LMTOF_REQ_BACKGROUND the preparation runs on the pool's stream
 * before the call returns (and no step runs meanwhile); the caller may free
 * the events on return.  With it, the call reserves the footprint and
 * returns at once; a thread of the pool prepares the request on a second
 * stream of the device (default priority), concurrently with the steps of
 * the active requests, and the request joins the batch at the first
 * lmtof_pool_step after its preparation has finished.  The events must then
 * stay valid and unchanged until lmtof_pool_poll has reported the request
 * done (or failed), or the pool is destroyed.  A failed preparation is
 * reported by lmtof_pool_poll for that id. */
int lmtof_pool_submit(lmtof_pool *pool, const lmtof_request *req, int64_t *id);
/* One batched iteration over all active requests (requests whose
 * background preparation has finished join first); *n_active receives how
 * many were active (0: nothing to do now, though background preparations
 * may still be running).  Requests that reach their iteration count become
 * finished (images kept until polled). */
int lmtof_pool_step(lmtof_pool *pool, int *n_active);
/* *done = 1 and the image copied to out (nx*ny*nz floats in `mem`) if
 * request id has finished; the request is then released.  *done = 0 if it
 * is still being prepared or running.  EINVAL for an unknown id; the code
 * of a failed background preparation (the request is then released). */
int lmtof_pool_poll(lmtof_pool *pool, int64_t id, int *done, float *out, int64_t n, int mem);
/* Bytes reserved, budget, active and finished-but-unpolled request counts
 * (requests being prepared in the background count in `used` only). */
int lmtof_pool_info(const lmtof_pool *pool, int64_t *used, int64_t *budget, int *n_active, int *n_finished);

#ifdef __cplusplus
}
#endif

#endif /* LMTOF_H */

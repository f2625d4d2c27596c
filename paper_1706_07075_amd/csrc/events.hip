// Event ingest for gfx950: validation, packing and the coherence bucketing sort.
//
// List-mode data (arXiv 1706.07075, Section 1: events processed one by one,
// chosen for large axial field-of-view 3D data) arrive as endpoint pairs
// plus a time difference.  At load every event is checked (finite values,
// distinct endpoints, and for packed storage int16 range at 0.1 mm and a
// binary16-representable dt), optionally packed to 16 bytes, and reordered
// by a counting sort on an integer key:
//   key = ((((region * ncz + bz) * ncy + by) * ncx + bx) * n_dir + dir) * n_sub + sub,
// where (bx, by, bz) is the 16^3-voxel brick holding the TOF centre, dir
// bins the undirected line direction (azimuth over [0, pi), elevation) and
// sub is the sub-cell of the brick holding the centre.  A wavefront of
// consecutive events then traces near-parallel, co-located rays (its image
// gathers share cache lines), and the events whose windows cross a given
// brick - those centred in it and, from each neighbour, the few direction
// bins pointing at it - form a few long runs of the stored order, so the
// brick-parallel back projection reads them nearly contiguously.  MLEM
// itself does not depend on event order; the permutation is kept so
// per-event inputs and outputs stay in the caller's order.  The region
// index (TOF-assisted data division, Section 2.5) is the most significant
// part of the key, and bricks are counted from each region sub-volume's
// first plane, so each region's events are contiguous and its bricks
// align with the ones its back projection uses.  The
// region's events end up contiguous.
#include "lmtof_internal.h"

#include <hip/hip_fp16.h>

namespace lmtof {
namespace {

constexpr int kBlock = 256;

struct RawEvent {
    float p[7];
};

// Read raw event i: 0 = float32 x 7 (caller), 1 = packed 16 B, 2 = stored plain (float32 x 8).
__device__ __forceinline__ void read_raw(const void *raw, int fmt, int64_t i, float p[7], bool &fin) {
    if (fmt == 2) {
        const float *e = reinterpret_cast<const float *>(raw) + 8 * i;
#pragma unroll
        for (int k = 0; k < 7; ++k) p[k] = e[k];
        fin = true;
    } else if (fmt == 0) {
        const float *e = reinterpret_cast<const float *>(raw) + 7 * i;
#pragma unroll
        for (int k = 0; k < 7; ++k) p[k] = e[k];
        fin = true;
#pragma unroll
        for (int k = 0; k < 7; ++k) fin = fin && isfinite(p[k]);
    } else {
        const uint4 w = reinterpret_cast<const uint4 *>(raw)[i];
        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int16_t q = (int16_t)((ww[k >> 1] >> (16 * (k & 1))) & 0xffffu);
            p[k] = (float)q * 0.1f;
        }
        __half_raw hr;
        hr.x = (unsigned short)(w.w & 0xffffu);
        p[6] = __half2float(__half(hr));
        fin = isfinite(p[6]);
    }
}

__device__ __forceinline__ uint32_t event_key(const KeyGeom &g, const float p[7]) {
    float dx = p[3] - p[0], dy = p[4] - p[1], dz = p[5] - p[2];
    float iL = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    float ux = dx * iL, uy = dy * iL, uz = dz * iL;
    float sh = g.tof ? g.half_c * p[6] : 0.0f;
    float mx = fmaf(sh, ux, 0.5f * (p[0] + p[3]));
    float my = fmaf(sh, uy, 0.5f * (p[1] + p[4]));
    float mz = fmaf(sh, uz, 0.5f * (p[2] + p[5]));
    uint32_t region = 0;
    float z0 = g.oz;
    if (g.n_regions > 1) {
        int r = 0;
        for (int k = 1; k < g.n_regions; ++k)
            if (mz >= g.region_z[k]) r = k;
        region = (uint32_t)r;
        z0 = g.region_z0[r];
    }
    if (!g.sort) return region;
    const float fx = (mx - g.ox) * g.bx_inv, fy = (my - g.oy) * g.by_inv, fz = (mz - z0) * g.bz_inv;
    const int bx = min(max((int)floorf(fx), 0), g.ncx - 1);
    const int by = min(max((int)floorf(fy), 0), g.ncy - 1);
    const int bz = min(max((int)floorf(fz), 0), g.ncz - 1);
    const int sx = min(max((int)floorf((fx - (float)bx) * (float)g.nsx), 0), g.nsx - 1);
    const int sy = min(max((int)floorf((fy - (float)by) * (float)g.nsy), 0), g.nsy - 1);
    const int sz = min(max((int)floorf((fz - (float)bz) * (float)g.nsz), 0), g.nsz - 1);
    // undirected line: canonical direction has uy > 0 (or uy = 0, ux >= 0)
    if (uy < 0.0f || (uy == 0.0f && ux < 0.0f)) {
        ux = -ux;
        uy = -uy;
        uz = -uz;
    }
    const float phi = atan2f(uy, ux);  // [0, pi]
    int bp = (int)(phi * (float)g.n_phi * 0.318309886f);
    int bl = (int)((uz + 1.0f) * 0.5f * (float)g.n_lam);
    bp = min(max(bp, 0), g.n_phi - 1);
    bl = min(max(bl, 0), g.n_lam - 1);
    const uint32_t brick = ((region * (uint32_t)g.ncz + bz) * (uint32_t)g.ncy + by) * (uint32_t)g.ncx + bx;
    const uint32_t dir = (uint32_t)(bp * g.n_lam + bl);
    const uint32_t sub = (uint32_t)((sz * g.nsy + sy) * g.nsx + sx);
    return (brick * (uint32_t)(g.n_phi * g.n_lam) + dir) * (uint32_t)(g.nsx * g.nsy * g.nsz) + sub;
}

// Runs of equal keys among a wavefront's lanes (lane order): whether this
// lane starts a run, the lane that starts its run and the run's length.
// Every lane of the wavefront must be active; lanes without a key pass a
// value no key takes, distinct per lane.  Events re-sorted from bucketed
// order arrive in long runs of one key, whose same-address atomics would
// serialise; one atomic per run takes their place.
struct KeyRun {
    bool head;
    int start, len;
};
__device__ __forceinline__ KeyRun key_run(uint32_t key) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t prev = (uint32_t)__shfl_up((int)key, 1, 64);
    KeyRun r;
    r.head = lane == 0 || key != prev;
    const unsigned long long heads = __ballot(r.head);
    const unsigned long long below = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
    r.start = 63 - __clzll((long long)(heads & below));
    const unsigned long long above = heads & ~below;
    r.len = (above ? __ffsll((long long)above) - 1 : 64) - r.start;
    return r;
}

// A value no key takes (keys stay below 2^26), distinct per lane.
__device__ __forceinline__ uint32_t no_key() { return 0xffffff00u | (threadIdx.x & 63u); }

__global__ void __launch_bounds__(kBlock) k_ingest_keys(const void *__restrict__ raw, int fmt, int64_t n, KeyGeom g,
                                                        int check_pack, uint32_t *__restrict__ keys,
                                                        uint32_t *__restrict__ hist, uint32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t key = no_key();
    if (i < n) {
        float p[7];
        bool fin;
        read_raw(raw, fmt, i, p, fin);
        uint32_t e = 0;
        if (!fin) e |= 1u;
        if (p[0] == p[3] && p[1] == p[4] && p[2] == p[5]) e |= 2u;
        if (check_pack && fmt == 0 && fin) {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if (fabsf(rintf(p[k] * 10.0f)) > 32767.0f) e |= 4u;
            if (fabsf(p[6]) > 65504.0f) e |= 8u;
        }
        if (e) {
            atomicOr(err, e);
            if (keys) keys[i] = 0;
        } else if (keys) {
            key = event_key(g, p);
            keys[i] = key;
        }
    }
    if (!keys) return;  // (uniform)
    const KeyRun run = key_run(key);
    if (run.head && key != no_key()) atomicAdd(hist + key, (uint32_t)run.len);
}

// ---- exclusive scan: per-block sums, scan of the sums, per-block scan with offset
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sm, uint32_t &total) {
    // inclusive wave scan
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sm[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            uint32_t t = sm[w];
            sm[w] = run;
            run += t;
        }
        sm[blockDim.x >> 6] = run;
    }
    __syncthreads();
    total = sm[blockDim.x >> 6];
    uint32_t res = x - v + sm[wid];
    __syncthreads();
    return res;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tile_sums(const uint32_t *__restrict__ d, int64_t n,
                                                               uint32_t *__restrict__ sums) {
    __shared__ uint32_t sm[kScanBlock / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) v += d[base + k];
    uint32_t tot;
    block_excl_scan(v, sm, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(uint32_t *__restrict__ sums, int64_t m) {
    __shared__ uint32_t sm[kScanBlock / 64 + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < m; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        uint32_t v = i < m ? sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, sm, tot);
        if (i < m) sums[i] = ex + carry;
        carry += tot;
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(uint32_t *__restrict__ d, int64_t n,
                                                           const uint32_t *__restrict__ sums) {
    __shared__ uint32_t sm[kScanBlock / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t loc[kScanItems];
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = (base + k < n) ? d[base + k] : 0u;
        v += loc[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(v, sm, tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) d[base + k] = ex;
        ex += loc[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter(const void *__restrict__ raw, int fmt, int64_t n,
                                                    const uint32_t *__restrict__ keys, uint32_t *__restrict__ cursor,
                                                    int store_packed, void *__restrict__ store,
                                                    int64_t *__restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t pos = i;
    if (cursor) {  // (uniform)
        const uint32_t key = i < n ? keys[i] : no_key();
        const KeyRun run = key_run(key);
        uint32_t base = 0;
        if (run.head && i < n) base = atomicAdd(cursor + key, (uint32_t)run.len);
        pos = (int64_t)(uint32_t)__shfl((int)base, run.start, 64) + ((int)(threadIdx.x & 63u) - run.start);
    }
    if (i >= n) return;
    perm[pos] = i;
    if (fmt == 1 && store_packed) {
        reinterpret_cast<uint4 *>(store)[pos] = reinterpret_cast<const uint4 *>(raw)[i];
        return;
    }
    float p[7];
    bool fin;
    read_raw(raw, fmt, i, p, fin);
    if (store_packed) {
        // round half to even at 0.1 mm; dt to the nearest binary16
        uint32_t q[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = (uint32_t)(uint16_t)(int16_t)(int)rintf(p[k] * 10.0f);
        const __half h = __float2half_rn(p[6]);
        const uint32_t hb = (uint32_t)__half_raw(h).x;
        reinterpret_cast<uint4 *>(store)[pos] =
            make_uint4(q[0] | (q[1] << 16), q[2] | (q[3] << 16), q[4] | (q[5] << 16), hb);
    } else {
        float4 *o = reinterpret_cast<float4 *>(store) + 2 * pos;
        o[0] = make_float4(p[0], p[1], p[2], p[3]);
        o[1] = make_float4(p[4], p[5], p[6], 0.0f);
    }
}

__global__ void k_gather_perm(const float *__restrict__ src, const int64_t *__restrict__ perm, int64_t n,
                              float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_scatter_perm(const float *__restrict__ src, const int64_t *__restrict__ perm, int64_t n,
                               float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

__global__ void k_unpermute_packed(const uint4 *__restrict__ src, const int64_t *__restrict__ perm, int64_t n,
                                   uint4 *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

__global__ void k_gather_perm_i64(const int64_t *__restrict__ src, const int64_t *__restrict__ perm, int64_t n,
                                  int64_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_fill_by_perm(const int64_t *__restrict__ perm, int64_t n, int32_t value,
                               int32_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = value;
}

dim3 grid1(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

uint32_t key_count(const KeyGeom &g) {
    const uint64_t nr = g.n_regions > 1 ? (uint64_t)g.n_regions : 1u;
    if (!g.sort) return (uint32_t)nr;
    return (uint32_t)(nr * g.ncx * g.ncy * g.ncz * g.n_phi * g.n_lam * g.nsx * g.nsy * g.nsz);
}

hipError_t launch_ingest_keys(const Launch &L, const void *raw, int fmt, int64_t n, const KeyGeom &g,
                              int check_pack, uint32_t *keys, uint32_t *hist, uint32_t *err) {
    KeyGeom gg = g;
    void *args[] = {&raw, &fmt, &n, &gg, &check_pack, &keys, &hist, &err};
    return do_launch(L, reinterpret_cast<const void *>(&k_ingest_keys), grid1(n), dim3(kBlock), 0, args);
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_exclusive_scan(const Launch &L, uint32_t *data, int64_t n, uint32_t *tmp) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    void *a1[] = {&data, &n, &tmp};
    hipError_t e = do_launch(L, reinterpret_cast<const void *>(&k_scan_tile_sums), dim3((unsigned)tiles),
                             dim3(kScanBlock), 0, a1);
    if (e != hipSuccess) return e;
    int64_t m = tiles;
    void *a2[] = {&tmp, &m};
    e = do_launch(L, reinterpret_cast<const void *>(&k_scan_sums), dim3(1), dim3(kScanBlock), 0, a2);
    if (e != hipSuccess) return e;
    void *a3[] = {&data, &n, &tmp};
    return do_launch(L, reinterpret_cast<const void *>(&k_scan_apply), dim3((unsigned)tiles), dim3(kScanBlock), 0,
                     a3);
}

hipError_t launch_scatter_events(const Launch &L, const void *raw, int fmt, int64_t n, const uint32_t *keys,
                                 uint32_t *cursor, int store_packed, void *store, int64_t *perm) {
    void *args[] = {&raw, &fmt, &n, &keys, &cursor, &store_packed, &store, &perm};
    return do_launch(L, reinterpret_cast<const void *>(&k_scatter), grid1(n), dim3(kBlock), 0, args);
}

hipError_t launch_gather_by_perm(const Launch &L, const float *src_caller, const int64_t *perm, int64_t n,
                                 float *dst_stored) {
    void *args[] = {&src_caller, &perm, &n, &dst_stored};
    return do_launch(L, reinterpret_cast<const void *>(&k_gather_perm), grid1(n), dim3(kBlock), 0, args);
}

hipError_t launch_scatter_by_perm(const Launch &L, const float *src_stored, const int64_t *perm, int64_t n,
                                  float *dst_caller) {
    void *args[] = {&src_stored, &perm, &n, &dst_caller};
    return do_launch(L, reinterpret_cast<const void *>(&k_scatter_perm), grid1(n), dim3(kBlock), 0, args);
}

hipError_t launch_fill_by_perm(const Launch &L, const int64_t *perm, int64_t n, int32_t value, int32_t *dst_caller) {
    void *args[] = {&perm, &n, &value, &dst_caller};
    return do_launch(L, reinterpret_cast<const void *>(&k_fill_by_perm), grid1(n), dim3(kBlock), 0, args);
}

hipError_t launch_compose_perm(const Launch &L, const int64_t *outer, const int64_t *inner, int64_t n,
                               int64_t *out) {
    void *args[] = {&outer, &inner, &n, &out};
    return do_launch(L, reinterpret_cast<const void *>(&k_gather_perm_i64), grid1(n), dim3(kBlock), 0, args);
}

hipError_t launch_unpermute_packed(const Launch &L, const uint4 *store, const int64_t *perm, int64_t n,
                                   uint4 *out) {
    void *args[] = {&store, &perm, &n, &out};
    return do_launch(L, reinterpret_cast<const void *>(&k_unpermute_packed), grid1(n), dim3(kBlock), 0, args);
}

}  // namespace lmtof

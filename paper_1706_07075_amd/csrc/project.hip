// TOF-weighted list-mode projector for gfx950: forward + ratio, brick-owned
// back projection, and the brick item lists they run on.
//
// Model (arXiv 1706.07075, Sections 2.3-2.4): every event is inserted into
// the image through a Gaussian TOF kernel centred on the annihilation point
// that its time difference gives along the line of response, normalised so
// that its weights along the line sum to one.  Here the kernel is truncated
// at +-K sigma, renormalised, and integrated exactly over each piece of the
// line inside a voxel (Siddon-style traversal):
//   a_ij = Phi(t_b) - Phi(t_a),  Phi(t) = erf(t / (sigma sqrt 2)) / (2 erf(K / sqrt 2)),
// for the piece [t_a, t_b] of r(t) = mu + t u in voxel j.  Without TOF the
// weight is the piece length.
//
// GPU design.
//  * Rays are parametrised from the TOF centre mu (|t| <= K sigma), and mu is
//    kept relative to an integer anchor plane (formed with error-free FP32
//    transformations), so a plane crossing (k - j) v - d is resolved to
//    ~1e-6 mm anywhere in a 2.4 m field of view.  Every crossing comes from
//    its integer plane index, never by accumulating steps.  A brick face
//    is a voxel plane, so the crossing where one brick's piece ends is
//    bitwise the one where the next begins and the weights telescope.
//  * Phi comes from an LDS table (the paper keeps its TOF samples in a
//    look-up table too): 1024 nodes over [-K, K] sigma, each holding the value
//    and the first- and second-order Taylor coefficients, so one 16-byte LDS
//    read and two FMAs give Phi to ~2e-9, with no divergent branch.
//  * Forward + ratio is event-parallel: one lane per event, events bucketed
//    at load so a wavefront traces near-parallel, co-located rays and its
//    image gathers coalesce; the lane keeps f_i and writes r_i = 1 / f_i.
//  * Back projection is brick-parallel.  At load every event's window is cut
//    into pieces per 16^3-voxel brick (item lists), and each brick's list
//    into chunks of bounded length.  One workgroup takes one chunk: it
//    accumulates a_ij r_i with LDS atomics and writes its tile with plain
//    stores; a small kernel adds a brick's chunk tiles into b.  There is no
//    global atomic on the image (device-scope FP32 atomics sustain only
//    ~21 G/s on this part, a third of a random gather's rate).  Chunks are
//    launched largest first so the uneven work balances across CUs.
#include "lmtof_internal.h"

#include <hip/hip_fp16.h>

namespace lmtof {
namespace {

constexpr float kInf = __builtin_huge_valf();
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A ray r(t) = mu + t u, with mu held relative to an anchor voxel plane:
// mu_a = o_a + j_a v_a + d_a, |d_a| <~ v_a.  Plane k on axis a then lies at
// (k - j_a) v_a - d_a from mu, which FP32 resolves to ~1e-6 mm whatever the
// absolute position (1.2 m from the centre an absolute FP32 coordinate
// carries ~6e-5 mm of rounding).
struct Ray {
    int jx, jy, jz;    // anchor plane indices
    float dx, dy, dz;  // mu - anchor plane (mm)
    float ux, uy, uz;  // unit direction P1 -> P2
    float t0, t1;      // window (mm from mu)
};

// Decode stored event i (plain: 2 x float4; packed: int16 x 6 at 0.1 mm +
// binary16 dt).  Endpoints come as double-float pairs p = h + l: plain
// coordinates are exact FP32 (l = 0); a packed coordinate q * 0.1 mm is not,
// so l holds the FMA residual of q * 0.1f plus q * (0.1 - 0.1f), keeping the
// decoded endpoint exact to ~1e-15 relative (an FP32 decode alone would be
// off by up to 6e-5 mm 1.2 m from the centre).
struct EventGeom {
    float h[6], l[6];  // P1.xyz, P2.xyz
    float dt;
};

__device__ __forceinline__ void load_event(const void *events, int packed, int64_t i, EventGeom &ev) {
    if (!packed) {
        const f32x4 *e = reinterpret_cast<const f32x4 *>(events) + 2 * i;
        const f32x4 a = __builtin_nontemporal_load(e), b = __builtin_nontemporal_load(e + 1);
        ev.h[0] = a[0]; ev.h[1] = a[1]; ev.h[2] = a[2]; ev.h[3] = a[3];
        ev.h[4] = b[0]; ev.h[5] = b[1]; ev.dt = b[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) ev.l[k] = 0.0f;
    } else {
        const u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(events) + i);
        const float tenth = 0.1f, tenth_lo = -1.4901161e-09f;  // 0.1 - 0.1f
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float q = (float)(int16_t)((w[k >> 1] >> (16 * (k & 1))) & 0xffffu);
            ev.h[k] = q * tenth;
            ev.l[k] = fmaf(q, tenth, -ev.h[k]) + q * tenth_lo;
        }
        __half_raw hr;
        hr.x = (unsigned short)(w[3] & 0xffffu);
        ev.dt = __half2float(__half(hr));
    }
}

// Error-free transformations (Knuth's TwoSum; TwoProd with an FMA): a + b =
// s + e and a * b = p + e exactly in FP32.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e) {
    p = a * b;
    e = fmaf(a, b, -p);
}

struct RayInv {
    float ix, iy, iz;  // 1 / u (0 when u = 0)
    int sx, sy, sz;    // sign of u
};

// Offset from mu of plane k on an axis with anchor j, offset d, voxel size v.
__device__ __forceinline__ float plane_rel(int k, int j, float v, float d) { return fmaf((float)(k - j), v, -d); }

// Clip the line to planes [klo, khi) of one axis.
__device__ __forceinline__ void slab(int klo, int khi, int j, float v, float d, float iu, int su, float &t0,
                                     float &t1) {
    const float lo = plane_rel(klo, j, v, d), hi = plane_rel(khi, j, v, d);
    if (su) {
        const float a = lo * iu, b = hi * iu;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else if (!(lo <= 0.0f && hi > 0.0f)) {
        t0 = kInf;
        t1 = -kInf;
    }
}

// Anchor one axis: mu = (mh + ml) = o + j v + d.
__device__ __forceinline__ void anchor(float mh, float ml, float o, float v, float iv, int &j, float &d) {
    j = (int)rintf((mh - o) * iv);
    const float q = fmaf((float)j, v, o);
    d = (mh - q) + ml;
}

// Event geometry: direction, anchored TOF centre and window (clipped to the
// grid box and, with TOF, to +-K sigma).  False if the window is empty.
// The midpoint and the TOF shift along the endpoint difference are formed
// exactly (double-float); the shift is scaled along d = P2 - P1 itself, so
// rounding of the scale factor only moves mu along the line.
__device__ __forceinline__ bool make_ray(const Problem &P, const void *events, int64_t i, Ray &r, RayInv &q) {
    EventGeom ev;
    load_event(events, P.packed, i, ev);
    float dh[3], dl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        two_sum(ev.h[3 + k], -ev.h[k], dh[k], dl[k]);
        dl[k] += ev.l[3 + k] - ev.l[k];
    }
    const float iL = 1.0f / sqrtf(dh[0] * dh[0] + dh[1] * dh[1] + dh[2] * dh[2]);
    r.ux = dh[0] * iL;
    r.uy = dh[1] * iL;
    r.uz = dh[2] * iL;
    const float kappa = P.tof ? P.half_c * ev.dt * iL : 0.0f;  // mu = (P1 + P2) / 2 + kappa (P2 - P1)
    auto centre = [&](int k, float o, float v, float iv, int &j, float &d) {
        float sh, se, ph, pe, mh, me;
        two_sum(ev.h[k], ev.h[3 + k], sh, se);
        se += ev.l[k] + ev.l[3 + k];
        two_prod(kappa, dh[k], ph, pe);
        two_sum(0.5f * sh, ph, mh, me);
        const float ml = me + (0.5f * se + fmaf(kappa, dl[k], pe));
        anchor(mh, ml, o, v, iv, j, d);
    };
    centre(0, P.ox, P.vx, P.ivx, r.jx, r.dx);
    centre(1, P.oy, P.vy, P.ivy, r.jy, r.dy);
    centre(2, P.oz, P.vz, P.ivz, r.jz, r.dz);
    q.sx = (r.ux > 0.0f) - (r.ux < 0.0f);
    q.sy = (r.uy > 0.0f) - (r.uy < 0.0f);
    q.sz = (r.uz > 0.0f) - (r.uz < 0.0f);
    q.ix = q.sx ? 1.0f / r.ux : 0.0f;
    q.iy = q.sy ? 1.0f / r.uy : 0.0f;
    q.iz = q.sz ? 1.0f / r.uz : 0.0f;
    float t0 = -kInf, t1 = kInf;
    slab(0, P.nx, r.jx, P.vx, r.dx, q.ix, q.sx, t0, t1);
    slab(0, P.ny, r.jy, P.vy, r.dy, q.iy, q.sy, t0, t1);
    slab(0, P.nz, r.jz, P.vz, r.dz, q.iz, q.sz, t0, t1);
    if (P.tof) {
        t0 = fmaxf(t0, -P.k_sigma);
        t1 = fminf(t1, P.k_sigma);
    }
    r.t0 = t0;
    r.t1 = t1;
    return t0 < t1;
}

// Voxel index along one axis at parameter t.
__device__ __forceinline__ int voxel_at(float t, float u, int j, float d, float iv) {
    return j + (int)floorf(fmaf(t, u, d) * iv);
}

// Truncated-kernel CDF from the LDS table: node k at u_k = -K + k h (sigma
// units) holds (Phi_k, Phi'_k h, Phi''_k h^2 / 2); pos = t * lut_a + lut_b.
struct Cdf {
    const float4 *tab;
    float a, b;
    __device__ __forceinline__ float operator()(float t) const {
        const float pos = fmaf(t, a, b);
        const float kf = fminf(fmaxf(rintf(pos), 0.0f), (float)(kLutN - 1));
        const float dp = pos - kf;
        const float4 e = tab[(int)kf];
        return fmaf(dp, fmaf(dp, e.z, e.y), e.x);
    }
};

// A voxel box the traversal is confined to (the whole grid or one brick),
// with the strides of the index it reports.
struct Box {
    int x0, y0, z0;  // first voxel (global indices)
    int nx, ny, nz;  // extent
    int sy, sz;      // strides of the reported index
};

// Walk the voxels of ray r between ta and tb (already inside the box) and
// call visit(j, a) for every piece; j is box-local.  A plane tie gives a
// zero-length piece (a = 0).
template <bool TOF, class Visit>
__device__ __forceinline__ void walk(const Problem &P, const Ray &r, const RayInv &q, float ta, float tb,
                                     const Box &B, const Cdf &cdf, Visit &&visit) {
    int ix = voxel_at(ta, r.ux, r.jx, r.dx, P.ivx);
    int iy = voxel_at(ta, r.uy, r.jy, r.dy, P.ivy);
    int iz = voxel_at(ta, r.uz, r.jz, r.dz, P.ivz);
    ix = min(max(ix, B.x0), B.x0 + B.nx - 1);
    iy = min(max(iy, B.y0), B.y0 + B.ny - 1);
    iz = min(max(iz, B.z0), B.z0 + B.nz - 1);
    // next plane on each axis, from its global index
    const int ux1 = q.sx > 0, uy1 = q.sy > 0, uz1 = q.sz > 0;
    float tnx = q.sx ? plane_rel(ix + ux1, r.jx, P.vx, r.dx) * q.ix : kInf;
    float tny = q.sy ? plane_rel(iy + uy1, r.jy, P.vy, r.dy) * q.iy : kInf;
    float tnz = q.sz ? plane_rel(iz + uz1, r.jz, P.vz, r.dz) * q.iz : kInf;
    int lx = ix - B.x0, ly = iy - B.y0, lz = iz - B.z0;
    int j = lx + B.sy * ly + B.sz * lz;
    const int djy = q.sy * B.sy, djz = q.sz * B.sz;
    float t = ta;
    float c = TOF ? cdf(ta) : 0.0f;
    const int max_steps = B.nx + B.ny + B.nz + 2;
    for (int step = 0; step < max_steps; ++step) {
        const float tmin = fminf(fminf(tnx, tny), tnz);
        const bool last = tmin >= tb;
        const float tn = fmaxf(fminf(tmin, tb), t);
        float a;
        if (TOF) {
            const float cn = cdf(tn);
            a = cn - c;
            c = cn;
        } else {
            a = tn - t;
        }
        visit(j, a);
        if (last) break;
        t = tn;
        if (tnx == tmin) {
            lx += q.sx;
            if ((unsigned)lx >= (unsigned)B.nx) break;
            j += q.sx;
            tnx = plane_rel(lx + B.x0 + ux1, r.jx, P.vx, r.dx) * q.ix;
        } else if (tny == tmin) {
            ly += q.sy;
            if ((unsigned)ly >= (unsigned)B.ny) break;
            j += djy;
            tny = plane_rel(ly + B.y0 + uy1, r.jy, P.vy, r.dy) * q.iy;
        } else {
            lz += q.sz;
            if ((unsigned)lz >= (unsigned)B.nz) break;
            j += djz;
            tnz = plane_rel(lz + B.z0 + uz1, r.jz, P.vz, r.dz) * q.iz;
        }
    }
}

__device__ __forceinline__ Box grid_box(const Problem &P) {
    Box B;
    B.x0 = B.y0 = B.z0 = 0;
    B.nx = P.nx;
    B.ny = P.ny;
    B.nz = P.nz;
    B.sy = P.nx;
    B.sz = P.nx * P.ny;
    return B;
}

// Brick (bx, by, bz) of problem P as a box with LDS-tile strides.
__device__ __forceinline__ Box brick_box(const Problem &P, int bx, int by, int bz) {
    Box B;
    B.x0 = bx * kBrickX;
    B.y0 = by * kBrickY;
    B.z0 = bz * kBrickZ;
    B.nx = min(kBrickX, P.nx - B.x0);
    B.ny = min(kBrickY, P.ny - B.y0);
    B.nz = min(kBrickZ, P.nz - B.z0);
    B.sy = kBrickX;
    B.sz = kBrickX * kBrickY;
    return B;
}

// Part of the window inside box B (same plane formulas as the walk).
__device__ __forceinline__ void clip_to_box(const Problem &P, const Ray &r, const RayInv &q, const Box &B,
                                            float &ta, float &tb) {
    ta = r.t0;
    tb = r.t1;
    slab(B.x0, B.x0 + B.nx, r.jx, P.vx, r.dx, q.ix, q.sx, ta, tb);
    slab(B.y0, B.y0 + B.ny, r.jy, P.vy, r.dy, q.iy, q.sy, ta, tb);
    slab(B.z0, B.z0 + B.nz, r.jz, P.vz, r.dz, q.iz, q.sz, ta, tb);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int find_problem(const Problem *probs, int n_probs, int64_t c) {
    int p = n_probs - 1;
    while (p > 0 && probs[p].chunk_begin > c) --p;
    return p;
}

__device__ __forceinline__ int find_brick_problem(const Problem *probs, int n_probs, uint32_t b) {
    int p = n_probs - 1;
    while (p > 0 && (uint32_t)probs[p].brick_base > b) --p;
    return p;
}

__device__ __forceinline__ void stage_lut(float4 *lds, const float4 *src) {
    for (int k = threadIdx.x; k < kLutN; k += blockDim.x) lds[k] = src[k];
}

// Forward projection of one chunk of events.  mode 0 (MLEM): out[i] =
// 1 / f_i (0 if f_i <= 0) plus per-chunk partials (events with f > 0, sum
// of log f); mode 1: out[i] = f_i.  out is indexed by stored event position.
template <bool TOF>
__global__ void __launch_bounds__(kForwardBlock) k_forward(const Problem *__restrict__ probs, int n_probs, int ept,
                                                           int mode, int *__restrict__ part_neff,
                                                           double *__restrict__ part_ll) {
    __shared__ float4 lut[kLutN];
    __shared__ int s_n[kForwardBlock / 64];
    __shared__ double s_l[kForwardBlock / 64];
    const int64_t c = blockIdx.x;
    const Problem P = probs[find_problem(probs, n_probs, c)];
    if (TOF) stage_lut(lut, P.lut);
    __syncthreads();
    const Cdf cdf{lut, P.lut_a, P.lut_b};
    const Box B = grid_box(P);
    const float *__restrict__ x = P.x;
    float *__restrict__ out = P.rw;
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    int neff = 0;
    float ll = 0.0f;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        RayInv q;
        float f = 0.0f;
        if (make_ray(P, P.events, i, r, q))
            walk<TOF>(P, r, q, r.t0, r.t1, B, cdf, [&](int j, float a) { f = fmaf(a, x[j], f); });
        if (mode == 0) {
            const bool pos = f > 0.0f;
            neff += pos;
            ll += pos ? logf(f) : 0.0f;
            out[i] = pos ? 1.0f / f : 0.0f;
        } else {
            out[i] = f;
        }
    }
    if (mode == 0) {
        const int wn = wave_sum(neff);
        const double wl = wave_sum((double)ll);
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) {
            s_n[wid] = wn;
            s_l[wid] = wl;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tn = 0;
            double tl = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                tn += s_n[w];
                tl += s_l[w];
            }
            part_neff[c] = tn;
            part_ll[c] = tl;
        }
    }
}

// Back projection, in three launches over the brick chunks.
//
// The LDS accumulation is 64-bit fixed point: FP32 LDS atomic adds run at
// ~0.2 T/s on this part, 64-bit integer ones at ~2.8 T/s.  A brick's
// contributions a w (each an FP32 product) are scaled by S = 2^e and
// rounded to integers, e being chosen per brick from its item count n, the
// problem's bound a_max on a piece weight and the brick's largest |w|, so
// that n a_max w_max S < 2^62: no sum can overflow.  Chunk tiles stay 64-bit
// and are added exactly, so b does not depend on how the brick's items are
// ordered or cut into chunks: the result is deterministic, and the same
// for a problem run alone or batched with others.
//
// Brick table entry (brick id, first tile slot, end tile slot, items in the
// brick); chunk (brick table index, first item, end item, tile slot).

// 1. Largest |w| over each chunk's items, per tile slot.
__global__ void __launch_bounds__(256) k_chunk_wmax(const Problem *__restrict__ probs, int n_probs,
                                                    const uint4 *__restrict__ chunks,
                                                    const uint4 *__restrict__ bricks) {
    __shared__ float s_m[4];
    const uint4 ch = chunks[blockIdx.x];
    const uint4 br = bricks[ch.x];
    const Problem &P = probs[find_brick_problem(probs, n_probs, br.x)];
    const uint32_t *__restrict__ items = P.items;
    const float *__restrict__ w = P.rw;
    float wm = 0.0f;
    for (uint32_t k = ch.y + threadIdx.x; k < ch.z; k += blockDim.x) wm = fmaxf(wm, fabsf(w[items[k]]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wm = fmaxf(wm, __shfl_xor(wm, off, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = wm;
    __syncthreads();
    if (threadIdx.x == 0) P.wmax[ch.w] = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
}

// Fixed-point exponent of a brick (same value in every chunk and the reduce).
__device__ __forceinline__ int brick_exponent(const Problem &P, const uint4 &br, float &wmax) {
    float wm = 0.0f;
    for (uint32_t sl = br.y; sl < br.z; ++sl) wm = fmaxf(wm, P.wmax[sl]);
    wmax = wm;
    int en, ea, ew;
    frexpf((float)br.w, &en);
    frexpf(P.a_max, &ea);
    frexpf(wm, &ew);
    return min(max(62 - (en + ea + ew), -126), 126);
}

// 2. One chunk: sum over its items of round(a_ij w_i 2^e) in an LDS tile,
//    stored (64-bit) to the chunk's tile slot.
template <bool TOF>
__global__ void __launch_bounds__(kBackBlock) k_back_chunks(const Problem *__restrict__ probs, int n_probs,
                                                            const uint4 *__restrict__ chunks,
                                                            const uint4 *__restrict__ bricks) {
    __shared__ unsigned long long tile[kBrickVox];
    __shared__ float4 lut[kLutN];
    const uint4 ch = chunks[blockIdx.x];
    const uint4 br = bricks[ch.x];
    const uint32_t bid = br.x;
    const Problem P = probs[find_brick_problem(probs, n_probs, bid)];
    const uint32_t bl = bid - (uint32_t)P.brick_base;
    const int bx = (int)(bl % (uint32_t)P.nbx), by = (int)((bl / (uint32_t)P.nbx) % (uint32_t)P.nby),
              bz = (int)(bl / ((uint32_t)P.nbx * (uint32_t)P.nby));
    const Box B = brick_box(P, bx, by, bz);
    const uint32_t *__restrict__ items = P.items;
    const float *__restrict__ w = P.rw;
    for (int k = threadIdx.x; k < kBrickVox; k += blockDim.x) tile[k] = 0ull;
    if (TOF) stage_lut(lut, P.lut);
    __syncthreads();
    float wm;
    const int e = brick_exponent(P, br, wm);
    const float S = ldexpf(1.0f, e);
    const Cdf cdf{lut, P.lut_a, P.lut_b};
    if (wm > 0.0f) {
        for (uint32_t k = ch.y + threadIdx.x; k < ch.z; k += blockDim.x) {
            const uint32_t i = items[k];
            const float ws = w[i] * S;
            if (ws == 0.0f) continue;
            Ray r;
            RayInv q;
            if (!make_ray(P, P.events, (int64_t)i, r, q)) continue;
            float ta, tb;
            clip_to_box(P, r, q, B, ta, tb);
            if (!(ta < tb)) continue;
            walk<TOF>(P, r, q, ta, tb, B, cdf, [&](int j, float a) {
                if (a != 0.0f) atomicAdd(&tile[j], (unsigned long long)__float2ll_rn(a * ws));
            });
        }
    }
    __syncthreads();
    unsigned long long *__restrict__ dst = P.tiles + (size_t)ch.w * kBrickVox;
    for (int k = threadIdx.x; k < kBrickVox; k += blockDim.x) dst[k] = tile[k];
}

// 3. b over one brick = (exact sum of its chunk tiles) 2^-e.
__global__ void __launch_bounds__(256) k_reduce_tiles(const Problem *__restrict__ probs, int n_probs,
                                                      const uint4 *__restrict__ bricks) {
    const uint4 br = bricks[blockIdx.x];
    const Problem &P = probs[find_brick_problem(probs, n_probs, br.x)];
    const uint32_t bl = br.x - (uint32_t)P.brick_base;
    const int bx = (int)(bl % (uint32_t)P.nbx), by = (int)((bl / (uint32_t)P.nbx) % (uint32_t)P.nby),
              bz = (int)(bl / ((uint32_t)P.nbx * (uint32_t)P.nby));
    const Box B = brick_box(P, bx, by, bz);
    float wm;
    const float inv = ldexpf(1.0f, -brick_exponent(P, br, wm));
    float *__restrict__ b = P.b;
    const unsigned long long *__restrict__ tiles = P.tiles;
    for (int k = threadIdx.x; k < kBrickVox; k += blockDim.x) {
        unsigned long long acc = 0ull;
        for (uint32_t sl = br.y; sl < br.z; ++sl) acc += tiles[(size_t)sl * kBrickVox + k];
        const int lx = k % kBrickX, ly = (k / kBrickX) % kBrickY, lz = k / (kBrickX * kBrickY);
        if (lx < B.nx && ly < B.ny && lz < B.nz)
            b[(B.x0 + lx) + (int64_t)P.nx * ((B.y0 + ly) + (int64_t)P.ny * (B.z0 + lz))] =
                __ll2float_rn((long long)acc) * inv;
    }
}

// Per-block open-addressing table in LDS mapping a brick id to a slot.
constexpr int kHashSlots = 1024;
constexpr uint32_t kEmpty = 0xffffffffu;

__device__ __forceinline__ int hash_slot(uint32_t key) { return (int)((key * 2654435761u) >> 22); }

// Slot of key, inserting it if absent; -1 if the table is full.
__device__ __forceinline__ int hash_insert(uint32_t *keys, uint32_t key) {
    int h = hash_slot(key);
    for (int probe = 0; probe < kHashSlots; ++probe) {
        uint32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kEmpty) {
            k = atomicCAS(&keys[h], kEmpty, key);
            if (k == kEmpty) return h;
        }
        if (k == key) return h;
        h = (h + 1) & (kHashSlots - 1);
    }
    return -1;
}

__device__ __forceinline__ int hash_find(const uint32_t *keys, uint32_t key) {
    int h = hash_slot(key);
    for (int probe = 0; probe < kHashSlots; ++probe) {
        const uint32_t k = keys[h];
        if (k == key) return h;
        if (k == kEmpty) return -1;
        h = (h + 1) & (kHashSlots - 1);
    }
    return -1;
}

// Walk one event's window through the brick grid of P and call
// visit(global brick id) for every brick crossed over a positive length.
// Brick faces are voxel planes, so this uses the voxel walk's crossing
// formulas and cuts the window exactly where the brick pieces meet.
template <class Visit>
__device__ __forceinline__ void brick_walk(const Problem &P, const Ray &r, const RayInv &q, Visit &&visit) {
    const int ux1 = q.sx > 0, uy1 = q.sy > 0, uz1 = q.sz > 0;
    int bx = min(max(voxel_at(r.t0, r.ux, r.jx, r.dx, P.ivx), 0), P.nx - 1) / kBrickX;
    int by = min(max(voxel_at(r.t0, r.uy, r.jy, r.dy, P.ivy), 0), P.ny - 1) / kBrickY;
    int bz = min(max(voxel_at(r.t0, r.uz, r.jz, r.dz, P.ivz), 0), P.nz - 1) / kBrickZ;
    float tnx = q.sx ? plane_rel((bx + ux1) * kBrickX, r.jx, P.vx, r.dx) * q.ix : kInf;
    float tny = q.sy ? plane_rel((by + uy1) * kBrickY, r.jy, P.vy, r.dy) * q.iy : kInf;
    float tnz = q.sz ? plane_rel((bz + uz1) * kBrickZ, r.jz, P.vz, r.dz) * q.iz : kInf;
    float t = r.t0;
    const int max_steps = P.nbx + P.nby + P.nbz + 2;
    for (int step = 0; step < max_steps; ++step) {
        const float tmin = fminf(fminf(tnx, tny), tnz);
        const float tn = fminf(tmin, r.t1);
        if (tn > t) visit((uint32_t)P.brick_base + (uint32_t)(bx + P.nbx * (by + P.nby * bz)));
        if (tmin >= r.t1) break;
        t = fmaxf(tn, t);
        if (tnx == tmin) {
            bx += q.sx;
            if ((unsigned)bx >= (unsigned)P.nbx) break;
            tnx = plane_rel((bx + ux1) * kBrickX, r.jx, P.vx, r.dx) * q.ix;
        } else if (tny == tmin) {
            by += q.sy;
            if ((unsigned)by >= (unsigned)P.nby) break;
            tny = plane_rel((by + uy1) * kBrickY, r.jy, P.vy, r.dy) * q.iy;
        } else {
            bz += q.sz;
            if ((unsigned)bz >= (unsigned)P.nbz) break;
            tnz = plane_rel((bz + uz1) * kBrickZ, r.jz, P.vz, r.dz) * q.iz;
        }
    }
}

// Brick item lists.  Counting (fill == 0): ctr[brick] += pieces.  Filling:
// every piece gets a position from ctr[brick]++ (never past end[brick]) and
// P.items[position] = its problem-local event index.  A block first tallies
// its pieces per brick in an LDS hash table, then touches each global
// counter once (bucketed events make whole blocks hit the same few bricks,
// and same-address global atomics serialise); when filling, the block then
// re-walks its events and hands out positions from its reserved ranges.
__global__ void __launch_bounds__(kForwardBlock) k_brick_items(const Problem *__restrict__ probs, int n_probs,
                                                               int ept, uint32_t *__restrict__ ctr,
                                                               const uint32_t *__restrict__ end, int fill) {
    __shared__ uint32_t hkey[kHashSlots], hcnt[kHashSlots], hbase[kHashSlots];
    for (int k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
        hkey[k] = kEmpty;
        hcnt[k] = 0;
    }
    __syncthreads();
    const int64_t c = blockIdx.x;
    const Problem P = probs[find_problem(probs, n_probs, c)];
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    uint32_t *__restrict__ items = const_cast<uint32_t *>(P.items);
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        Ray r;
        RayInv q;
        if (i >= P.n_events || !make_ray(P, P.events, i, r, q)) continue;
        brick_walk(P, r, q, [&](uint32_t key) {
            const int h = hash_insert(hkey, key);
            if (h >= 0) {
                atomicAdd(&hcnt[h], 1u);
            } else if (!fill) {
                atomicAdd(ctr + key, 1u);
            } else {
                const uint32_t pos = atomicAdd(ctr + key, 1u);
                if (pos < end[key]) items[pos] = (uint32_t)i;
            }
        });
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
        if (hkey[k] == kEmpty) continue;
        const uint32_t b = atomicAdd(ctr + hkey[k], hcnt[k]);
        if (fill) {
            hbase[k] = b;
            hcnt[k] = 0;
        }
    }
    if (!fill) return;
    __syncthreads();
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        Ray r;
        RayInv q;
        if (i >= P.n_events || !make_ray(P, P.events, i, r, q)) continue;
        brick_walk(P, r, q, [&](uint32_t key) {
            const int h = hash_find(hkey, key);
            if (h < 0) return;  // placed directly in the first walk
            const uint32_t pos = hbase[h] + atomicAdd(&hcnt[h], 1u);
            if (pos < end[key]) items[pos] = (uint32_t)i;
        });
    }
}

// Diagnostic: voxel pieces visited per chunk and how many have non-zero weight.
template <bool TOF>
__global__ void __launch_bounds__(kForwardBlock) k_count_pieces(const Problem *__restrict__ probs, int n_probs,
                                                                int ept, unsigned long long *__restrict__ part) {
    __shared__ float4 lut[kLutN];
    __shared__ unsigned long long s_c[kForwardBlock / 64], s_z[kForwardBlock / 64];
    const int64_t c = blockIdx.x;
    const Problem P = probs[find_problem(probs, n_probs, c)];
    if (TOF) stage_lut(lut, P.lut);
    __syncthreads();
    const Cdf cdf{lut, P.lut_a, P.lut_b};
    const Box B = grid_box(P);
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    unsigned long long cnt = 0, nz = 0;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        RayInv q;
        if (!make_ray(P, P.events, i, r, q)) continue;
        walk<TOF>(P, r, q, r.t0, r.t1, B, cdf, [&](int, float a) {
            ++cnt;
            nz += (a != 0.0f);
        });
    }
    const unsigned long long wc = wave_sum(cnt), wz = wave_sum(nz);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        s_c[wid] = wc;
        s_z[wid] = wz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            a += s_c[k];
            b += s_z[k];
        }
        part[2 * c] = a;
        part[2 * c + 1] = b;
    }
}

}  // namespace

int64_t project_chunk_events(int block, int ept) { return (int64_t)block * ept; }

hipError_t launch_forward(const Launch &L, bool tof, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept,
                          int mode, int *part_neff, double *part_ll) {
    void *args[] = {&d_probs, &n_probs, &ept, &mode, &part_neff, &part_ll};
    const void *fn = tof ? reinterpret_cast<const void *>(&k_forward<true>)
                         : reinterpret_cast<const void *>(&k_forward<false>);
    return do_launch(L, fn, dim3((unsigned)n_chunks), dim3(kForwardBlock), 0, args);
}

hipError_t launch_back_chunks(const Launch &L, bool tof, const Problem *d_probs, int n_probs, const uint4 *chunks,
                              uint32_t n_chunks, const uint4 *bricks) {
    void *args[] = {&d_probs, &n_probs, &chunks, &bricks};
    const void *fn = tof ? reinterpret_cast<const void *>(&k_back_chunks<true>)
                         : reinterpret_cast<const void *>(&k_back_chunks<false>);
    return do_launch(L, fn, dim3(n_chunks), dim3(kBackBlock), 0, args);
}

hipError_t launch_chunk_wmax(const Launch &L, const Problem *d_probs, int n_probs, const uint4 *chunks,
                             uint32_t n_chunks, const uint4 *bricks) {
    void *args[] = {&d_probs, &n_probs, &chunks, &bricks};
    return do_launch(L, reinterpret_cast<const void *>(&k_chunk_wmax), dim3(n_chunks), dim3(256), 0, args);
}

hipError_t launch_reduce_tiles(const Launch &L, const Problem *d_probs, int n_probs, const uint4 *bricks,
                               uint32_t n_bricks) {
    void *args[] = {&d_probs, &n_probs, &bricks};
    return do_launch(L, reinterpret_cast<const void *>(&k_reduce_tiles), dim3(n_bricks), dim3(256), 0, args);
}

hipError_t launch_brick_items(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept,
                              uint32_t *ctr, const uint32_t *end, int fill) {
    void *args[] = {&d_probs, &n_probs, &ept, &ctr, &end, &fill};
    return do_launch(L, reinterpret_cast<const void *>(&k_brick_items), dim3((unsigned)n_chunks),
                     dim3(kForwardBlock), 0, args);
}

hipError_t launch_count_pieces(const Launch &L, bool tof, const Problem *d_probs, int n_probs, int64_t n_chunks,
                               int ept, unsigned long long *part) {
    void *args[] = {&d_probs, &n_probs, &ept, &part};
    const void *fn = tof ? reinterpret_cast<const void *>(&k_count_pieces<true>)
                         : reinterpret_cast<const void *>(&k_count_pieces<false>);
    return do_launch(L, fn, dim3((unsigned)n_chunks), dim3(kForwardBlock), 0, args);
}

}  // namespace lmtof

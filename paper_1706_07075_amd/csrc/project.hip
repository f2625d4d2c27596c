// TOF-weighted list-mode projector for gfx950 (forward, ratio, back).
//
// Model (arXiv 1706.07075, Sections 2.3-2.4): every event is inserted into
// the image through a Gaussian TOF kernel centred on the annihilation point
// that the time difference gives along the line of response, the kernel
// being normalised so that its weights along the line sum to one.  Here the
// kernel is truncated at +-K sigma, renormalised, and integrated exactly
// over each piece of the line inside a voxel, the pieces coming from a
// Siddon-style traversal: a_ij = [erf(t_b / (sigma sqrt 2)) -
// erf(t_a / (sigma sqrt 2))] / (2 erf(K / sqrt 2)) for the piece [t_a, t_b]
// of the line r(t) = mu + t u in voxel j.  Without TOF the weight is the
// piece length.
//
// GPU design: one lane per event.  The ray is parametrised from the TOF
// centre mu (|t| <= K sigma, so FP32 keeps ~1e-6 mm resolution even 1.2 m
// from the scanner centre), and every plane crossing is computed from its
// integer plane index, never by accumulating steps, so crossings do not
// drift.  The per-piece kernel integral is a difference of consecutive erf
// values, so the weights telescope: they sum to the kernel mass inside the
// window up to one rounding.  The forward pass gathers x_j; the ratio
// 1 / f_i stays in a register; the back pass re-traces the same ray and adds
// a_ij / f_i to b_j with FP32 atomics (MLEM does not depend on the order).
// Events are read with non-temporal loads so they do not evict the image
// from L2 / MALL.
#include "lmtof_internal.h"

#include <hip/hip_fp16.h>

namespace lmtof {
namespace {

constexpr float kInf = __builtin_huge_valf();

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Ray {
    float mx, my, mz;  // TOF centre (mm)
    float ux, uy, uz;  // unit direction P1 -> P2
    float t0, t1;      // window (mm from mu)
};

// Decode stored event i of problem P into endpoints and dt.
__device__ __forceinline__ void load_event(const Problem &P, int64_t i, float &p1x, float &p1y, float &p1z,
                                           float &p2x, float &p2y, float &p2z, float &dt) {
    if (!P.packed) {
        const f32x4 *e = reinterpret_cast<const f32x4 *>(P.events) + 2 * i;
        const f32x4 a = __builtin_nontemporal_load(e), b = __builtin_nontemporal_load(e + 1);
        p1x = a[0]; p1y = a[1]; p1z = a[2]; p2x = a[3];
        p2y = b[0]; p2z = b[1]; dt = b[2];
    } else {
        const u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(P.events) + i);
        const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
        const float q = 0.1f;
        p1x = (float)(int16_t)(w0 & 0xffffu) * q;
        p1y = (float)(int16_t)(w0 >> 16) * q;
        p1z = (float)(int16_t)(w1 & 0xffffu) * q;
        p2x = (float)(int16_t)(w1 >> 16) * q;
        p2y = (float)(int16_t)(w2 & 0xffffu) * q;
        p2z = (float)(int16_t)(w2 >> 16) * q;
        __half_raw hr;
        hr.x = (unsigned short)(w3 & 0xffffu);
        dt = __half2float(__half(hr));
    }
}

// Clip one axis of the line to the slab [lo, hi).
__device__ __forceinline__ void slab(float m, float u, float lo, float hi, float &t0, float &t1) {
    if (u != 0.0f) {
        float iu = 1.0f / u;
        float a = (lo - m) * iu, b = (hi - m) * iu;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else if (!(m >= lo && m < hi)) {
        t0 = kInf;
        t1 = -kInf;
    }
}

// Event geometry: direction, TOF centre and window.  False if the window is empty.
__device__ __forceinline__ bool make_ray(const Problem &P, int64_t i, Ray &r) {
    float p1x, p1y, p1z, p2x, p2y, p2z, dt;
    load_event(P, i, p1x, p1y, p1z, p2x, p2y, p2z, dt);
    float dx = p2x - p1x, dy = p2y - p1y, dz = p2z - p1z;
    float iL = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    r.ux = dx * iL;
    r.uy = dy * iL;
    r.uz = dz * iL;
    float sh = P.tof ? P.half_c * dt : 0.0f;
    r.mx = fmaf(sh, r.ux, 0.5f * (p1x + p2x));
    r.my = fmaf(sh, r.uy, 0.5f * (p1y + p2y));
    r.mz = fmaf(sh, r.uz, 0.5f * (p1z + p2z));
    float t0 = -kInf, t1 = kInf;
    slab(r.mx, r.ux, P.ox, P.hx, t0, t1);
    slab(r.my, r.uy, P.oy, P.hy, t0, t1);
    slab(r.mz, r.uz, P.oz, P.hz, t0, t1);
    if (P.tof) {
        t0 = fmaxf(t0, -P.k_sigma);
        t1 = fminf(t1, P.k_sigma);
    }
    r.t0 = t0;
    r.t1 = t1;
    return t0 < t1;
}

// Walk the voxels of ray r inside its window and call visit(j, a_ij) for
// each piece (a zero-length piece at a plane tie yields a_ij = 0).
template <class Visit>
__device__ __forceinline__ void traverse(const Problem &P, const Ray &r, Visit &&visit) {
    // Entry voxel: the point at t0, clamped (t0 may sit on the grid boundary).
    int ix = (int)floorf((fmaf(r.t0, r.ux, r.mx) - P.ox) * P.ivx);
    int iy = (int)floorf((fmaf(r.t0, r.uy, r.my) - P.oy) * P.ivy);
    int iz = (int)floorf((fmaf(r.t0, r.uz, r.mz) - P.oz) * P.ivz);
    ix = min(max(ix, 0), P.nx - 1);
    iy = min(max(iy, 0), P.ny - 1);
    iz = min(max(iz, 0), P.nz - 1);
    const int sx = (r.ux > 0.0f) - (r.ux < 0.0f);
    const int sy = (r.uy > 0.0f) - (r.uy < 0.0f);
    const int sz = (r.uz > 0.0f) - (r.uz < 0.0f);
    const float iux = sx ? 1.0f / r.ux : 0.0f;
    const float iuy = sy ? 1.0f / r.uy : 0.0f;
    const float iuz = sz ? 1.0f / r.uz : 0.0f;
    // Next plane crossed on each axis, from its integer index.
    auto cross = [](int idx, int s, float o, float v, float m, float iu) -> float {
        return s ? (fmaf((float)(idx + (s > 0)), v, o) - m) * iu : kInf;
    };
    float tnx = cross(ix, sx, P.ox, P.vx, r.mx, iux);
    float tny = cross(iy, sy, P.oy, P.vy, r.my, iuy);
    float tnz = cross(iz, sz, P.oz, P.vz, r.mz, iuz);
    const int sxy = P.nx, sxyz = P.nx * P.ny;
    int j = ix + sxy * iy + sxyz * iz;
    const bool tof = P.tof;
    float t = r.t0;
    float e_prev = tof ? erff(t * P.inv_sig_sqrt2) : 0.0f;
    const int max_steps = P.nx + P.ny + P.nz + 2;
    for (int step = 0; step < max_steps; ++step) {
        float tn = fminf(fminf(tnx, tny), fminf(tnz, r.t1));
        tn = fmaxf(tn, t);
        float a;
        if (tof) {
            float e = erff(tn * P.inv_sig_sqrt2);
            a = (e - e_prev) * P.norm;
            e_prev = e;
        } else {
            a = tn - t;
        }
        visit(j, a);
        if (tn >= r.t1) break;
        if (tnx <= tny && tnx <= tnz) {
            ix += sx;
            if ((unsigned)ix >= (unsigned)P.nx) break;
            j += sx;
            tnx = cross(ix, sx, P.ox, P.vx, r.mx, iux);
        } else if (tny <= tnz) {
            iy += sy;
            if ((unsigned)iy >= (unsigned)P.ny) break;
            j += sy * sxy;
            tny = cross(iy, sy, P.oy, P.vy, r.my, iuy);
        } else {
            iz += sz;
            if ((unsigned)iz >= (unsigned)P.nz) break;
            j += sz * sxyz;
            tnz = cross(iz, sz, P.oz, P.vz, r.mz, iuz);
        }
        t = tn;
    }
}

// Which problem owns chunk c (block-uniform; problems are few and ordered).
__device__ __forceinline__ int find_problem(const Problem *probs, int n_probs, int64_t c) {
    int p = n_probs - 1;
    while (p > 0 && probs[p].chunk_begin > c) --p;
    return p;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fused MLEM projector: forward, ratio, back for every event of one chunk.
// Per-chunk partials: number of events with f > 0 and sum of log f.
__global__ void __launch_bounds__(1024) k_project_fused(const Problem *__restrict__ probs, int n_probs, int ept,
                                                        int *__restrict__ part_neff,
                                                        double *__restrict__ part_ll) {
    const int64_t c = blockIdx.x;
    const int p = find_problem(probs, n_probs, c);
    const Problem &P = probs[p];
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    const float *__restrict__ x = P.x;
    float *__restrict__ b = P.b;
    int neff = 0;
    float ll = 0.0f;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        if (!make_ray(P, i, r)) continue;
        float f = 0.0f;
        traverse(P, r, [&](int j, float a) { f = fmaf(a, x[j], f); });
        if (!(f > 0.0f)) continue;
        ++neff;
        ll += logf(f);
        const float rf = 1.0f / f;
        traverse(P, r, [&](int j, float a) {
            if (a != 0.0f) unsafeAtomicAdd(b + j, a * rf);
        });
    }
    // block reduction of the partials
    __shared__ int s_n[16];
    __shared__ double s_l[16];
    int wn = wave_sum(neff);
    double wl = wave_sum((double)ll);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { s_n[wid] = wn; s_l[wid] = wl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tn = 0;
        double tl = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { tn += s_n[w]; tl += s_l[w]; }
        part_neff[c] = tn;
        part_ll[c] = tl;
    }
}

// Forward projection only: f_out[stored index] = (A x)_i.
__global__ void __launch_bounds__(1024) k_project_forward(const Problem *__restrict__ probs, int n_probs, int ept,
                                                          float *__restrict__ f_out) {
    const int64_t c = blockIdx.x;
    const int p = find_problem(probs, n_probs, c);
    const Problem &P = probs[p];
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        float f = 0.0f;
        if (make_ray(P, i, r)) traverse(P, r, [&](int j, float a) { f = fmaf(a, P.x[j], f); });
        f_out[P.ev_offset + i] = f;
    }
}

// Back projection only: b_j += sum_i a_ij w[stored index].
__global__ void __launch_bounds__(1024) k_project_back(const Problem *__restrict__ probs, int n_probs, int ept,
                                                       const float *__restrict__ w_in) {
    const int64_t c = blockIdx.x;
    const int p = find_problem(probs, n_probs, c);
    const Problem &P = probs[p];
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        const float w = w_in[P.ev_offset + i];
        if (w == 0.0f) continue;
        Ray r;
        if (!make_ray(P, i, r)) continue;
        traverse(P, r, [&](int j, float a) {
            if (a != 0.0f) unsafeAtomicAdd(P.b + j, a * w);
        });
    }
}

// Diagnostic: number of voxel pieces each chunk's rays visit (one gather in
// the forward pass and at most one atomic in the back pass per piece).
__global__ void __launch_bounds__(1024) k_count_pieces(const Problem *__restrict__ probs, int n_probs, int ept,
                                                       unsigned long long *__restrict__ part) {
    const int64_t c = blockIdx.x;
    const int p = find_problem(probs, n_probs, c);
    const Problem &P = probs[p];
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    unsigned long long cnt = 0, nz = 0;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        if (!make_ray(P, i, r)) continue;
        traverse(P, r, [&](int, float a) {
            ++cnt;
            nz += (a != 0.0f);
        });
    }
    __shared__ unsigned long long s_c[16], s_z[16];
    unsigned long long wc = wave_sum(cnt), wz = wave_sum(nz);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { s_c[wid] = wc; s_z[wid] = wz; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += s_c[w]; b += s_z[w]; }
        part[2 * c] = a;
        part[2 * c + 1] = b;
    }
}

}  // namespace

hipError_t launch_count_pieces(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int block,
                               int ept, unsigned long long *part) {
    void *args[] = {&d_probs, &n_probs, &ept, &part};
    return do_launch(L, reinterpret_cast<const void *>(&k_count_pieces), dim3((unsigned)n_chunks), dim3(block), 0,
                     args);
}

int64_t project_chunk_events(int block, int ept) { return (int64_t)block * ept; }

hipError_t launch_project_fused(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int block,
                                int ept, int *part_neff, double *part_ll) {
    void *args[] = {&d_probs, &n_probs, &ept, &part_neff, &part_ll};
    return do_launch(L, reinterpret_cast<const void *>(&k_project_fused), dim3((unsigned)n_chunks), dim3(block), 0,
                     args);
}

hipError_t launch_project_forward(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int block,
                                  int ept, float *f_out) {
    void *args[] = {&d_probs, &n_probs, &ept, &f_out};
    return do_launch(L, reinterpret_cast<const void *>(&k_project_forward), dim3((unsigned)n_chunks), dim3(block),
                     0, args);
}

hipError_t launch_project_back(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int block,
                               int ept, const float *w_in) {
    void *args[] = {&d_probs, &n_probs, &ept, &w_in};
    return do_launch(L, reinterpret_cast<const void *>(&k_project_back), dim3((unsigned)n_chunks), dim3(block), 0,
                     args);
}

}  // namespace lmtof

// MLEM image update and the FP64 bookkeeping sums (gfx950).
//
// Update (arXiv 1706.07075, Section 2.4, list-mode MLEM after Shepp & Vardi):
// x_j <- x_j * b_j / s_j with b the back-projected ratios of the iteration
// and s the sensitivity; voxels with s_j = 0 are held at 0.  The same pass
// clears b for the next iteration and forms, in FP64, sum_j s_j x_j before
// and after the update (their difference to the event count is the EM
// normalisation check).  All reductions write per-block partials that one
// small kernel sums in a fixed order: deterministic, no FP64 atomics.
#include "lmtof_internal.h"

namespace lmtof {
namespace {

constexpr int kUpdBlock = 256;
constexpr int kUpdPerThread = 16;
constexpr int64_t kUpdChunk = (int64_t)kUpdBlock * kUpdPerThread;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
template <class T>
__device__ __forceinline__ T block_sum(T v, T *smem) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    T t = T(0);
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) t += smem[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ int find_vproblem(const Problem *probs, int n_probs, int64_t c) {
    int p = n_probs - 1;
    while (p > 0 && probs[p].vchunk_begin > c) --p;
    return p;
}

__global__ void __launch_bounds__(kUpdBlock) k_update(const Problem *__restrict__ probs, int n_probs,
                                                      double *__restrict__ part_old, double *__restrict__ part_new) {
    __shared__ double sm[kUpdBlock / 64];
    const int64_t c = blockIdx.x;
    const Problem &P = probs[find_vproblem(probs, n_probs, c)];
    const int64_t V = (int64_t)P.nx * P.ny * P.nz;
    const int64_t base = (c - P.vchunk_begin) * kUpdChunk;
    float *__restrict__ x = P.x;
    float *__restrict__ b = P.b;
    const float *__restrict__ s = P.s;
    double so = 0.0, sn = 0.0;
#pragma unroll 4
    for (int k = 0; k < kUpdPerThread; ++k) {
        const int64_t j = base + (int64_t)k * kUpdBlock + threadIdx.x;
        if (j >= V) break;
        const float xo = x[j], bj = b[j], sj = s[j];
        const float xn = sj > 0.0f ? xo * bj / sj : 0.0f;
        x[j] = xn;
        b[j] = 0.0f;
        so += (double)sj * (double)xo;
        sn += (double)sj * (double)xn;
    }
    so = block_sum(so, sm);
    sn = block_sum(sn, sm);
    if (threadIdx.x == 0) {
        part_old[c] = so;
        part_new[c] = sn;
    }
}

constexpr int kFinBlock = 1024;
constexpr int kFinLoads = 16;  // partials per thread in flight

__global__ void __launch_bounds__(kFinBlock) k_finalize(const Problem *__restrict__ probs, int n_probs,
                                                  int64_t n_chunks, int64_t n_vchunks,
                                                  const int *__restrict__ part_neff,
                                                  const double *__restrict__ part_ll,
                                                  const double *__restrict__ part_old,
                                                  const double *__restrict__ part_new, DevStats *__restrict__ stats,
                                                  int iter) {
    __shared__ double smd[kFinBlock / 64];
    __shared__ int64_t smi[kFinBlock / 64];
    const int p = blockIdx.x;
    const Problem &P = probs[p];
    const int64_t c0 = P.chunk_begin, c1 = (p + 1 < n_probs) ? probs[p + 1].chunk_begin : n_chunks;
    const int64_t v0 = P.vchunk_begin, v1 = (p + 1 < n_probs) ? probs[p + 1].vchunk_begin : n_vchunks;
    int64_t ne = 0;
    double ll = 0.0, so = 0.0, sn = 0.0;
    // each thread adds its partials in index order; kFinLoads of them are
    // loaded before they are added, so the loads overlap
    const int64_t step = (int64_t)blockDim.x;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += kFinLoads * step) {
        int nv[kFinLoads];
        double lv[kFinLoads];
#pragma unroll
        for (int u = 0; u < kFinLoads; ++u) {
            const int64_t k = c + u * step;
            nv[u] = k < c1 ? part_neff[k] : 0;
            lv[u] = k < c1 ? part_ll[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinLoads; ++u) {
            ne += nv[u];
            ll += lv[u];
        }
    }
    for (int64_t c = v0 + threadIdx.x; c < v1; c += kFinLoads * step) {
        double ov[kFinLoads], nw[kFinLoads];
#pragma unroll
        for (int u = 0; u < kFinLoads; ++u) {
            const int64_t k = c + u * step;
            ov[u] = k < v1 ? part_old[k] : 0.0;
            nw[u] = k < v1 ? part_new[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinLoads; ++u) {
            so += ov[u];
            sn += nw[u];
        }
    }
    ne = block_sum(ne, smi);
    ll = block_sum(ll, smd);
    so = block_sum(so, smd);
    sn = block_sum(sn, smd);
    if (threadIdx.x == 0) {
        DevStats &d = stats[(int64_t)iter * n_probs + p];
        d.n_eff = ne;
        d.sum_logf = ll;
        d.sum_sx_old = so;
        d.sum_sx = sn;
    }
}

__global__ void __launch_bounds__(256) k_sum_positive(const float *__restrict__ s, int64_t n,
                                                      double *__restrict__ partials) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const float v = s[j];
        if (v > 0.0f) acc += (double)v;
    }
    acc = block_sum(acc, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256) k_sum_partials(const double *__restrict__ partials, int n,
                                                      double *__restrict__ out) {
    __shared__ double sm[4];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) acc += partials[k];
    acc = block_sum(acc, sm);
    if (threadIdx.x == 0) *out = acc;
}

__global__ void k_uniform_image(const float *__restrict__ s, int64_t n, const double *__restrict__ sum,
                                double n_events, float *__restrict__ x) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double tot = *sum;
    x[j] = (s[j] > 0.0f && tot > 0.0) ? (float)(n_events / tot) : 0.0f;
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float v) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}

// a <- a * w (per-event ratio weights)
__global__ void k_mul(float *__restrict__ a, const float *__restrict__ w, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        a[j] *= w[j];
}

// a <- exp(a) (attenuation factors from line integrals)
__global__ void k_exp(float *__restrict__ a, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        a[j] = expf(a[j]);
}

__global__ void k_copy(const float *__restrict__ src, int64_t n, float *__restrict__ dst) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

__global__ void k_add(const float *__restrict__ src, int64_t n, float *__restrict__ dst) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        dst[j] += src[j];
}

unsigned grid_for(int64_t n, int block, unsigned cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int64_t update_chunk_voxels() { return kUpdChunk; }

hipError_t launch_update(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_vchunks, double *part_old,
                         double *part_new) {
    void *args[] = {&d_probs, &n_probs, &part_old, &part_new};
    return do_launch(L, reinterpret_cast<const void *>(&k_update), dim3((unsigned)n_vchunks), dim3(kUpdBlock), 0,
                     args);
}

hipError_t launch_finalize(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks,
                           int64_t n_vchunks, const int *part_neff, const double *part_ll, const double *part_old,
                           const double *part_new, DevStats *stats, int iter) {
    void *args[] = {&d_probs, &n_probs, &n_chunks, &n_vchunks, &part_neff, &part_ll,
                    &part_old, &part_new, &stats, &iter};
    return do_launch(L, reinterpret_cast<const void *>(&k_finalize), dim3((unsigned)n_probs), dim3(kFinBlock), 0,
                     args);
}

hipError_t launch_sum_positive(const Launch &L, const float *s, int64_t n, double *partials, int n_part,
                               double *out) {
    void *a1[] = {&s, &n, &partials};
    hipError_t e = do_launch(L, reinterpret_cast<const void *>(&k_sum_positive), dim3((unsigned)n_part), dim3(256),
                             0, a1);
    if (e != hipSuccess) return e;
    void *a2[] = {&partials, &n_part, &out};
    return do_launch(L, reinterpret_cast<const void *>(&k_sum_partials), dim3(1), dim3(256), 0, a2);
}

hipError_t launch_uniform_image(const Launch &L, const float *s, int64_t n, const double *sum, double n_events,
                                float *x) {
    void *args[] = {&s, &n, &sum, &n_events, &x};
    return do_launch(L, reinterpret_cast<const void *>(&k_uniform_image), dim3(grid_for(n, 256, 1u << 30)),
                     dim3(256), 0, args);
}

hipError_t launch_fill(const Launch &L, float *p, int64_t n, float v) {
    void *args[] = {&p, &n, &v};
    return do_launch(L, reinterpret_cast<const void *>(&k_fill), dim3(grid_for(n, 256)), dim3(256), 0, args);
}

hipError_t launch_mul(const Launch &L, float *a, const float *w, int64_t n) {
    void *args[] = {&a, &w, &n};
    return do_launch(L, reinterpret_cast<const void *>(&k_mul), dim3(grid_for(n, 256)), dim3(256), 0, args);
}

hipError_t launch_exp(const Launch &L, float *a, int64_t n) {
    void *args[] = {&a, &n};
    return do_launch(L, reinterpret_cast<const void *>(&k_exp), dim3(grid_for(n, 256)), dim3(256), 0, args);
}

hipError_t launch_copy_slab(const Launch &L, const float *src, int64_t plane, int z_lo, int nzs, float *dst) {
    const float *from = src + plane * z_lo;
    int64_t n = plane * nzs;
    void *args[] = {&from, &n, &dst};
    return do_launch(L, reinterpret_cast<const void *>(&k_copy), dim3(grid_for(n, 256)), dim3(256), 0, args);
}

hipError_t launch_add_slab(const Launch &L, const float *src, int64_t plane, int z_lo, int nzs, float *dst) {
    float *to = dst + plane * z_lo;
    int64_t n = plane * nzs;
    void *args[] = {&src, &n, &to};
    return do_launch(L, reinterpret_cast<const void *>(&k_add), dim3(grid_for(n, 256)), dim3(256), 0, args);
}

}  // namespace lmtof

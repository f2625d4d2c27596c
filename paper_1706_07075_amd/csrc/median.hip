// Median sieve between MLEM iterations (gfx950).
//
// arXiv 1706.07075, Section 2.4: a median filter is applied to the image
// estimate after each iteration to suppress high-frequency noise (a sieve).
// The paper gives neither the neighbourhood nor the border rule; here it is
// the 3 x 3 x 3 block around each voxel, voxels outside the grid counting as
// 0 (the paper remarks that null neighbours pull border voxels down).  The
// median of 27 values is their 14th smallest, an element of the input, so
// the result is exact.
//
// One lane per voxel.  The 27 values sit in registers and the median comes
// from forgetful selection: a pool of the first 15 values (half the count
// plus two) repeatedly loses its smallest and its largest, which cannot be
// the median of all 27, and takes in the next value, until all 27 have
// entered and three remain, whose middle one is the median.  195
// compare-exchanges (a min and a max each), no branches.
#include "lmtof_internal.h"

namespace lmtof {
namespace {

// Put the smallest of v[LO, LO + P) at v[LO] and the largest at v[LO + P - 1].
template <int LO, int P>
__device__ __forceinline__ void extremes(float (&v)[27]) {
#pragma unroll
    for (int k = LO + 1; k < LO + P; ++k) {
        const float a = v[LO], b = v[k];
        v[LO] = fminf(a, b);
        v[k] = fmaxf(a, b);
    }
#pragma unroll
    for (int k = LO + 1; k < LO + P - 1; ++k) {
        const float a = v[k], b = v[LO + P - 1];
        v[k] = fminf(a, b);
        v[LO + P - 1] = fmaxf(a, b);
    }
}

// Step R: the pool is v[R, 15); drop its extremes, then the largest's slot
// v[14] takes the next value v[15 + R].  After step 11 the pool is v[12, 15).
template <int R>
struct Forget {
    static __device__ __forceinline__ void run(float (&v)[27]) {
        extremes<R, 15 - R>(v);
        v[14] = v[15 + R];
        Forget<R + 1>::run(v);
    }
};
template <>
struct Forget<12> {
    static __device__ __forceinline__ void run(float (&v)[27]) { extremes<12, 3>(v); }
};

__global__ void __launch_bounds__(256) k_median3(const float *__restrict__ x, float *__restrict__ y, int nx, int ny,
                                                 int nz) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
    float v[27];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                const bool in = jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz;
                // out-of-grid neighbours read the centre voxel (in bounds) and count as 0
                const int64_t j = in ? (int64_t)jx + (int64_t)nx * (jy + (int64_t)ny * jz) : i;
                const float xv = x[j];
                v[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = in ? xv : 0.0f;
            }
    Forget<0>::run(v);
    y[i] = v[13];
}

// x <- t, t <- 0 (t is the back projection buffer, used as the filter's
// output and left cleared for the next iteration).
__global__ void __launch_bounds__(256) k_take_clear(float *__restrict__ x, float *__restrict__ t, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] = t[i];
    t[i] = 0.0f;
}

}  // namespace

hipError_t launch_median3(const Launch &L, const float *x, float *y, int nx, int ny, int nz) {
    const int64_t n = (int64_t)nx * ny * nz;
    void *args[] = {&x, &y, &nx, &ny, &nz};
    return do_launch(L, reinterpret_cast<const void *>(&k_median3), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     args);
}

hipError_t launch_take_clear(const Launch &L, float *x, float *t, int64_t n) {
    void *args[] = {&x, &t, &n};
    return do_launch(L, reinterpret_cast<const void *>(&k_take_clear), dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, args);
}

}  // namespace lmtof

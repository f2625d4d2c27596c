// The paper's own TOF projector (arXiv 1706.07075, Section 2.3), kept for
// comparison with the exact-integral projector of project.hip (gfx950).
//
// Each event is sampled at kSamples points spaced equally along its LOR over
// the kernel window [-K sigma, K sigma] around the TOF centre (midpoints of
// equal steps); a point's weight is the Gaussian density there, the weights
// normalised to sum to 1 (a table computed on the host, passed by value);
// each point reads or adds into the voxel that holds it ("direct voxel
// filling"); points outside the grid are dropped.  One lane per event.  The
// forward pass gathers; the back pass adds with device-scope FP32 atomics
// (the paper's scheme), so its sums are not bit-reproducible.
#include "lmtof_internal.h"

#include <hip/hip_fp16.h>

namespace lmtof {
namespace {

// Stored event i: endpoints and dt (plain 2 x float4, or packed int16
// endpoints at 0.1 mm and a binary16 dt).
template <bool PACKED>
__device__ __forceinline__ void stored_event(const void *events, int64_t i, float p[7]) {
    if (!PACKED) {
        const float4 *e = reinterpret_cast<const float4 *>(events) + 2 * i;
        const float4 a = e[0], b = e[1];
        p[0] = a.x; p[1] = a.y; p[2] = a.z; p[3] = a.w;
        p[4] = b.x; p[5] = b.y; p[6] = b.z;
    } else {
        const uint4 w = reinterpret_cast<const uint4 *>(events)[i];
        const uint32_t q[3] = {w.x, w.y, w.z};
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k] = (float)(int16_t)((q[k >> 1] >> (16 * (k & 1))) & 0xffffu) * 0.1f;
        __half_raw hr;
        hr.x = (unsigned short)(w.w & 0xffffu);
        p[6] = __half2float(__half(hr));
    }
}

template <bool PACKED, bool BACK>
__global__ void __launch_bounds__(256) k_sampled(const void *__restrict__ events, int64_t n, SampledGeom G,
                                                 const float *__restrict__ x, float *__restrict__ f,
                                                 const float *__restrict__ r, float *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float p[7];
    stored_event<PACKED>(events, i, p);
    const float dx = p[3] - p[0], dy = p[4] - p[1], dz = p[5] - p[2];
    const float il = rsqrtf(dx * dx + dy * dy + dz * dz);
    const float ux = dx * il, uy = dy * il, uz = dz * il;
    const float sh = G.half_c * p[6];
    const float cx = fmaf(sh, ux, 0.5f * (p[0] + p[3]));
    const float cy = fmaf(sh, uy, 0.5f * (p[1] + p[4]));
    const float cz = fmaf(sh, uz, 0.5f * (p[2] + p[5]));
    const float ri = BACK ? r[i] : 0.0f;
    float acc = 0.0f;
#pragma unroll 4
    for (int k = 0; k < kSampledN; ++k) {
        const float t = fmaf((float)k + 0.5f, G.step, G.t_lo);
        const int ix = (int)floorf((fmaf(t, ux, cx) - G.ox) * G.ivx);
        const int iy = (int)floorf((fmaf(t, uy, cy) - G.oy) * G.ivy);
        const int iz = (int)floorf((fmaf(t, uz, cz) - G.oz) * G.ivz);
        if (ix < 0 || ix >= G.nx || iy < 0 || iy >= G.ny || iz < 0 || iz >= G.nz) continue;
        const int64_t j = ix + (int64_t)G.nx * (iy + (int64_t)G.ny * iz);
        if (BACK)
            atomicAdd(b + j, G.w[k] * ri);
        else
            acc = fmaf(G.w[k], x[j], acc);
    }
    if (!BACK) f[i] = acc;
}

}  // namespace

hipError_t launch_sampled(const Launch &L, const void *events, bool packed, int64_t n, const SampledGeom &G,
                          const float *x, float *f, const float *r, float *b) {
    SampledGeom g = G;
    void *args[] = {&events, &n, &g, &x, &f, &r, &b};
    const bool back = r != nullptr;
    const void *fn = packed ? (back ? reinterpret_cast<const void *>(&k_sampled<true, true>)
                                    : reinterpret_cast<const void *>(&k_sampled<true, false>))
                            : (back ? reinterpret_cast<const void *>(&k_sampled<false, true>)
                                    : reinterpret_cast<const void *>(&k_sampled<false, false>));
    return do_launch(L, fn, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, args);
}

}  // namespace lmtof

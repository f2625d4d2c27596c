// Geometric sensitivity of a single-bed cylindrical scanner (gfx950).
//
// The "sensitive matrix" of the MLEM update (arXiv 1706.07075, Section 2.4)
// is read as the detection probability of an emission at each voxel centre:
// an isotropic back-to-back pair at p is detected when both ends meet the
// barrel (radius R, |z| <= H) and the LOR elevation is within the axial
// acceptance cut (45 degrees in Section 2.1.2).  For azimuth phi the
// transverse line meets the circle at signed distances s+ > 0 > s-, and the
// pair is detected iff tan(lambda) lies in
//   [max(-(H+z)/s+, -(H-z)/|s-|), min((H-z)/s+, (H+z)/|s-|)],
// so with g(tau) = sin(atan tau) = tau / sqrt(1 + tau^2)
//   P(p) = (1 / 4 pi) int_0^{2 pi} [g(tau_hi) - g(tau_lo)]_+ dphi,
// evaluated by the midpoint rule on n_phi nodes.
//
// GPU design: s+- depend on the transaxial position and phi only, so each
// thread owns one (x, y) column and a run of z voxels and reuses the two
// roots for all of them.  The integrand is FP32 (stable root formulas, no
// cancellation); each voxel's quadrature sum is accumulated in FP64.
#include "lmtof_internal.h"

namespace lmtof {
namespace {

constexpr int kSensBlock = 256;
constexpr int kSensZ = 16;      // z voxels per thread
constexpr int kMaxPhi = 4096;   // LDS table capacity (32 KB)

__global__ void __launch_bounds__(kSensBlock) k_sensitivity(SensGeom g, float *__restrict__ s) {
    __shared__ float2 cs[kMaxPhi];
    for (int k = threadIdx.x; k < g.n_phi; k += blockDim.x) {
        float sn, cn;
        sincospif((2.0f * (float)k + 1.0f) / (float)g.n_phi, &sn, &cn);
        cs[k] = make_float2(cn, sn);
    }
    __syncthreads();
    const int zblocks = (g.nz + kSensZ - 1) / kSensZ;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncol = (int64_t)g.nx * g.ny;
    if (tid >= ncol * zblocks) return;
    const int64_t col = tid % ncol;
    const int zb = (int)(tid / ncol);
    const int ix = (int)(col % g.nx), iy = (int)(col / g.nx);
    const float px = (float)(g.ox + (ix + 0.5) * g.vx);
    const float py = (float)(g.oy + (iy + 0.5) * g.vy);
    const float R = (float)g.R, H = (float)g.H;
    const float r = sqrtf(px * px + py * py);
    const float c = (R - r) * (R + r);  // R^2 - |p|^2 > 0 inside the barrel
    const int z0 = zb * kSensZ;
    const int nzl = min(kSensZ, g.nz - z0);
    float hm[kSensZ], hp[kSensZ];       // H - z, H + z
    double acc[kSensZ];
#pragma unroll
    for (int q = 0; q < kSensZ; ++q) {
        const float z = (float)(g.oz + (z0 + q + 0.5) * g.vz);
        hm[q] = H - z;
        hp[q] = H + z;
        acc[q] = 0.0;
    }
    const float tmax = g.tan_lmax > 0.0 ? (float)g.tan_lmax : __builtin_huge_valf();
    if (c > 0.0f) {
        for (int k = 0; k < g.n_phi; ++k) {
            const float2 t = cs[k];
            const float bb = px * t.x + py * t.y;
            const float sq = sqrtf(fmaf(bb, bb, c));
            float sp, sm;  // s+ and |s-|, each from its cancellation-free form
            if (bb >= 0.0f) {
                sm = bb + sq;
                sp = c / sm;
            } else {
                sp = sq - bb;
                sm = c / sp;
            }
            const float isp = 1.0f / sp, ism = 1.0f / sm;
#pragma unroll
            for (int q = 0; q < kSensZ; ++q) {
                float th = fminf(hm[q] * isp, hp[q] * ism);
                float tl = fmaxf(-hp[q] * isp, -hm[q] * ism);
                th = fminf(th, tmax);
                tl = fmaxf(tl, -tmax);
                const float gh = th * rsqrtf(fmaf(th, th, 1.0f));
                const float gl = tl * rsqrtf(fmaf(tl, tl, 1.0f));
                const float d = gh - gl;
                acc[q] += (double)fmaxf(d, 0.0f);
            }
        }
    }
    const double scale = (2.0 * 3.14159265358979323846 / g.n_phi) / (4.0 * 3.14159265358979323846);
    for (int q = 0; q < nzl; ++q) {
        const int64_t j = col + ncol * (int64_t)(z0 + q);
        s[j] = (c > 0.0f) ? (float)(acc[q] * scale) : 0.0f;
    }
}

}  // namespace

hipError_t launch_sensitivity(const Launch &L, const SensGeom &g, float *s) {
    if (g.n_phi < 1 || g.n_phi > kMaxPhi) return hipErrorInvalidValue;
    const int64_t ncol = (int64_t)g.nx * g.ny;
    const int64_t nthreads = ncol * ((g.nz + kSensZ - 1) / kSensZ);
    const unsigned grid = (unsigned)((nthreads + kSensBlock - 1) / kSensBlock);
    SensGeom gg = g;
    void *args[] = {&gg, &s};
    return do_launch(L, reinterpret_cast<const void *>(&k_sensitivity), dim3(grid), dim3(kSensBlock), 0, args);
}

}  // namespace lmtof

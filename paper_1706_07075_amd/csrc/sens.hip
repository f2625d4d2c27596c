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
// The acceptance is invariant under x -> -x, y -> -y, x <-> y (rotations
// and reflections of the barrel) and z -> -z, and so is the midpoint rule
// on n_phi nodes (n_phi a multiple of 4 for the swap).  When the voxel
// lattice is symmetric too, only one representative per orbit is
// integrated (1/16 of the voxels for a centred square grid) and its value
// written to every image.
#include "lmtof_internal.h"

#include <cmath>

namespace lmtof {
namespace {

constexpr int kSensBlock = 256;
constexpr int kSensZ = 16;      // z voxels per thread
constexpr int kMaxPhi = 4096;   // LDS table capacity (32 KB)

// Representative columns: x offsets [hx, nx) when mirrored in x (hx =
// nx / 2; an odd centre column maps to itself), else [0, nx); likewise y;
// with the x <-> y swap only dy <= dx of the (square) quadrant.
struct SensDomain {
    int hx, hy, hz, mx, my, mz;  // first representative index and count per axis
    int64_t ncol;                // representative columns
};

__host__ __device__ __forceinline__ SensDomain sens_domain(const SensGeom &g) {
    SensDomain d;
    d.hx = g.sym_x ? g.nx / 2 : 0;
    d.hy = g.sym_y ? g.ny / 2 : 0;
    d.hz = g.sym_z ? g.nz / 2 : 0;
    d.mx = g.nx - d.hx;
    d.my = g.ny - d.hy;
    d.mz = g.nz - d.hz;
    d.ncol = g.sym_xy ? (int64_t)d.mx * (d.mx + 1) / 2 : (int64_t)d.mx * d.my;
    return d;
}

__global__ void __launch_bounds__(kSensBlock) k_sensitivity(SensGeom g, float *__restrict__ s) {
    __shared__ float2 cs[kMaxPhi];
    for (int k = threadIdx.x; k < g.n_phi; k += blockDim.x) {
        float sn, cn;
        sincospif((2.0f * (float)k + 1.0f) / (float)g.n_phi, &sn, &cn);
        cs[k] = make_float2(cn, sn);
    }
    __syncthreads();
    const SensDomain D = sens_domain(g);
    const int zblocks = (D.mz + kSensZ - 1) / kSensZ;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= D.ncol * zblocks) return;
    const int64_t col = tid % D.ncol;
    const int zb = (int)(tid / D.ncol);
    int dx, dy;
    if (g.sym_xy) {  // col = dx (dx + 1) / 2 + dy, 0 <= dy <= dx
        dx = (int)((sqrtf(8.0f * (float)col + 1.0f) - 1.0f) * 0.5f);
        while ((int64_t)dx * (dx + 1) / 2 > col) --dx;
        while ((int64_t)(dx + 1) * (dx + 2) / 2 <= col) ++dx;
        dy = (int)(col - (int64_t)dx * (dx + 1) / 2);
    } else {
        dx = (int)(col % D.mx);
        dy = (int)(col / D.mx);
    }
    const int ix = D.hx + dx, iy = D.hy + dy;
    const float px = (float)(g.ox + (ix + 0.5) * g.vx);
    const float py = (float)(g.oy + (iy + 0.5) * g.vy);
    const float R = (float)g.R, H = (float)g.H;
    const float r = sqrtf(px * px + py * py);
    const float c = (R - r) * (R + r);  // R^2 - |p|^2 > 0 inside the barrel
    const int z0 = D.hz + zb * kSensZ;
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
    // images of (ix, iy) under the x/y mirrors and the swap
    int cx[8], cy[8];
    int nc = 0;
    for (int sw = 0; sw < (g.sym_xy ? 2 : 1); ++sw) {
        const int ax = sw ? iy : ix, ay = sw ? ix : iy;
        for (int fx = 0; fx < (g.sym_x ? 2 : 1); ++fx)
            for (int fy = 0; fy < (g.sym_y ? 2 : 1); ++fy) {
                cx[nc] = fx ? g.nx - 1 - ax : ax;
                cy[nc] = fy ? g.ny - 1 - ay : ay;
                ++nc;
            }
    }
    const int64_t plane = (int64_t)g.nx * g.ny;
    for (int q = 0; q < nzl; ++q) {
        const float v = (c > 0.0f) ? (float)(acc[q] * scale) : 0.0f;
        const int iz = z0 + q;
        for (int fz = 0; fz < (g.sym_z ? 2 : 1); ++fz) {
            const int64_t zo = plane * (fz ? g.nz - 1 - iz : iz);
            for (int m = 0; m < nc; ++m) s[zo + cx[m] + (int64_t)g.nx * cy[m]] = v;
        }
    }
}

}  // namespace

hipError_t launch_sensitivity(const Launch &L, const SensGeom &g, float *s) {
    if (g.n_phi < 1 || g.n_phi > kMaxPhi) return hipErrorInvalidValue;
    SensGeom gg = g;
    // a lattice axis is mirror-symmetric when the grid is centred on it (to
    // a millionth of a voxel; the FP32 centre coordinates then agree to
    // rounding); the azimuth nodes are symmetric for even n_phi, and under
    // the swap for n_phi divisible by 4
    auto centred = [](double o, int n, double v) { return std::fabs(o + 0.5 * n * v) <= 1e-6 * v; };
    const bool even = g.n_phi % 2 == 0;
    gg.sym_x = even && centred(g.ox, g.nx, g.vx);
    gg.sym_y = even && centred(g.oy, g.ny, g.vy);
    gg.sym_z = centred(g.oz, g.nz, g.vz);
    gg.sym_xy = gg.sym_x && gg.sym_y && g.n_phi % 4 == 0 && g.nx == g.ny && g.vx == g.vy;
    const SensDomain D = sens_domain(gg);
    const int64_t nthreads = D.ncol * ((D.mz + kSensZ - 1) / kSensZ);
    const unsigned grid = (unsigned)((nthreads + kSensBlock - 1) / kSensBlock);
    void *args[] = {&gg, &s};
    return do_launch(L, reinterpret_cast<const void *>(&k_sensitivity), dim3(grid), dim3(kSensBlock), 0, args);
}

}  // namespace lmtof

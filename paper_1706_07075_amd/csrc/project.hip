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
//    look-up table too): 1025 nodes over [-K, K] sigma, each holding the
//    value and the first- and second-order Taylor coefficients, so one LDS
//    read and two FMAs give Phi to ~2e-9, with no divergent branch (the back
//    projection keeps 8-byte nodes and derives the second-order term).
//  * Both projections are brick-parallel.  At load every event's window is
//    cut into pieces per 16^3-voxel brick (items), and each brick's list
//    into chunks of bounded length.  One workgroup takes one chunk.
//  * Forward: the workgroup stages its brick of x in LDS, so every image
//    gather of its items is an LDS read, and writes each item's partial sum
//    of a x; a combine pass adds an event's partials (in the order its
//    window crosses the bricks), forms r_i = 1 / f_i and writes r_i back to
//    the event's items, where the back projection reads it coalesced.  (An
//    event-parallel forward pass, one lane per event gathering from a
//    blocked copy of x in global memory, is kept for the testing surface
//    and as a launch option: it is bound by the texture units' per-line
//    work, ~50 distinct cache lines per wavefront gather.)
//  * Back: the workgroup accumulates a_ij r_i with LDS atomics and writes
//    its tile with plain stores; a small kernel adds a brick's chunk tiles
//    into b.  There is no
//    global atomic on the image (device-scope FP32 atomics sustain only
//    ~21 G/s on this part, a third of a random gather's rate).  Chunks are
//    launched largest first so the uneven work balances across CUs, and a
//    brick's items are grouped by their step count so a wavefront's lanes
//    finish together.
#include "lmtof_internal.h"

#include <hip/hip_fp16.h>

namespace lmtof {
namespace {

constexpr float kInf = __builtin_huge_valf();
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Device-memory views: pointers read from the problem table are generic;
// casting them to the global address space lets loads and stores use the
// global (not flat) instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> global(T *p) {
    return (gptr<T>)p;
}

// A ray r(t) = mu + t u, with mu held relative to an anchor voxel plane:
// mu_a = o_a + j_a v_a + d_a, |d_a| <~ v_a.  Plane k on axis a is crossed at
//   T_a(k) = (k - j_a) A_a + B_a,  A_a = v_a / u_a,  B_a = -d_a / u_a
// (one FMA on an exactly represented small integer), which FP32 resolves to
// ~1e-6 mm of the TOF window whatever the absolute position (1.2 m from the
// centre an absolute FP32 coordinate carries ~6e-5 mm of rounding).  Every
// kernel gets every crossing from this one formula, so a piece boundary on
// a brick face is bitwise the same on both sides of it.  An axis with
// u_a = 0 is never crossed: A_a = 0, B_a = +inf.
struct Ray {
    int jx, jy, jz;    // anchor plane indices
    float dx, dy, dz;  // mu - anchor plane (mm)
    float ux, uy, uz;  // unit direction P1 -> P2
    float ax, ay, az;  // A: t per plane
    float bx, by, bz;  // B: crossing time of the anchor plane
    float t0, t1;      // window (mm from mu)
};

__device__ __forceinline__ float cross(int k, int j, float a, float b) { return fmaf((float)(k - j), a, b); }

// Decode stored event i (plain: 2 x float4; packed: int16 x 6 at 0.1 mm +
// binary16 dt).  Endpoints come as double-float pairs p = h + l: plain
// coordinates are exact FP32 (l = 0).  A packed coordinate q / 10 mm is
// not: h = fl(q * 0.1f) and l = (q - 10 h) / 10, where q - 10 h is exact
// (one FMA), so h + l is q / 10 to ~1e-8 ulp(h), and exactly q / 10
// whenever that is an FP32 number (a coordinate on a voxel plane stays on
// it; an FP32 decode alone would be off by up to 6e-5 mm 1.2 m from the
// centre).
struct EventGeom {
    float h[6], l[6];  // P1.xyz, P2.xyz
    float dt;
};

template <bool PACKED>
__device__ __forceinline__ void load_event(const void *events, int64_t i, EventGeom &ev) {
    // No contraction: h must be the rounded product that l corrects, also
    // where h later feeds an addition (a fused q * 0.1f + h' would double
    // count the residual held in l).
#pragma clang fp contract(off)
    if (!PACKED) {
        const gptr<const f32x4> e = global(reinterpret_cast<const f32x4 *>(events)) + 2 * i;
        const f32x4 a = __builtin_nontemporal_load(e), b = __builtin_nontemporal_load(e + 1);
        ev.h[0] = a[0]; ev.h[1] = a[1]; ev.h[2] = a[2]; ev.h[3] = a[3];
        ev.h[4] = b[0]; ev.h[5] = b[1]; ev.dt = b[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) ev.l[k] = 0.0f;
    } else {
        const u32x4 w = __builtin_nontemporal_load(global(reinterpret_cast<const u32x4 *>(events)) + i);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float q = (float)(int16_t)((w[k >> 1] >> (16 * (k & 1))) & 0xffffu);
            ev.h[k] = q * 0.1f;
            ev.l[k] = fmaf(-10.0f, ev.h[k], q) * 0.1f;  // (q - 10 h) exactly, over 10
        }
        __half_raw hr;
        hr.x = (unsigned short)(w[3] & 0xffffu);
        ev.dt = __half2float(__half(hr));
    }
}

// Error-free transformations (Knuth's TwoSum; TwoProd with an FMA): a + b =
// s + e and a * b = p + e exactly in FP32.  Contraction is off so that no
// operation here is fused with the product that formed an input.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e) {
#pragma clang fp contract(off)
    p = a * b;
    e = fmaf(a, b, -p);
}

// Offset from mu of plane k on an axis with anchor j, offset d, voxel size v.
__device__ __forceinline__ float plane_rel(int k, int j, float v, float d) { return fmaf((float)(k - j), v, -d); }

// Clip the line to planes [klo, khi) of one axis.
__device__ __forceinline__ void slab(int klo, int khi, int j, float v, float d, float u, float a, float b, float &t0,
                                     float &t1) {
    if (u != 0.0f) {
        const float lo = cross(klo, j, a, b), hi = cross(khi, j, a, b);
        t0 = fmaxf(t0, fminf(lo, hi));
        t1 = fminf(t1, fmaxf(lo, hi));
    } else if (!(plane_rel(klo, j, v, d) <= 0.0f && plane_rel(khi, j, v, d) > 0.0f)) {
        t0 = kInf;
        t1 = -kInf;
    }
}

// Anchor one axis: mu = (mh + ml) = o + j v + d; crossing coefficients A, B.
__device__ __forceinline__ void anchor(float mh, float ml, float o, float v, float iv, float u, int &j, float &d,
                                       float &a, float &b) {
#pragma clang fp contract(off)
    j = (int)rintf((mh - o) * iv);
    const float q = fmaf((float)j, v, o);
    d = (mh - q) + ml;
    const float iu = __builtin_amdgcn_rcpf(u);
    a = u != 0.0f ? v * iu : 0.0f;
    b = u != 0.0f ? -d * iu : kInf;
}

// Event geometry: direction, anchored TOF centre and window (clipped to the
// grid box and, with TOF, to +-K sigma).  False if the window is empty.
// The midpoint and the TOF shift along the endpoint difference are formed
// exactly (double-float); the shift is scaled along d = P2 - P1 itself, so
// rounding of the scale factor only moves mu along the line.
template <bool PACKED>
__device__ __forceinline__ bool make_ray_from(const Problem &P, const void *records, int64_t i, Ray &r) {
    // Contraction off: every kernel that inlines this must derive bitwise
    // the same ray from an event (brick lists, forward and back passes).
#pragma clang fp contract(off)
    EventGeom ev;
    load_event<PACKED>(records, i, ev);
    float dh[3], dl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        two_sum(ev.h[3 + k], -ev.h[k], dh[k], dl[k]);
        dl[k] += ev.l[3 + k] - ev.l[k];
    }
    const float iL = __builtin_amdgcn_rsqf(dh[0] * dh[0] + dh[1] * dh[1] + dh[2] * dh[2]);
    r.ux = dh[0] * iL;
    r.uy = dh[1] * iL;
    r.uz = dh[2] * iL;
    const float kappa = P.tof ? P.half_c * ev.dt * iL : 0.0f;  // mu = (P1 + P2) / 2 + kappa (P2 - P1)
    auto centre = [&](int k, float o, float v, float iv, float u, int &j, float &d, float &a, float &b) {
        float sh, se, ph, pe, mh, me;
        two_sum(ev.h[k], ev.h[3 + k], sh, se);
        se += ev.l[k] + ev.l[3 + k];
        two_prod(kappa, dh[k], ph, pe);
        two_sum(0.5f * sh, ph, mh, me);
        const float ml = me + (0.5f * se + fmaf(kappa, dl[k], pe));
        anchor(mh, ml, o, v, iv, u, j, d, a, b);
    };
    centre(0, P.ox, P.vx, P.ivx, r.ux, r.jx, r.dx, r.ax, r.bx);
    centre(1, P.oy, P.vy, P.ivy, r.uy, r.jy, r.dy, r.ay, r.by);
    centre(2, P.oz, P.vz, P.ivz, r.uz, r.jz, r.dz, r.az, r.bz);
    float t0 = -kInf, t1 = kInf;
    slab(0, P.nx, r.jx, P.vx, r.dx, r.ux, r.ax, r.bx, t0, t1);
    slab(0, P.ny, r.jy, P.vy, r.dy, r.uy, r.ay, r.by, t0, t1);
    slab(0, P.nz, r.jz, P.vz, r.dz, r.uz, r.az, r.bz, t0, t1);
    if (P.tof) {
        t0 = fmaxf(t0, -P.k_sigma);
        t1 = fminf(t1, P.k_sigma);
    }
    r.t0 = t0;
    r.t1 = t1;
    return t0 < t1;
}

// Ray of stored event i of problem P.
template <bool PACKED>
__device__ __forceinline__ bool make_ray(const Problem &P, int64_t i, Ray &r) {
    return make_ray_from<PACKED>(P, P.events, i, r);
}

// Voxel index along one axis at parameter t.
__device__ __forceinline__ int voxel_at(float t, float u, int j, float d, float iv) {
#pragma clang fp contract(off)
    return j + (int)floorf(fmaf(t, u, d) * iv);
}

// Truncated-kernel CDF from the LDS table: node k at u_k = -K + k h (sigma
// units) holds (Phi_k, Phi'_k h, Phi''_k h^2 / 2) at entry k + 1 (entries 0
// and kLutN + 1 pad the ends).  The node position of t (mm) is t a + c with
// c = (kLutN - 1) / 2, an integer; b = c + 1.5 2^23, so fma(t, a, b) rounds
// the position to the nearest node k and returns 1.5 2^23 + k exactly, whose
// bit pattern is that of 1.5 2^23 plus k: one shift-add gives the entry's
// byte offset.  |t| <= K sigma keeps k in [0, kLutN - 1].
constexpr uint32_t kLutAddrBias = 16u - (0x4B400000u << 4);  // 16 (k + 1) - (bits(1.5 2^23 + k) << 4)

// One vector-register copy of a uniform value for a loop, instead of a
// scalar-to-vector move at each use (a vector instruction reads at most one
// scalar operand here).
template <class T>
__device__ __forceinline__ T in_vgpr(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

struct Cdf {
    const float4 *tab;
    float a, b;
    __device__ __forceinline__ float operator()(float t) const {
        const float y = fmaf(t, a, b);      // 1.5 2^23 + k
        const float f = fmaf(t, a, b - y);  // position - k, in [-1/2, 1/2]
        const float4 e = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tab) +
                                                           ((__float_as_uint(y) << 4) + kLutAddrBias));
        return fmaf(f, fmaf(f, e.z, e.y), e.x);
    }
};

// Byte offset of entry j + 1 of an 8-byte-entry table from the bits of
// 1.5 2^23 + j.
constexpr uint32_t kLutAddrBias2 = 8u - (0x4B400000u << 3);  // 8 (j + 1) - (bits(1.5 2^23 + j) << 3)

// The brick projectors' CDF: the piecewise-linear table (see Problem.lin).
// fma(t, a, b) rounds the cell position to the nearest integer j and
// returns 1.5 2^23 + j (as the Cdf above); f = position - j is the offset
// from the cell's middle, and CDF = mid + f diff: one LDS read of 8 bytes
// and three FMAs (plus the address), against five more for the quadratic
// nodes.
struct CdfLin {
    const float2 *tab;
    float a, b;
    __device__ __forceinline__ float operator()(float t) const {
        const float y = fmaf(t, a, b);      // 1.5 2^23 + j
        const float f = fmaf(t, a, b - y);  // position - j, in [-1/2, 1/2]
        const float2 e = *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(tab) +
                                                           ((__float_as_uint(y) << 3) + kLutAddrBias2));
        return fmaf(f, e.y, e.x);
    }
};

__device__ __forceinline__ void stage_lin(float2 *lds, const float2 *src) {
    for (int k = threadIdx.x; k < kLinN + 2; k += blockDim.x) lds[k] = src[k];
}

// A voxel box the traversal is confined to (the whole grid or one brick),
// with the strides of the index it reports.
struct Box {
    int x0, y0, z0;  // first voxel (global indices)
    int nx, ny, nz;  // extent
    int sy, sz;      // strides of the reported index
};

// LDS tile of the back projection: a brick's voxels at kTileBase + x +
// kTileSy y + kTileSz z (8-byte entries), with a one-voxel margin on every
// side: x = 16 and y = 16 fall in a row's and a plane's spare slots, and
// the planes z = -1 and z = 16 and the offset kTileBase hold the rest.  A
// walk can end one step past the brick on any axes (a crossing that
// rounding puts just before the exit time: a piece of ~zero weight), and
// such a piece lands in the margin, which is not copied out.
//
// An 8-byte entry spans two of the 32 four-byte LDS banks, so its bank
// pair is the slot index mod 16.  Steps along x, y and z move the slot by
// 1, 18 and 310, i.e. by 1, 2 and 6 bank pairs: the voxels that a
// wavefront's side-by-side rays reach at one step (a patch across the rays'
// direction) spread over the bank pairs.  With strides 17 and 289 (a step
// along any axis moving one pair) the brick kernel ran 5 % slower.
constexpr int kTileSy = kBrickX + 2, kTileSz = kTileSy * (kBrickY + 1) + 4;
static_assert(kTileSy > kBrickX && kTileSz > kTileSy * kBrickY, "the tile needs its margin");
constexpr int kTileBase = 1 + kTileSy + kTileSz;
constexpr int kTileSlots = kTileBase + kBrickX + kTileSy * kBrickY + kTileSz * kBrickZ + 1;

// Voxel-by-voxel traversal of a ray inside a box, without divergent
// branches: each step advances the axis whose next plane is crossed first
// (ties go x, then y, then z; the tied axes follow with zero-length pieces).
// Crossing times come from the plane index (never by adding up steps).
struct Stepper {
    float kx, ky, kz;  // next plane on each axis, minus the anchor index
    float tx, ty, tz;  // its crossing time
    float sx, sy, sz;  // +-1: plane index step
    int j;             // current voxel, box-local index
    int djx, djy, djz; // index step per axis
    int max_steps;

    // Start in the voxel holding r(ta), clamped into B.
    __device__ __forceinline__ Stepper(const Problem &P, const Ray &r, float ta, const Box &B) {
        int ix = min(max(voxel_at(ta, r.ux, r.jx, r.dx, P.ivx), B.x0), B.x0 + B.nx - 1);
        int iy = min(max(voxel_at(ta, r.uy, r.jy, r.dy, P.ivy), B.y0), B.y0 + B.ny - 1);
        int iz = min(max(voxel_at(ta, r.uz, r.jz, r.dz, P.ivz), B.z0), B.z0 + B.nz - 1);
        const bool px = r.ux > 0.0f, py = r.uy > 0.0f, pz = r.uz > 0.0f;
        sx = px ? 1.0f : -1.0f;
        sy = py ? 1.0f : -1.0f;
        sz = pz ? 1.0f : -1.0f;
        kx = (float)(ix + px - r.jx);
        ky = (float)(iy + py - r.jy);
        kz = (float)(iz + pz - r.jz);
        tx = fmaf(kx, r.ax, r.bx);
        ty = fmaf(ky, r.ay, r.by);
        tz = fmaf(kz, r.az, r.bz);
        j = (ix - B.x0) + B.sy * (iy - B.y0) + B.sz * (iz - B.z0);
        djx = px ? 1 : -1;
        djy = py ? B.sy : -B.sy;
        djz = pz ? B.sz : -B.sz;
        max_steps = B.nx + B.ny + B.nz + 2;
    }
    // Start from a brick item's walk record (see write_item_walk): kxy and
    // kzv are its packed plane indices, first voxel and entry code.  j is
    // then the brick-local voxel index times unit (the caller's bytes per
    // voxel), and [ta, tb] the item's piece of the window [tw0, tw1]: ta is
    // the crossing of the plane behind the first voxel on the axis the code
    // names (the face the window entered the brick by), or tw0; tb the
    // first crossing of the brick's three far faces, or tw1.
    __device__ __forceinline__ Stepper(const Ray &r, uint32_t kxy, uint32_t kzv, int unit, float tw0, float tw1,
                                       float &ta, float &tb) {
        const bool px = r.ax > 0.0f, py = r.ay > 0.0f, pz = r.az > 0.0f;  // A has the sign of u
        sx = px ? 1.0f : -1.0f;
        sy = py ? 1.0f : -1.0f;
        sz = pz ? 1.0f : -1.0f;
        kx = (float)(int16_t)(kxy & 0xffffu);
        ky = (float)(int16_t)(kxy >> 16);
        kz = (float)(int16_t)(kzv & 0xffffu);
        tx = fmaf(kx, r.ax, r.bx);
        ty = fmaf(ky, r.ay, r.by);
        tz = fmaf(kz, r.az, r.bz);
        const int v = (int)((kzv >> 16) & (uint32_t)(kBrickVox - 1));  // brick-local voxel, x fastest
        const int vx = v & (kBrickX - 1), vy = (v / kBrickX) & (kBrickY - 1), vz = v / (kBrickX * kBrickY);
        j = (kTileBase + vx + kTileSy * vy + kTileSz * vz) * unit;
        djx = px ? unit : -unit;
        djy = (py ? kTileSy : -kTileSy) * unit;
        djz = (pz ? kTileSz : -kTileSz) * unit;
        max_steps = kBrickX + kBrickY + kBrickZ + 2;
        const uint32_t code = kzv >> 28;
        const float ex = fmaf(kx - sx, r.ax, r.bx), ey = fmaf(ky - sy, r.ay, r.by), ez = fmaf(kz - sz, r.az, r.bz);
        ta = code == 1u ? ex : (code == 2u ? ey : (code == 3u ? ez : tw0));
        // the far face is (brick edge - 1 - v) planes past the next plane
        // going up an axis, v planes going down
        const float qx = fmaf(sx, (float)(px ? kBrickX - 1 - vx : vx), kx);
        const float qy = fmaf(sy, (float)(py ? kBrickY - 1 - vy : vy), ky);
        const float qz = fmaf(sz, (float)(pz ? kBrickZ - 1 - vz : vz), kz);
        tb = fminf(fminf(fminf(fmaf(qx, r.ax, r.bx), fmaf(qy, r.ay, r.by)), fmaf(qz, r.az, r.bz)), tw1);
    }
    __device__ __forceinline__ float next() const { return fminf(fminf(tx, ty), tz); }
    __device__ __forceinline__ void advance(const Ray &r, float tmin) {
        // (the masks are combined as wavefront bit masks: the tie rules
        // then cost two vector compares, not three)
        const uint64_t ex = __builtin_amdgcn_ballot_w64(tx == tmin);
        const uint64_t ey = __builtin_amdgcn_ballot_w64(ty == tmin);
        const bool mx = __builtin_amdgcn_inverse_ballot_w64(ex);
        const bool my = __builtin_amdgcn_inverse_ballot_w64(ey & ~ex);
        const bool mz = __builtin_amdgcn_inverse_ballot_w64(~(ex | ey));
        kx += mx ? sx : 0.0f;
        ky += my ? sy : 0.0f;
        kz += mz ? sz : 0.0f;
        tx = fmaf(kx, r.ax, r.bx);
        ty = fmaf(ky, r.ay, r.by);
        tz = fmaf(kz, r.az, r.bz);
        // exactly one axis moves (selects between values held in
        // registers; selecting between members by reference would be
        // folded into a load through a selected address, off registers)
        const int dx = djx, dy = djy, dz = djz;
        j += mx ? dx : (my ? dy : dz);
    }
};

// The same traversal over the whole grid, reporting the voxel's byte
// offset in the blocked copy of the image (the forward pass gathers from
// it).  A step along an axis adds +-1 to that axis's bits of the offset
// (the sub-block bits and the block field): OR-ing in the other bits
// carries through them, and the other bits are then put back.
struct StepperB {
    float kx, ky, kz, tx, ty, tz, sx, sy, sz;
    uint32_t off;                 // byte offset of the current voxel
    uint32_t mx_, my_, mz_;       // each axis's bits of the offset
    uint32_t dx_, dy_, dz_;       // +1 (lowest bit) or -1 (all bits) within them
    int max_steps;

    __device__ __forceinline__ StepperB(const Problem &P, const Ray &r, float ta) {
        const int ix = min(max(voxel_at(ta, r.ux, r.jx, r.dx, P.ivx), 0), P.nx - 1);
        const int iy = min(max(voxel_at(ta, r.uy, r.jy, r.dy, P.ivy), 0), P.ny - 1);
        const int iz = min(max(voxel_at(ta, r.uz, r.jz, r.dz, P.ivz), 0), P.nz - 1);
        const bool px = r.ux > 0.0f, py = r.uy > 0.0f, pz = r.uz > 0.0f;
        sx = px ? 1.0f : -1.0f;
        sy = py ? 1.0f : -1.0f;
        sz = pz ? 1.0f : -1.0f;
        kx = (float)(ix + px - r.jx);
        ky = (float)(iy + py - r.jy);
        kz = (float)(iz + pz - r.jz);
        tx = fmaf(kx, r.ax, r.bx);
        ty = fmaf(ky, r.ay, r.by);
        tz = fmaf(kz, r.az, r.bz);
        const uint32_t fx = (uint32_t)P.xfx, fxy = (uint32_t)(P.xfx + P.xfy);
        const uint32_t blk = ((uint32_t)(iz >> 2) << fxy) | ((uint32_t)(iy >> 2) << fx) | (uint32_t)(ix >> 2);
        off = ((blk << 6) | ((uint32_t)(iz & 3) << 4) | ((uint32_t)(iy & 3) << 2) | (uint32_t)(ix & 3)) << 2;
        mx_ = in_vgpr((3u << 2) | (((1u << fx) - 1u) << 8));
        my_ = in_vgpr((3u << 4) | (((1u << P.xfy) - 1u) << (8 + fx)));
        mz_ = in_vgpr((3u << 6) | (~0u << (8 + fxy)));
        dx_ = px ? 4u : mx_;
        dy_ = py ? 16u : my_;
        dz_ = pz ? 64u : mz_;
        max_steps = P.nx + P.ny + P.nz + 2;
    }
    __device__ __forceinline__ float next() const { return fminf(fminf(tx, ty), tz); }
    __device__ __forceinline__ void advance(const Ray &r, float tmin) {
        const bool mx = tx == tmin;
        const bool my = !mx && ty == tmin;
        const bool mz = !mx && !my;
        kx += mx ? sx : 0.0f;
        ky += my ? sy : 0.0f;
        kz += mz ? sz : 0.0f;
        tx = fmaf(kx, r.ax, r.bx);
        ty = fmaf(ky, r.ay, r.by);
        tz = fmaf(kz, r.az, r.bz);
        const uint32_t ax = mx_, ay = my_, az = mz_, ex = dx_, ey = dy_, ez = dz_;
        const uint32_t m = mx ? ax : (my ? ay : az);
        const uint32_t d = mx ? ex : (my ? ey : ez);
        const uint32_t v = (off & m) | ~m;
        off = ((v + d) & m) | (off & ~m);
    }
};

// Walk the voxels of ray r between ta and tb (already inside box B) and call
// visit(j, a) for every piece, j box-local.  A plane tie gives a
// zero-length piece (a = 0).  The piece [t, t'] ends at the next crossing
// clamped into [t, tb].
template <bool TOF, class C, class Visit>
__device__ __forceinline__ void walk_from(Stepper &s, const Ray &r, float ta, float tb, const C &cdf,
                                          Visit &&visit);

template <bool TOF, class C, class Visit>
__device__ __forceinline__ void walk(const Problem &P, const Ray &r, float ta, float tb, const Box &B,
                                     const C &cdf, Visit &&visit) {
    Stepper s(P, r, ta, B);
    walk_from<TOF>(s, r, ta, tb, cdf, visit);
}

template <bool TOF, class C, class Visit>
__device__ __forceinline__ void walk_from(Stepper &s, const Ray &r, float ta, float tb, const C &cdf,
                                          Visit &&visit) {
    float t = ta;
    float c = TOF ? cdf(ta) : 0.0f;
    for (int step = 0; step < s.max_steps; ++step) {
        const float tmin = s.next();
        const float tn = __builtin_amdgcn_fmed3f(tmin, t, tb);
        float a;
        if (TOF) {
            const float cn = cdf(tn);
            a = cn - c;
            c = cn;
        } else {
            a = tn - t;
        }
        t = tn;
        visit(s.j, a);
        if (tmin >= tb) break;
        s.advance(r, tmin);
    }
}

// walk_from for a brick item (a Stepper made from its walk record, at
// most kBrickX + kBrickY + kBrickZ + 2 steps): the same pieces in the same
// order, unrolled so that the step bound is tested once per five pieces.
template <bool TOF, class C, class Visit>
__device__ __forceinline__ void walk_item(Stepper &s, const Ray &r, float ta, float tb, const C &cdf,
                                          Visit &&visit) {
    float t = ta;
    float c = TOF ? cdf(ta) : 0.0f;
#pragma unroll 5
    for (int step = 0; step < kBrickX + kBrickY + kBrickZ + 2; ++step) {
        const float tmin = s.next();
        const float tn = __builtin_amdgcn_fmed3f(tmin, t, tb);
        float a;
        if (TOF) {
            const float cn = cdf(tn);
            a = cn - c;
            c = cn;
        } else {
            a = tn - t;
        }
        t = tn;
        visit(s.j, a);
        if (tmin >= tb) break;
        s.advance(r, tmin);
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

// Part of the window inside box B (same crossing formula as the walk).
__device__ __forceinline__ void clip_to_box(const Problem &P, const Ray &r, const Box &B, float &ta, float &tb) {
    ta = r.t0;
    tb = r.t1;
    slab(B.x0, B.x0 + B.nx, r.jx, P.vx, r.dx, r.ux, r.ax, r.bx, ta, tb);
    slab(B.y0, B.y0 + B.ny, r.jy, P.vy, r.dy, r.uy, r.ay, r.by, ta, tb);
    slab(B.z0, B.z0 + B.nz, r.jz, P.vz, r.dz, r.uz, r.az, r.bz, ta, tb);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

__device__ __forceinline__ int find_problem(const Problem *probs, int n_probs, int64_t c) {
    int p = n_probs - 1;
    while (p > 0 && probs[p].chunk_begin > c) --p;
    return p;
}

// Chunk of workgroup b of n: the hardware deals workgroups to the 8 XCDs
// in turn (b mod 8); this gives XCD x the x-th contiguous eighth of the
// chunks, in order.
__device__ __forceinline__ int64_t xcd_chunk(uint32_t b, uint32_t n) {
    const uint32_t per = (n + 7) / 8, x = b & 7u, r = b >> 3;
    const uint32_t full = n - (per - 1) * 8;  // XCDs that get `per` chunks (the rest get per - 1)
    return x < full ? (int64_t)x * per + r : (int64_t)full * per + (int64_t)(x - full) * (per - 1) + r;
}

__device__ __forceinline__ int find_brick_problem(const Problem *probs, int n_probs, uint32_t b) {
    int p = n_probs - 1;
    while (p > 0 && (uint32_t)probs[p].brick_base > b) --p;
    return p;
}

__device__ __forceinline__ void stage_lut(float4 *lds, const float4 *src) {
    for (int k = threadIdx.x; k < kLutN + 2; k += blockDim.x) lds[k] = src[k];
}

__device__ __forceinline__ float at_byte(gptr<const float> p, uint32_t off) {
    return *reinterpret_cast<gptr<const float>>(reinterpret_cast<gptr<const char>>(p) + off);
}

// f_i = sum_j a_ij x_j over the window of ray r, gathering from the blocked
// image copy.  The image value of the next voxel is fetched one piece
// ahead, so its latency overlaps the weight computation of the current piece.
template <bool TOF>
__device__ __forceinline__ float forward_ray(const Problem &P, const Ray &r, const Cdf &cdf, gptr<const float> xb,
                                             uint32_t last_off) {
    StepperB s(P, r, r.t0);
    const float tb = r.t1;
    float t = r.t0;
    float c = TOF ? cdf(t) : 0.0f;
    float f = 0.0f;
    float xj = at_byte(xb, min(s.off, last_off));
    for (int step = 0; step < s.max_steps; ++step) {
        const float tmin = s.next();
        const float tn = __builtin_amdgcn_fmed3f(tmin, t, tb);
        float a;
        if (TOF) {
            const float cn = cdf(tn);
            a = cn - c;
            c = cn;
        } else {
            a = tn - t;
        }
        t = tn;
        f = fmaf(a, xj, f);
        if (tmin >= tb) break;
        s.advance(r, tmin);
        xj = at_byte(xb, min(s.off, last_off));
    }
    return f;
}

// Forward projection of one chunk of events.  mode 0 (MLEM): out[i] =
// 1 / f_i (0 if f_i <= 0) plus per-chunk partials (events with f > 0, sum
// of log f); mode 1: out[i] = f_i.  out is indexed by stored event position.
template <bool TOF, bool PACKED>
__device__ __forceinline__ void forward_chunk(const Problem &P, int64_t base, int ept, int mode, const Cdf &cdf,
                                              int &neff, float &ll) {
    const gptr<const float> xb = global(P.xb);
    const gptr<float> out = global(P.rw);
    // last float of the copy: steps just past the grid edge stay inside it
    const uint32_t last_off = (uint32_t)(xblocks(P) * 256 - 4);
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        const float f = make_ray<PACKED>(P, i, r) ? forward_ray<TOF>(P, r, cdf, xb, last_off) : 0.0f;
        if (mode == 0) {
            const bool pos = f > 0.0f;
            const float w = pos ? 1.0f / f : 0.0f;
            neff += pos;
            ll += pos ? logf(f) : 0.0f;
            out[i] = w;
        } else {
            out[i] = f;
        }
    }
}

template <bool TOF>
__global__ void __launch_bounds__(kForwardBlock) k_forward(const Problem *__restrict__ probs, int n_probs, int ept,
                                                           int mode, int *__restrict__ part_neff,
                                                           double *__restrict__ part_ll) {
    __shared__ float4 lut[kLutN + 2];
    __shared__ int s_n[kForwardBlock / 64];
    __shared__ double s_l[kForwardBlock / 64];
    const int64_t c = blockIdx.x;
    const Problem P = probs[find_problem(probs, n_probs, c)];
    if (TOF) stage_lut(lut, P.lut);
    __syncthreads();
    const Cdf cdf{lut, in_vgpr(P.lut_a), P.lut_b};
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    int neff = 0;
    float ll = 0.0f;
    if (P.packed)
        forward_chunk<TOF, true>(P, base, ept, mode, cdf, neff, ll);
    else
        forward_chunk<TOF, false>(P, base, ept, mode, cdf, neff, ll);
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

// Back projection, in two launches over the brick chunks.
//
// The LDS accumulation is 64-bit fixed point: FP32 LDS atomic adds run at
// ~0.2 T/s on this part, 64-bit integer ones at ~2.8 T/s.  A brick's
// contributions a w are scaled by S = 2^e and rounded to integers, e being
// chosen per brick from its item count n, the problem's bound a_max on a
// piece weight and the brick's largest |w|, so that n a_max w_max S < 2^62:
// no sum can overflow.  Chunk tiles stay 64-bit
// and are added exactly, so b does not depend on how the brick's items are
// ordered or cut into chunks: the result is deterministic, and the same
// for a problem run alone or batched with others.
//
// Brick table entry (brick id, first tile slot, end tile slot, items in the
// brick); chunk (brick table index, first item, end item, tile slot).

// P.bwmax <- 0 over every problem's bricks and P.gflag <- 0 (before the
// combine pass sets them).
__global__ void __launch_bounds__(256) k_clear_bwmax(const Problem *__restrict__ probs, int n_probs,
                                                     int64_t n_bricks) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_bricks) return;
    const Problem &P = probs[find_brick_problem(probs, n_probs, (uint32_t)g)];
    const uint32_t bl = (uint32_t)g - (uint32_t)P.brick_base;
    P.bwmax[bl] = 0u;
    if (bl == 0) P.gflag[0] = 0u;
}

// A brick's fixed-point scale depends only on the binary exponent of its
// largest |w|, so P.bwmax keeps, per brick, the largest exponent field of
// its items' |w| (1 for a subnormal, 0 for zero), stored as that power of
// two's float bits: it has the largest |w|'s frexp exponent.
__device__ __forceinline__ uint32_t weight_exponent(float w) {
    const uint32_t u = __float_as_uint(w) & 0x7fffffffu;
    const uint32_t e = u >> 23;
    return e == 0u && u != 0u ? 1u : e;
}

// The largest exponent of |w| over a brick chunk's items into its brick's
// P.bwmax, for problems whose combine pass wrote weights outside its runs.
__global__ void __launch_bounds__(256) k_brick_wmax(const Problem *__restrict__ probs, int n_probs,
                                                    const uint4 *__restrict__ chunks,
                                                    const uint4 *__restrict__ bricks) {
    __shared__ uint32_t s_max;
    const uint4 ch = chunks[blockIdx.x];
    const uint4 br = bricks[ch.x];
    const Problem &P = probs[find_brick_problem(probs, n_probs, br.x)];
    if (global(P.gflag)[0] == 0u) return;  // (uniform)
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    const gptr<const float> pw = global(P.pw);
    uint32_t m = 0u;
    for (uint32_t k = ch.y + threadIdx.x; k < ch.z; k += blockDim.x) m = max(m, weight_exponent(pw[k]));
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomicMax(&s_max, m);
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(P.bwmax + (br.x - (uint32_t)P.brick_base), s_max << 23);
}

// Fixed-point exponent of a brick (same value in every chunk and the
// reduce), from the exponent of the largest |w| over its items (an
// order-independent bound: the same whatever events share the forward
// chunks).
__device__ __forceinline__ int brick_exponent(const Problem &P, const uint4 &br, float &wmax) {
    const float wm = __uint_as_float(P.bwmax[br.x - (uint32_t)P.brick_base]);
    wmax = wm;
    int en, ea, ew;
    frexpf((float)br.w, &en);
    frexpf(P.a_max, &ea);
    frexpf(wm, &ew);
    // n a_max w_max 2^e < 2^62 (no sum overflows) and a_max w_max 2^e < 2^51
    // (each term is in range of the conversion below)
    return min(max(min(62 - en, 51) - (ea + ew), -126), 126);
}

// round(a w) as a 64-bit two's-complement integer, for |a w| < 2^51: the
// FP64 sum a w + 1.5 2^52 (exact product, one rounding) lies in [2^52,
// 2^53), where doubles are the integers, so its bit pattern is that of
// 1.5 2^52 plus round(a w); the constant's low word is 0, so removing it
// only touches the high word.
__device__ __forceinline__ unsigned long long fixed_round(float a, double w) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(fma((double)a, w, 0x1.8p52));
    const uint32_t hi = (uint32_t)(u >> 32) - 0x43380000u;
    return ((unsigned long long)hi << 32) | (uint32_t)u;
}

// One item's pieces in its brick, from its walk record, added to the tile
// as round(a ws) (ws may be negative; so may a, by ~1e-10 where the
// interpolated CDF dips between nodes).
template <bool TOF>
__device__ __forceinline__ void back_item(const f32x4 &ra, const u32x4 &rb, float tw0, float tw1, float ws,
                                          const CdfLin &cdf, unsigned long long *tile) {
    Ray r;
    r.ax = ra[0];
    r.ay = ra[1];
    r.az = ra[2];
    r.bx = ra[3];
    r.by = __uint_as_float(rb[0]);
    r.bz = __uint_as_float(rb[1]);
    float ta, tb;
    Stepper s(r, rb[2], rb[3], (int)sizeof(unsigned long long), tw0, tw1, ta, tb);
    // j is a byte offset into the tile, inside its margin (see the tile)
    const double wsd = ws;
    walk_item<TOF>(s, r, ta, tb, cdf, [&](int j, float a) {
        atomicAdd(reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(tile) + j), fixed_round(a, wsd));
    });
}

template <bool TOF>
__device__ __forceinline__ void back_chunk_items(const Problem &P, const uint4 &ch, float S, const CdfLin &cdf,
                                                 unsigned long long *tile) {
    const gptr<const float> w = global(P.pw);
    const gptr<const f32x4> rec_a = global(reinterpret_cast<const f32x4 *>(P.rec_a));
    const gptr<const u32x4> rec_b = global(reinterpret_cast<const u32x4 *>(P.rec_b));
    const float tw0 = TOF ? -P.k_sigma : -kInf, tw1 = TOF ? P.k_sigma : kInf;
    // An item's weight sits at its own position (the combine pass put it
    // there), so a wavefront reads weights and walk records coalesced.
    for (uint32_t k = ch.y + threadIdx.x; k < ch.z; k += blockDim.x) {
        const float wv = w[k];
        const f32x4 ra = rec_a[k];
        const u32x4 rb = rec_b[k];
        // (no test for w = 0, which adds zeros: a branch here would let
        // the compiler move the record loads behind the weight's)
        back_item<TOF>(ra, rb, tw0, tw1, wv * S, cdf, tile);
    }
}

// 2. One chunk: sum over its items of round(a_ij w_i 2^e) in an LDS tile,
//    stored (64-bit) to the chunk's tile slot.
template <bool TOF>
__global__ void __launch_bounds__(kBackBlock) k_back_chunks(const Problem *__restrict__ probs, int n_probs,
                                                            const uint4 *__restrict__ chunks,
                                                            const uint4 *__restrict__ bricks) {
    __shared__ unsigned long long tile[kTileSlots];
    __shared__ float2 lut[kLinN + 2];
    const uint4 ch = chunks[blockIdx.x];
    const uint4 br = bricks[ch.x];
    const uint32_t bid = br.x;
    const Problem P = probs[find_brick_problem(probs, n_probs, bid)];
    for (int k = threadIdx.x; k < kTileSlots; k += blockDim.x) tile[k] = 0ull;
    if (TOF) stage_lin(lut, P.lin);
    __syncthreads();
    float wm;
    const int e = brick_exponent(P, br, wm);
    const float S = ldexpf(1.0f, e);
    const CdfLin cdf{lut, in_vgpr(P.lin_a), P.lin_b};
    if (wm > 0.0f) back_chunk_items<TOF>(P, ch, S, cdf, tile);
    __syncthreads();
    const gptr<unsigned long long> dst = global(P.tiles) + (size_t)ch.w * kBrickVox;
    for (int k = threadIdx.x; k < kBrickVox; k += blockDim.x)
        dst[k] = tile[kTileBase + (k & (kBrickX - 1)) + kTileSy * ((k / kBrickX) & (kBrickY - 1)) +
                      kTileSz * (k / (kBrickX * kBrickY))];
}

// 3. b over one brick = (exact sum of its chunk tiles) 2^-e.
//    Four blocks per brick, each a quarter of its voxels.
__global__ void __launch_bounds__(256) k_reduce_tiles(const Problem *__restrict__ probs, int n_probs,
                                                      const uint4 *__restrict__ bricks) {
    const uint4 br = bricks[blockIdx.x >> 2];
    const int k0 = (int)(blockIdx.x & 3u) * (kBrickVox / 4);
    const Problem &P = probs[find_brick_problem(probs, n_probs, br.x)];
    const uint32_t bl = br.x - (uint32_t)P.brick_base;
    const int bx = (int)(bl % (uint32_t)P.nbx), by = (int)((bl / (uint32_t)P.nbx) % (uint32_t)P.nby),
              bz = (int)(bl / ((uint32_t)P.nbx * (uint32_t)P.nby));
    const Box B = brick_box(P, bx, by, bz);
    float wm;
    const float inv = ldexpf(1.0f, -brick_exponent(P, br, wm));
    float *__restrict__ b = P.b;
    const unsigned long long *__restrict__ tiles = P.tiles;
    // each thread sums kReduceVox voxels, their tiles' loads issued together
    constexpr int kReduceVox = kBrickVox / 4 / 256;
    unsigned long long acc[kReduceVox] = {};
    uint32_t sl = br.y;
    for (; sl + 1 < br.z; sl += 2) {  // (two tiles' loads in flight; integer sums, any order)
        unsigned long long u[2][kReduceVox];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < kReduceVox; ++q) u[h][q] = tiles[(size_t)(sl + h) * kBrickVox + k0 + threadIdx.x + 256 * q];
#pragma unroll
        for (int q = 0; q < kReduceVox; ++q) acc[q] += u[0][q] + u[1][q];
    }
    if (sl < br.z) {
#pragma unroll
        for (int q = 0; q < kReduceVox; ++q) acc[q] += tiles[(size_t)sl * kBrickVox + k0 + threadIdx.x + 256 * q];
    }
#pragma unroll
    for (int q = 0; q < kReduceVox; ++q) {
        const int k = k0 + (int)threadIdx.x + 256 * q;
        const int lx = k % kBrickX, ly = (k / kBrickX) % kBrickY, lz = k / (kBrickX * kBrickY);
        if (lx < B.nx && ly < B.ny && lz < B.nz)
            b[(B.x0 + lx) + (int64_t)P.nx * ((B.y0 + ly) + (int64_t)P.ny * (B.z0 + lz))] =
                __ll2float_rn((long long)acc[q]) * inv;
    }
}

// Forward projection by brick chunks (the back projection's chunks).  A
// workgroup stages its brick of x in an LDS tile (the back projection's
// slot layout, FP32, margin 0: the ~zero-weight piece that a walk can take
// one step past the brick reads 0, as do voxels past the grid edge), then
// walks its items' pieces with every gather served by the LDS, and writes
// each item's partial sum of a x to the item's position in P.pw.  An
// event's partials are added by the combine pass, in the order its window
// crosses the bricks, so f does not depend on chunking or batch.
template <bool TOF>
__global__ void __launch_bounds__(kBackBlock) k_forward_items(const Problem *__restrict__ probs, int n_probs,
                                                              const uint4 *__restrict__ chunks,
                                                              const uint4 *__restrict__ bricks) {
    __shared__ float tile[kTileSlots];
    __shared__ float2 lut[kLinN + 2];
    const uint4 ch = chunks[blockIdx.x];
    const uint4 br = bricks[ch.x];
    const Problem P = probs[find_brick_problem(probs, n_probs, br.x)];
    const uint32_t bl = br.x - (uint32_t)P.brick_base;
    const int bx = (int)(bl % (uint32_t)P.nbx), by = (int)((bl / (uint32_t)P.nbx) % (uint32_t)P.nby),
              bz = (int)(bl / ((uint32_t)P.nbx * (uint32_t)P.nby));
    const Box B = brick_box(P, bx, by, bz);
    for (int k = threadIdx.x; k < kTileSlots; k += blockDim.x) tile[k] = 0.0f;
    if (TOF) stage_lin(lut, P.lin);
    __syncthreads();
    const gptr<const float> x = global(P.x);
    for (int k = threadIdx.x; k < kBrickVox; k += blockDim.x) {
        const int lx = k & (kBrickX - 1), ly = (k / kBrickX) & (kBrickY - 1), lz = k / (kBrickX * kBrickY);
        if (lx < B.nx && ly < B.ny && lz < B.nz)
            tile[kTileBase + lx + kTileSy * ly + kTileSz * lz] =
                x[(B.x0 + lx) + (int64_t)P.nx * ((B.y0 + ly) + (int64_t)P.ny * (B.z0 + lz))];
    }
    __syncthreads();
    const CdfLin cdf{lut, in_vgpr(P.lin_a), P.lin_b};
    const gptr<float> pw = global(P.pw);
    const gptr<const f32x4> rec_a = global(reinterpret_cast<const f32x4 *>(P.rec_a));
    const gptr<const u32x4> rec_b = global(reinterpret_cast<const u32x4 *>(P.rec_b));
    const float tw0 = TOF ? -P.k_sigma : -kInf, tw1 = TOF ? P.k_sigma : kInf;
    for (uint32_t k = ch.y + threadIdx.x; k < ch.z; k += blockDim.x) {
        const f32x4 ra = rec_a[k];
        const u32x4 rb = rec_b[k];
        Ray r;
        r.ax = ra[0];
        r.ay = ra[1];
        r.az = ra[2];
        r.bx = ra[3];
        r.by = __uint_as_float(rb[0]);
        r.bz = __uint_as_float(rb[1]);
        float ta, tb;
        Stepper s(r, rb[2], rb[3], (int)sizeof(float), tw0, tw1, ta, tb);
        float p = 0.0f;
        // j is a byte offset into the tile, inside its margin (see the tile)
        walk_item<TOF>(s, r, ta, tb, cdf, [&](int j, float a) {
            p = fmaf(a, *reinterpret_cast<const float *>(reinterpret_cast<const char *>(tile) + j), p);
        });
        pw[k] = p;
    }
}

// The combine pass (see launch_combine), one forward chunk of events per
// 1024-lane workgroup.  The builder recorded the runs of consecutive
// positions the chunk's events fill (one per (brick, item class) key) and,
// per item, its slot in the chunk's event-major order (its event's offset
// plus its ordinal).  Phase 1 reads the items run by run (consecutive lanes,
// consecutive positions) into their LDS slots; phase 2 sums each event's
// slots in ordinal order (the order its window crosses the bricks) and puts
// its weight in every one of its slots; phase 3 writes the slots back to the
// items run by run and keeps the exponent field of each |w| in run order;
// phase 4 takes each brick's largest exponent in LDS, then adds it to
// P.bwmax (one global atomic per brick the chunk touches).  Events the builder flagged (an item placed
// outside the runs) are summed and written through evitems in phase 2, and
// P.gflag is set so that launch_brick_wmax takes their bricks' maxima; a
// chunk with more than kRunEvents events or kRunItems items takes that path
// for every event.
constexpr int kRunEvents = 2048;
constexpr int kRunItems = 8192;
constexpr int kMaxRuns = 1024;  // a chunk has at most one run per slot of the builder's hash table
constexpr int kCombineBlock = 1024;
constexpr int kRunItemsPerThread = kRunItems / kCombineBlock;
constexpr int kCombineEventsPerThread = 4;  // chunks of up to 4096 events (16 per lane of a 256-lane chunk)
constexpr int kBrickSlots = 256;            // LDS table of a chunk's bricks (their maxima)
constexpr int kRunsEager = 256;             // run rows loaded before the run count is known

// v from the lane `off` below in its row of 16 (row_shr); the row's first
// `off` lanes get no valid value (callers test the lane's place).
template <int off>
__device__ __forceinline__ uint32_t row_up(uint32_t v, uint32_t none) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)none, (int)v, 0x110 | off, 0xf, 0xf, false);
}
// v from the next lane in its row of 16 (row_shl:1); not valid in the row's
// last lane.
__device__ __forceinline__ uint32_t row_next(uint32_t v, uint32_t none) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)none, (int)v, 0x101, 0xf, 0xf, false);
}

// An event's f from its items' partials, through evitems.
__device__ __forceinline__ float combine_event_global(const Problem &P, uint32_t k0, uint32_t k1) {
    const gptr<const float> pw = global(P.pw);
    const gptr<const uint32_t> evitems = global(P.evitems);
    float f = 0.0f;
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t q = evitems[k];
        f += q < P.n_items ? pw[q] : 0.0f;
    }
    return f;
}

// An event's weight onto its items, through evitems.
__device__ __forceinline__ void scatter_event_global(const Problem &P, uint32_t k0, uint32_t k1, float w) {
    const gptr<float> pw = global(P.pw);
    const gptr<const uint32_t> evitems = global(P.evitems);
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t q = evitems[k];
        if (q < P.n_items) pw[q] = w;
    }
}

// EPT: events per lane (the chunk's events over kCombineBlock, rounded up).
template <int EPT>
__global__ void __launch_bounds__(kCombineBlock) k_combine(const Problem *__restrict__ probs, int n_probs, int ept,
                                                           int mode, int *__restrict__ part_neff,
                                                           double *__restrict__ part_ll) {
    __shared__ __align__(16) float slot[kRunItems];
    __shared__ __align__(16) uint16_t rid[kRunItems];
    __shared__ uint32_t rbase[kMaxRuns], rpre[kMaxRuns], rbrick[kMaxRuns], rlen[kMaxRuns];
    __shared__ int16_t rslot[kMaxRuns];
    __shared__ __align__(16) uint8_t wexp[kRunItems];
    __shared__ uint32_t bmax[kBrickSlots];
    __shared__ int s_n[kCombineBlock / 64];
    __shared__ double s_l[kCombineBlock / 64];
    // Workgroups are dealt to the 8 XCDs in turn; chunk c of XCD x's share
    // goes to x's workgroups in order, so neighbouring chunks (whose runs
    // sit side by side in the item lists and share cache lines) are
    // combined by one XCD at about the same time, in one L2.
    const int64_t c = xcd_chunk(blockIdx.x, gridDim.x);
    const Problem &P = probs[find_problem(probs, n_probs, c)];
    const int64_t base = (c - P.chunk_begin) * (int64_t)kForwardBlock * ept;
    const int n_ev = (int)min((int64_t)kForwardBlock * ept, P.n_events - base);
    const bool maxima = mode != kCombineF;
    const gptr<float> pw = global(P.pw);
    const gptr<const uint16_t> itemslot = global(P.itemslot);
    const gptr<const uint32_t> evoff = global(P.evoff);
    const gptr<const uint32_t> runs = global(P.runs) + (size_t)(c - P.chunk_begin) * kTabWords;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // this thread's events (tid + q blockDim), their offsets and flags,
    // loaded with the first runs
    uint32_t k0[EPT], k1[EPT];
    bool has_ev[EPT], flagged[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int le = tid + q * kCombineBlock;
        has_ev[q] = le < n_ev;
        k0[q] = has_ev[q] ? evoff[base + le] : 0u;
        k1[q] = has_ev[q] ? evoff[base + le + 1] : 0u;
        flagged[q] = has_ev[q] && P.evflag[base + le];
    }
    const uint32_t E0 = evoff[base], E1 = evoff[base + n_ev];
    const uint32_t nr = runs[0], T = runs[1];
    // run rows (see brick_items_pass); rows past kRunsEager are loaded once
    // the count says they exist (a chunk has ~100 runs)
    const gptr<const u32x4> rows = (gptr<const u32x4>)(runs + kTabHead);
    u32x4 row = {0u, 0u, 0u, 0u};
    if (tid < kRunsEager)
        row = rows[tid];
    else if ((uint32_t)tid < nr)
        row = rows[tid];
    const uint32_t bslot = (row.y >> 16) & 0x7fffu;
    const bool owner = maxima && (uint32_t)tid < nr && (row.y >> 31) != 0u && bslot != 0x7fffu;
    const bool by_runs = n_ev <= kRunEvents && E1 - E0 <= (uint32_t)kRunItems && T <= E1 - E0;
    if ((uint32_t)tid < nr) {
        rbase[tid] = row.x;
        rlen[tid] = row.y & 0xffffu;
        rpre[tid] = row.z;
        rbrick[tid] = row.w;
        rslot[tid] = bslot != 0x7fffu ? (int16_t)bslot : (int16_t)-1;
    }
    if (tid < kBrickSlots) bmax[tid] = 0u;
    __syncthreads();
    // the run of each run-order slot: a wavefront's lanes fill a run's slots
    if (by_runs)
        for (uint32_t r = (uint32_t)wid; r < nr; r += kCombineBlock / 64) {
            const uint32_t p0 = rpre[r], l = rlen[r];
            for (uint32_t j = (uint32_t)lane; j < l; j += 64) rid[p0 + j] = (uint16_t)r;
        }
    __syncthreads();
    // phase 1: the thread's items (positions and slots kept for phase 3)
    uint32_t pos[kRunItemsPerThread], sl[kRunItemsPerThread];
#pragma unroll
    for (int m = 0; m < kRunItemsPerThread; ++m) {
        const uint32_t t = (uint32_t)(tid + m * kCombineBlock);
        pos[m] = 0;
        sl[m] = 0xffffu;
        if (by_runs && t < T) {
            sl[m] = itemslot[E0 + t];  // (stored in run order: coalesced)
            const uint32_t r = rid[t];
            pos[m] = rbase[r] + (t - rpre[r]);
        }
    }
    if (mode != kCombineWeights) {
        // (loaded with the slots, not after them: pos is a run position)
        float v[kRunItemsPerThread];
#pragma unroll
        for (int m = 0; m < kRunItemsPerThread; ++m)
            v[m] = by_runs && (uint32_t)(tid + m * kCombineBlock) < T ? pw[pos[m]] : 0.0f;
#pragma unroll
        for (int m = 0; m < kRunItemsPerThread; ++m)
            if (sl[m] != 0xffffu) slot[sl[m]] = v[m];
    }
    __syncthreads();
    // phase 2: the thread's events
    int neff = 0;
    float ll = 0.0f;
    bool any_glob = false;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        if (!has_ev[q]) continue;
        const int64_t i = base + tid + q * kCombineBlock;
        const bool glob = !by_runs || flagged[q];
        const uint32_t s0 = k0[q] - E0, cnt = k1[q] - k0[q];
        float w;
        if (mode == kCombineWeights) {
            w = P.rw[i];
        } else {
            float f = 0.0f;
            if (glob) {
                f = combine_event_global(P, k0[q], k1[q]);
            } else {
                for (uint32_t k = 0; k < cnt; ++k) f += slot[s0 + k];
            }
            if (mode == kCombineF) {
                global(P.rw)[i] = f;
                continue;
            }
            const bool ok = f > 0.0f;
            w = ok ? 1.0f / f : 0.0f;
            neff += ok;
            ll += ok ? logf(f) : 0.0f;
        }
        if (P.evw) w *= P.evw[i];
        if (by_runs)
            for (uint32_t k = 0; k < cnt; ++k) slot[s0 + k] = w;
        if (glob) {
            scatter_event_global(P, k0[q], k1[q], w);
            any_glob = true;
        }
    }
    if (mode == kCombineF) return;
    // items written through evitems: their bricks' maxima are taken by
    // launch_brick_wmax
    if (any_glob) global(P.gflag)[0] = 1u;
    // the wavefront's count and log-likelihood, added up at the end
    {
        const int wn = wave_sum(neff);
        const double wl = wave_sum((double)ll);
        if (lane == 0) {
            s_n[wid] = wn;
            s_l[wid] = wl;
        }
    }
    __syncthreads();
    // phase 3: weights onto the items; the exponent field of each |w| to
    // the run order (in its own array: the slots are still being read)
#pragma unroll
    for (int m = 0; m < kRunItemsPerThread; ++m) {
        if (sl[m] != 0xffffu) {
            const float w = slot[sl[m]];
            pw[pos[m]] = w;
            wexp[tid + m * kCombineBlock] = (uint8_t)weight_exponent(w);
        }
    }
    __syncthreads();
    // phase 4: each brick's largest exponent.  A thread takes 8 consecutive slots
    // of the run order: a run that starts and ends among them goes to its
    // brick at once; the pieces of runs that cross thread boundaries are
    // combined by a segmented max scan over each row of 16 lanes (run ids
    // do not decrease along the lanes; DPP moves, no LDS), and the lane where
    // such a run ends, or the row's last lane, adds it.  The bricks' maxima
    // are kept in LDS, then added to P.bwmax.
    {
        const uint32_t t8 = 8u * (uint32_t)tid;
        constexpr uint32_t kNone = 0xffffffffu;
        uint32_t fk = kNone, lk = kNone;  // first and last piece's run
        uint32_t fv = 0u, lv = 0u;        // and their largest exponents
        bool multi = false;
        auto to_brick = [&](uint32_t run, uint32_t mx) {
            const int b = rslot[run];
            if (b >= 0)
                atomicMax(&bmax[b], mx);
            else
                atomicMax(P.bwmax + rbrick[run], mx << 23);  // brick table full
        };
        if (by_runs && t8 < T) {
            const uint2 ee = *reinterpret_cast<const uint2 *>(&wexp[t8]);
            const uint4 rr = *reinterpret_cast<const uint4 *>(&rid[t8]);
            const uint32_t v[8] = {ee.x & 0xffu, (ee.x >> 8) & 0xffu, (ee.x >> 16) & 0xffu, ee.x >> 24,
                                   ee.y & 0xffu, (ee.y >> 8) & 0xffu, (ee.y >> 16) & 0xffu, ee.y >> 24};
            const uint32_t r[8] = {rr.x & 0xffffu, rr.x >> 16, rr.y & 0xffffu, rr.y >> 16,
                                   rr.z & 0xffffu, rr.z >> 16, rr.w & 0xffffu, rr.w >> 16};
            const uint32_t n = min(8u, T - t8);
            fk = r[0];
            uint32_t cur = r[0];
            uint32_t mx = v[0];
#pragma unroll
            for (uint32_t k = 1; k < 8; ++k) {
                if (k >= n) break;
                if (r[k] != cur) {
                    if (!multi) {
                        fv = mx;
                        multi = true;
                    } else {
                        to_brick(cur, mx);  // the whole run is here
                    }
                    cur = r[k];
                    mx = v[k];
                } else {
                    mx = max(mx, v[k]);
                }
            }
            lk = cur;
            lv = mx;
        }
        // (the lane's place in its row decides which moves are valid)
        const int rl16 = lane & 15;
        uint32_t sv = lv;
        {
            // (every lane makes each move: none is inside a branch)
            uint32_t o = row_up<1>(sv, 0u), ok = row_up<1>(lk, kNone);
            sv = rl16 >= 1 && ok == lk ? max(sv, o) : sv;
            o = row_up<2>(sv, 0u);
            ok = row_up<2>(lk, kNone);
            sv = rl16 >= 2 && ok == lk ? max(sv, o) : sv;
            o = row_up<4>(sv, 0u);
            ok = row_up<4>(lk, kNone);
            sv = rl16 >= 4 && ok == lk ? max(sv, o) : sv;
            o = row_up<8>(sv, 0u);
            ok = row_up<8>(lk, kNone);
            sv = rl16 >= 8 && ok == lk ? max(sv, o) : sv;
        }
        const uint32_t pv = row_up<1>(sv, 0u), pk = row_up<1>(lk, kNone);
        const uint32_t nf = row_next(fk, kNone);
        // the first piece ends a run that began in an earlier lane or here
        if (multi) to_brick(fk, rl16 >= 1 && pk == fk ? max(fv, pv) : fv);
        if (lk != kNone && (rl16 == 15 || nf != lk)) to_brick(lk, sv);
    }
    __syncthreads();
    if (by_runs && owner) atomicMax(P.bwmax + row.w, bmax[bslot] << 23);
    if (tid == 0 && mode == kCombineRatio) {
        int tn = 0;
        double tl = 0.0;
        for (int w = 0; w < kCombineBlock / 64; ++w) {
            tn += s_n[w];
            tl += s_l[w];
        }
        part_neff[c] = tn;
        part_ll[c] = tl;
    }
}

// Per-block open-addressing table in LDS mapping a brick id to a slot.
constexpr int kHashSlots = 1024;
static_assert(kTabWords >= 2 * kHashSlots && kTabWords >= kTabHead + 4 * kMaxRuns,
              "a chunk's table holds its hash table, then its run rows");
static_assert(kHashSlots % kForwardBlock == 0 && kBrickSlots < 0x7fff && kRunEvents < 0x10000,
              "run rows: lengths in 16 bits, brick slots in 15");
static_assert(kHashSlots <= kMaxRuns && kMaxRuns <= kCombineBlock, "the combine pass loads every run of a chunk");
static_assert(kRunItems <= 65535 && kRunEvents <= kCombineEventsPerThread * kCombineBlock,
              "item slots are 16-bit; a thread holds its events");
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
// visit(global brick id, bx, by, bz, t_in, t_out) for every brick crossed
// over a positive length [t_in, t_out].
// Brick faces are voxel planes, so this uses the voxel walk's crossing
// formulas and cuts the window exactly where the brick pieces meet.
template <class Visit>
__device__ __forceinline__ void brick_walk(const Problem &P, const Ray &r, Visit &&visit) {
    const bool px = r.ux > 0.0f, py = r.uy > 0.0f, pz = r.uz > 0.0f;
    int bx = min(max(voxel_at(r.t0, r.ux, r.jx, r.dx, P.ivx), 0), P.nx - 1) / kBrickX;
    int by = min(max(voxel_at(r.t0, r.uy, r.jy, r.dy, P.ivy), 0), P.ny - 1) / kBrickY;
    int bz = min(max(voxel_at(r.t0, r.uz, r.jz, r.dz, P.ivz), 0), P.nz - 1) / kBrickZ;
    const int sx = px ? 1 : -1, sy = py ? 1 : -1, sz = pz ? 1 : -1;
    float tnx = cross((bx + px) * kBrickX, r.jx, r.ax, r.bx);
    float tny = cross((by + py) * kBrickY, r.jy, r.ay, r.by);
    float tnz = cross((bz + pz) * kBrickZ, r.jz, r.az, r.bz);
    float t = r.t0;
    const int max_steps = P.nbx + P.nby + P.nbz + 2;
    for (int step = 0; step < max_steps; ++step) {
        const float tmin = fminf(fminf(tnx, tny), tnz);
        const float tn = fminf(tmin, r.t1);
        if (tn > t) visit((uint32_t)P.brick_base + (uint32_t)(bx + P.nbx * (by + P.nby * bz)), bx, by, bz, t, tn);
        if (tmin >= r.t1) break;
        t = fmaxf(tn, t);
        // one axis moves (x, then y, then z on ties); masked updates of
        // values, not a branch per axis (which the compiler may turn into
        // stores and loads through a selected address, off registers)
        const bool mx = tnx == tmin;
        const bool my = !mx && tny == tmin;
        const bool mz = !mx && !my;
        bx += mx ? sx : 0;
        by += my ? sy : 0;
        bz += mz ? sz : 0;
        if ((unsigned)bx >= (unsigned)P.nbx || (unsigned)by >= (unsigned)P.nby || (unsigned)bz >= (unsigned)P.nbz)
            break;
        tnx = mx ? cross((bx + px) * kBrickX, r.jx, r.ax, r.bx) : tnx;
        tny = my ? cross((by + py) * kBrickY, r.jy, r.ay, r.by) : tny;
        tnz = mz ? cross((bz + pz) * kBrickZ, r.jz, r.az, r.bz) : tnz;
    }
}

// Brick item lists, counted and filled per (brick, item class) key =
// brick * kItemClasses + class.  Counting (fill == 0): ctr[key] += pieces,
// and each event's piece count into P.evoff[i] (the host turns the counts
// into offsets).  Filling: every piece gets a position from ctr[key]++
// (never past end[key]) where the item's walk record goes (crossing
// coefficients, its piece of the window, first voxel), so that both
// projections stream a chunk's records instead of gathering events and
// re-deriving rays (each event is walked once per brick it crosses); the
// event's k-th piece (in the order its window crosses the bricks) has its
// position at P.evitems[P.evoff[i] + k].  When counting, a block
// tallies its pieces per key in an LDS hash table, then touches each global
// counter once (bucketed events make whole blocks hit the same few bricks,
// and same-address global atomics serialise) and keeps the table; when
// filling, the block reloads its table, reserves each key's range, and
// walks its events once, handing out positions from the reserved ranges.
// Walk record of a brick item at position pos (32 bytes): the crossing
// coefficients (A_x, A_y, A_z, B_x), (B_y, B_z, k_x | k_y << 16, k_z | v <<
// 16 | entry << 28) with k the next plane index on each axis minus the
// anchor's and v the brick-local first voxel.  The item's piece [ta, tb]
// of the window is not stored: ta is either the window's start (entry 0,
// with TOF) or the crossing of the brick face the window entered by, which
// is the plane behind the first voxel on that axis (entry 1, 2, 3 for x, y,
// z: the brick walk cut the window there, with the same formula); tb is
// the first crossing of the brick's three far faces, or the window's end.
// (A brick on the grid's far edge reaches past it: its walk then goes on to
// the full brick's face through voxels outside the grid, where the forward
// tile holds zeros and the back projection's sums are not read.)
__device__ __forceinline__ void write_item_walk(const Problem &P, const Ray &r, int bx, int by, int bz, float ta,
                                                uint32_t pos) {
    const Box B = brick_box(P, bx, by, bz);
    const int ix = min(max(voxel_at(ta, r.ux, r.jx, r.dx, P.ivx), B.x0), B.x0 + B.nx - 1);
    const int iy = min(max(voxel_at(ta, r.uy, r.jy, r.dy, P.ivy), B.y0), B.y0 + B.ny - 1);
    const int iz = min(max(voxel_at(ta, r.uz, r.jz, r.dz, P.ivz), B.z0), B.z0 + B.nz - 1);
    const int kx = ix + (r.ux > 0.0f) - r.jx, ky = iy + (r.uy > 0.0f) - r.jy, kz = iz + (r.uz > 0.0f) - r.jz;
    const uint32_t j = (uint32_t)((ix - B.x0) + kBrickX * ((iy - B.y0) + kBrickY * (iz - B.z0)));
    // the face the piece starts on: the candidate crossing equal to ta
    // (the nearest one, should rounding ever leave none equal)
    const int sxi = r.ux > 0.0f ? 1 : -1, syi = r.uy > 0.0f ? 1 : -1, szi = r.uz > 0.0f ? 1 : -1;
    const float dx = fabsf(cross(kx - sxi, 0, r.ax, r.bx) - ta), dy = fabsf(cross(ky - syi, 0, r.ay, r.by) - ta),
                dz = fabsf(cross(kz - szi, 0, r.az, r.bz) - ta);
    uint32_t entry = dy < dx ? (dz < dy ? 3u : 2u) : (dz < dx ? 3u : 1u);
    if (P.tof && ta == -P.k_sigma) entry = 0u;
    // (register copies: element-wise reads of neighbouring Ray fields would
    // otherwise be merged into vector loads that keep the ray off registers)
    f32x4 a;
    u32x4 b;
    a[0] = in_vgpr(r.ax); a[1] = in_vgpr(r.ay); a[2] = in_vgpr(r.az); a[3] = in_vgpr(r.bx);
    b[0] = __float_as_uint(in_vgpr(r.by));
    b[1] = __float_as_uint(in_vgpr(r.bz));
    b[2] = ((uint32_t)kx & 0xffffu) | ((uint32_t)ky << 16);
    b[3] = ((uint32_t)kz & 0xffffu) | (j << 16) | (entry << 28);
    global(reinterpret_cast<f32x4 *>(const_cast<float4 *>(P.rec_a)))[pos] = a;
    global(reinterpret_cast<u32x4 *>(const_cast<float4 *>(P.rec_b)))[pos] = b;
}

// Item class of a brick piece [t0, t1] of ray r by its voxel-plane
// crossings (the voxel walk's step count): 0 for 32 or more, then 28-31,
// 25-27, 22-24, 19-21, 16-18, 13-15, 10-12, 7-9, 4-6, 2-3 and 0-1.  Items
// of one class walk nearly the same number of steps, so a wavefront's
// lanes finish together; finer classes would cut that divergence further
// but split a forward chunk's items into more runs, which the combine pass
// and the list build pay for.
__device__ __forceinline__ uint32_t item_class(const Problem &P, const Ray &r, float t0, float t1) {
    const int n = abs(voxel_at(t1, r.ux, r.jx, r.dx, P.ivx) - voxel_at(t0, r.ux, r.jx, r.dx, P.ivx)) +
                  abs(voxel_at(t1, r.uy, r.jy, r.dy, P.ivy) - voxel_at(t0, r.uy, r.jy, r.dy, P.ivy)) +
                  abs(voxel_at(t1, r.uz, r.jz, r.dz, P.ivz) - voxel_at(t0, r.uz, r.jz, r.dz, P.ivz));
    const int edge[kItemClasses - 1] = {32, 28, 25, 22, 19, 16, 13, 10, 7, 4, 2};
    uint32_t k = 0;
#pragma unroll
    for (int q = 0; q < kItemClasses - 1; ++q) k += n < edge[q];
    return k;
}

// Counting (fill == 0): tally the block's pieces per key in the LDS table,
// add them to ctr, and store the table to tab.  Filling: reload the table,
// reserve each key's range, then walk the events once.
template <bool PACKED>
__device__ __forceinline__ void brick_items_pass(const Problem &P, int64_t base, int ept,
                                                 uint32_t *__restrict__ ctr, const uint32_t *__restrict__ end,
                                                 int fill, uint32_t *hkey, uint32_t *hcnt, uint32_t *hbase,
                                                 uint32_t *nruns, uint16_t *qslot, uint32_t *bkey,
                                                 uint32_t *wsum, uint32_t *hpre, gptr<uint32_t> tab) {
    const gptr<uint32_t> evoff = global(const_cast<uint32_t *>(P.evoff));
    const gptr<uint32_t> evitems = global(const_cast<uint32_t *>(P.evitems));
    const gptr<uint16_t> itemslot = global(const_cast<uint16_t *>(P.itemslot));
    const gptr<uint8_t> evflag = global(const_cast<uint8_t *>(P.evflag));
    // the chunk's items in event-major order: [c0, c0 + its count); the
    // combine pass handles a chunk of at most kRunItems items by runs
    uint32_t c0 = 0;
    bool small = false;
    if (fill) {
        const int64_t last = min(base + (int64_t)blockDim.x * ept, P.n_events);
        c0 = evoff[base];
        small = evoff[last] - c0 <= (uint32_t)kRunItems;
    }
    if (fill) {
        // reserve each table key's run of positions (runs numbered in any order)
        for (int k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
            if (hkey[k] == kEmpty) continue;
            hbase[k] = atomicAdd(ctr + hkey[k], hcnt[k]);
            qslot[atomicAdd(nruns, 1u)] = (uint16_t)k;
        }
        __syncthreads();
        // The run rows replace the chunk's (key, count) table, already
        // loaded: the header (run count, items in runs) and per run its first
        // position, its length | brick slot << 16 | owner << 31, the prefix
        // of the lengths before it and its problem-local brick.  Runs of one
        // brick share a slot of the combine pass's LDS table of brick maxima
        // (kBrickSlots; 0x7fff once full); the run that took the slot owns it.
        const uint32_t nr = *nruns;
        constexpr int kPer = kHashSlots / kForwardBlock;
        uint32_t len[kPer], tot = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t q = kPer * threadIdx.x + j;
            len[j] = q < nr ? hcnt[qslot[q]] : 0u;
            tot += len[j];
        }
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        uint32_t x = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        uint32_t pre = x - tot;
        for (int w = 0; w < wid; ++w) pre += wsum[w];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t q = kPer * threadIdx.x + j;
            if (q < nr) {
                const uint32_t k = qslot[q];
                const uint32_t brick = hkey[k] / kItemClasses - (uint32_t)P.brick_base;
                bool owner = false;
                int bs = -1;
                int h = (int)((brick * 2654435761u) >> 24);
                for (int probe = 0; probe < kBrickSlots; ++probe) {
                    uint32_t kk = __hip_atomic_load(&bkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (kk == kEmpty) {
                        kk = atomicCAS(&bkey[h], kEmpty, brick);
                        if (kk == kEmpty) {
                            owner = true;
                            bs = h;
                            break;
                        }
                    }
                    if (kk == brick) {
                        bs = h;
                        break;
                    }
                    h = (h + 1) & (kBrickSlots - 1);
                }
                const uint32_t y = len[j] | ((bs >= 0 ? (uint32_t)bs : 0x7fffu) << 16) | (owner ? 1u << 31 : 0u);
                ((gptr<u32x4>)(tab + kTabHead))[q] = u32x4{hbase[k], y, pre, brick};
                hpre[k] = pre;
            }
            pre += len[j];
        }
        if (threadIdx.x == kForwardBlock - 1) {
            tab[0] = nr;
            tab[1] = pre;  // (the last thread's prefix after its runs: the total)
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kHashSlots; k += blockDim.x) hcnt[k] = 0;
        __syncthreads();
    }
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) continue;
        Ray r;
        const bool ok = make_ray<PACKED>(P, i, r);
        // the event's pieces so far; when filling, where its positions go
        // and whether an item falls outside the runs
        uint32_t n = 0;
        const uint32_t e0 = fill ? evoff[i] : 0u;
        bool outside = false;
        if (ok) brick_walk(P, r, [&](uint32_t brick, int bx, int by, int bz, float t0, float t1) {
            const uint32_t key = brick * kItemClasses + item_class(P, r, t0, t1);
            if (!fill) {
                const int h = hash_insert(hkey, key);
                if (h >= 0)
                    atomicAdd(&hcnt[h], 1u);
                else
                    atomicAdd(ctr + key, 1u);  // table full: counted directly
                ++n;
                return;
            }
            // a key is in the table in both passes, or counted directly in both
            const int h = hash_find(hkey, key);
            const uint32_t pos = h >= 0 ? hbase[h] + atomicAdd(&hcnt[h], 1u) : atomicAdd(ctr + key, 1u);
            const bool in = pos < end[key];
            const bool run = h >= 0 && small;
            if (in) write_item_walk(P, r, bx, by, bz, t0, pos);
            // a run item's slot, at its run-order index in the chunk's range
            // of the item lists (the writes of a chunk stay in a few KB)
            if (run) itemslot[c0 + hpre[h] + (pos - hbase[h])] = (uint16_t)(e0 + n - c0);
            outside = outside || h < 0 || !in;
            // (a position past the key's range, which a consistent count
            // never gives, is marked out of range for the combine pass)
            evitems[e0 + n] = in ? pos : 0xffffffffu;
            ++n;
        });
        if (!fill)
            evoff[i] = n;
        else
            evflag[i] = outside ? 1 : 0;
    }
    if (fill) return;
    __syncthreads();
    for (int k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
        if (hkey[k] != kEmpty) atomicAdd(ctr + hkey[k], hcnt[k]);
        tab[k] = hkey[k];
        tab[kHashSlots + k] = hcnt[k];
    }
}

__global__ void __launch_bounds__(kForwardBlock) k_brick_items(const Problem *__restrict__ probs, int n_probs,
                                                               int ept, uint32_t *__restrict__ ctr,
                                                               const uint32_t *__restrict__ end, int fill,
                                                               uint32_t *__restrict__ tabs) {
    __shared__ uint32_t hkey[kHashSlots], hcnt[kHashSlots], hbase[kHashSlots];
    __shared__ uint16_t qslot[kHashSlots];
    __shared__ uint32_t bkey[kBrickSlots], wsum[kForwardBlock / 64], hpre[kHashSlots];
    __shared__ uint32_t nruns;
    const int64_t c = blockIdx.x;
    const Problem P = probs[find_problem(probs, n_probs, c)];
    const gptr<uint32_t> tab = global(tabs) + (size_t)c * kTabWords;
    for (int k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
        hkey[k] = fill ? tab[k] : kEmpty;
        hcnt[k] = fill ? tab[kHashSlots + k] : 0u;
    }
    for (int k = threadIdx.x; k < kBrickSlots; k += blockDim.x) bkey[k] = kEmpty;
    if (threadIdx.x == 0) nruns = 0;
    __syncthreads();
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    if (P.packed)
        brick_items_pass<true>(P, base, ept, ctr, end, fill, hkey, hcnt, hbase, &nruns, qslot, bkey, wsum, hpre, tab);
    else
        brick_items_pass<false>(P, base, ept, ctr, end, fill, hkey, hcnt, hbase, &nruns, qslot, bkey, wsum, hpre, tab);
}

// Diagnostic: voxel pieces visited per chunk and how many have non-zero weight.
template <bool TOF>
__global__ void __launch_bounds__(kForwardBlock) k_count_pieces(const Problem *__restrict__ probs, int n_probs,
                                                                int ept, unsigned long long *__restrict__ part) {
    __shared__ float4 lut[kLutN + 2];
    __shared__ unsigned long long s_c[kForwardBlock / 64], s_z[kForwardBlock / 64];
    const int64_t c = blockIdx.x;
    const Problem P = probs[find_problem(probs, n_probs, c)];
    if (TOF) stage_lut(lut, P.lut);
    __syncthreads();
    const Cdf cdf{lut, in_vgpr(P.lut_a), P.lut_b};
    const Box B = grid_box(P);
    const int64_t base = (c - P.chunk_begin) * (int64_t)blockDim.x * ept;
    unsigned long long cnt = 0, nz = 0;
    for (int e = 0; e < ept; ++e) {
        const int64_t i = base + (int64_t)e * blockDim.x + threadIdx.x;
        if (i >= P.n_events) break;
        Ray r;
        if (!(P.packed ? make_ray<true>(P, i, r) : make_ray<false>(P, i, r))) continue;
        walk<TOF>(P, r, r.t0, r.t1, B, cdf, [&](int, float a) {
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

// xb <- x in 4^3 blocks: four blocks per 256-thread workgroup, one voxel
// per thread (voxels past the grid edge are 0; padding blocks are left
// alone: they are zeroed when the copy is laid out).
__global__ void __launch_bounds__(256) k_block_image(const Problem *__restrict__ probs, int n_probs) {
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int p = n_probs - 1;
    while (p > 0 && probs[p].xblk_begin > blk) --p;
    const Problem &P = probs[p];
    const int64_t lb = blk - P.xblk_begin;
    if (lb >= xblocks(P)) return;
    const int bx = (int)(lb & ((1 << P.xfx) - 1)), by = (int)((lb >> P.xfx) & ((1 << P.xfy) - 1)),
              bz = (int)(lb >> (P.xfx + P.xfy));
    if (bx >= P.nbx4 || by >= P.nby4) return;
    const int v = threadIdx.x & 63;
    const int ix = 4 * bx + (v & 3), iy = 4 * by + ((v >> 2) & 3), iz = 4 * bz + (v >> 4);
    const float val = (ix < P.nx && iy < P.ny && iz < P.nz) ? P.x[ix + (int64_t)P.nx * (iy + (int64_t)P.ny * iz)] : 0.0f;
    global(P.xb)[lb * 64 + v] = val;
}

// TOF scatter rejection (Section 2.2): keep[perm[i]] = 1 if the stretch of
// stored event i's LOR within half_width mm of its TOF centre (cut by the
// grid box) has a piece of positive length in a voxel whose mask byte is
// non-zero, else 0.  One problem: the whole grid (its k_sigma at least
// half_width).
template <bool PACKED>
__global__ void __launch_bounds__(256) k_tof_keep(const Problem *__restrict__ probs, float half_width,
                                                  const uint8_t *__restrict__ mask,
                                                  const int64_t *__restrict__ perm, uint8_t *__restrict__ keep) {
    const Problem &P = probs[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n_events) return;
    uint32_t k = 0;
    Ray r;
    if (make_ray<PACKED>(P, i, r)) {
        const float ta = fmaxf(r.t0, -half_width), tb = fminf(r.t1, half_width);
        if (ta < tb) {
            // the voxel walk of the projectors, stopping at the first body piece
            Stepper s(P, r, ta, grid_box(P));
            float t = ta;
            for (int step = 0; step < s.max_steps; ++step) {
                const float tmin = s.next();
                const float tn = __builtin_amdgcn_fmed3f(tmin, t, tb);
                if (tn > t && mask[s.j]) {
                    k = 1;
                    break;
                }
                t = tn;
                if (tmin >= tb) break;
                s.advance(r, tmin);
            }
        }
    }
    keep[perm[i]] = (uint8_t)k;
}

}  // namespace

int64_t project_chunk_events(int block, int ept) { return (int64_t)block * ept; }

int64_t brick_item_tab_words(int64_t n_chunks) { return n_chunks * kTabWords; }

hipError_t launch_block_image(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_xblk) {
    void *args[] = {&d_probs, &n_probs};
    return do_launch(L, reinterpret_cast<const void *>(&k_block_image), dim3((unsigned)((n_xblk + 3) / 4)),
                     dim3(256), 0, args);
}

hipError_t launch_forward(const Launch &L, bool tof, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept,
                          int mode, int *part_neff, double *part_ll) {
    void *args[] = {&d_probs, &n_probs, &ept, &mode, &part_neff, &part_ll};
    const void *fn = tof ? reinterpret_cast<const void *>(&k_forward<true>)
                         : reinterpret_cast<const void *>(&k_forward<false>);
    return do_launch(L, fn, dim3((unsigned)n_chunks), dim3(kForwardBlock), 0, args);
}

hipError_t launch_forward_items(const Launch &L, bool tof, const Problem *d_probs, int n_probs, const uint4 *chunks,
                                uint32_t n_chunks, const uint4 *bricks) {
    void *args[] = {&d_probs, &n_probs, &chunks, &bricks};
    const void *fn = tof ? reinterpret_cast<const void *>(&k_forward_items<true>)
                         : reinterpret_cast<const void *>(&k_forward_items<false>);
    return do_launch(L, fn, dim3(n_chunks), dim3(kBackBlock), 0, args);
}

hipError_t launch_combine(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept, int mode,
                          int *part_neff, double *part_ll) {
    const int64_t events = (int64_t)kForwardBlock * ept;
    if (events > (int64_t)kCombineEventsPerThread * kCombineBlock) return hipErrorInvalidValue;
    void *args[] = {&d_probs, &n_probs, &ept, &mode, &part_neff, &part_ll};
    const void *fn = events <= kCombineBlock       ? reinterpret_cast<const void *>(&k_combine<1>)
                     : events <= 2 * kCombineBlock ? reinterpret_cast<const void *>(&k_combine<2>)
                                                   : reinterpret_cast<const void *>(&k_combine<kCombineEventsPerThread>);
    return do_launch(L, fn, dim3((unsigned)n_chunks), dim3(kCombineBlock), 0, args);
}

hipError_t launch_back_chunks(const Launch &L, bool tof, const Problem *d_probs, int n_probs, const uint4 *chunks,
                              uint32_t n_chunks, const uint4 *bricks) {
    void *args[] = {&d_probs, &n_probs, &chunks, &bricks};
    const void *fn = tof ? reinterpret_cast<const void *>(&k_back_chunks<true>)
                         : reinterpret_cast<const void *>(&k_back_chunks<false>);
    return do_launch(L, fn, dim3(n_chunks), dim3(kBackBlock), 0, args);
}

hipError_t launch_clear_bwmax(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_bricks) {
    void *args[] = {&d_probs, &n_probs, &n_bricks};
    return do_launch(L, reinterpret_cast<const void *>(&k_clear_bwmax), dim3((unsigned)((n_bricks + 255) / 256)),
                     dim3(256), 0, args);
}

hipError_t launch_brick_wmax(const Launch &L, const Problem *d_probs, int n_probs, const uint4 *chunks,
                             uint32_t n_chunks, const uint4 *bricks) {
    void *args[] = {&d_probs, &n_probs, &chunks, &bricks};
    return do_launch(L, reinterpret_cast<const void *>(&k_brick_wmax), dim3(n_chunks), dim3(256), 0, args);
}

hipError_t launch_reduce_tiles(const Launch &L, const Problem *d_probs, int n_probs, const uint4 *bricks,
                               uint32_t n_bricks) {
    void *args[] = {&d_probs, &n_probs, &bricks};
    return do_launch(L, reinterpret_cast<const void *>(&k_reduce_tiles), dim3(4 * n_bricks), dim3(256), 0, args);
}

hipError_t launch_brick_items(const Launch &L, const Problem *d_probs, int n_probs, int64_t n_chunks, int ept,
                              uint32_t *ctr, const uint32_t *end, int fill, uint32_t *tabs) {
    void *args[] = {&d_probs, &n_probs, &ept, &ctr, &end, &fill, &tabs};
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

hipError_t launch_tof_keep(const Launch &L, const Problem *d_probs, bool packed, int64_t n_events, float half_width,
                          const uint8_t *mask, const int64_t *perm, uint8_t *keep) {
    void *args[] = {&d_probs, &half_width, &mask, &perm, &keep};
    const void *fn = packed ? reinterpret_cast<const void *>(&k_tof_keep<true>)
                            : reinterpret_cast<const void *>(&k_tof_keep<false>);
    return do_launch(L, fn, dim3((unsigned)((n_events + 255) / 256)), dim3(256), 0, args);
}

}  // namespace lmtof

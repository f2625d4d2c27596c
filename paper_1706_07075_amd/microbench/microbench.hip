// Hardware ceilings of one MI355X (gfx950) that the projector kernels are
// judged against: HBM streaming, random 4-byte gathers, device-scope global
// atomics, LDS atomics and reads, and the vector ALU's FMA rate.  Built as
// its own library (libmicrobench.so), separate from liblmtof.so; bench.py
// --microbench runs it.  Each probe times `reps` launches with HIP events
// on the null stream and reports one rate.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_copy(const float4 *__restrict__ a, float4 *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void __launch_bounds__(kBlock) k_read(const float4 *__restrict__ a, int64_t n, float *__restrict__ out) {
    float s = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == 12345.678f) out[0] = s;  // keeps the loads; never true for the data used
}

// SplitMix64 step: a counter-based index stream (no table).
__device__ __forceinline__ uint64_t mix(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Each lane gathers `per_lane` 4-byte values at random indices in [0, mask].
__global__ void __launch_bounds__(kBlock) k_gather(const float *__restrict__ t, uint32_t mask, int per_lane,
                                                   float *__restrict__ out) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.0f;
    uint64_t z = id * 0x2545f4914f6cdd1dull;
    for (int k = 0; k < per_lane; k += 4) {
        const uint64_t r0 = mix(z), r1 = mix(z + 1);
        z += 2;
        s += t[(uint32_t)r0 & mask] + t[(uint32_t)(r0 >> 32) & mask] + t[(uint32_t)r1 & mask] +
             t[(uint32_t)(r1 >> 32) & mask];
    }
    if (s == 12345.678f) out[id] = s;
}

// Device-scope FP32 atomic adds (no return) at random indices in [0, mask].
__global__ void __launch_bounds__(kBlock) k_atomic_f32(float *__restrict__ t, uint32_t mask, int per_lane) {
    const uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t z = id * 0x2545f4914f6cdd1dull;
    for (int k = 0; k < per_lane; k += 2) {
        const uint64_t r = mix(z++);
        atomicAdd(t + ((uint32_t)r & mask), 1.0f);
        atomicAdd(t + ((uint32_t)(r >> 32) & mask), 1.0f);
    }
}

// LDS: random adds (FP32 or 64-bit integer) or reads over a 32 KiB table.
template <int MODE>  // 0: ds_add_f32, 1: ds_add_u64, 2: ds_read_b32
__global__ void __launch_bounds__(1024) k_lds(int per_lane, float *__restrict__ out) {
    __shared__ unsigned long long tab[4096];
    for (int k = threadIdx.x; k < 4096; k += blockDim.x) tab[k] = 0;
    __syncthreads();
    uint64_t z = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 0x2545f4914f6cdd1dull;
    float s = 0.0f;
    for (int k = 0; k < per_lane; k += 2) {
        const uint64_t r = mix(z++);
        const uint32_t a = (uint32_t)r & 4095u, b = (uint32_t)(r >> 32) & 4095u;
        if (MODE == 0) {
            atomicAdd(reinterpret_cast<float *>(tab) + 2 * a, 1.0f);
            atomicAdd(reinterpret_cast<float *>(tab) + 2 * b, 1.0f);
        } else if (MODE == 1) {
            atomicAdd(tab + a, 1ull);
            atomicAdd(tab + b, 1ull);
        } else {
            s += reinterpret_cast<const float *>(tab)[2 * a] + reinterpret_cast<const float *>(tab)[2 * b];
        }
    }
    __syncthreads();
    if (MODE == 2 && s == 12345.678f) out[0] = s;
    if (MODE != 2 && threadIdx.x == 0) out[blockIdx.x] = reinterpret_cast<float *>(tab)[0];
}

// Independent FMA chains: 8 per lane, `iters` rounds of 8 FMAs.
__global__ void __launch_bounds__(kBlock) k_fma(int iters, float *__restrict__ out) {
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
    const float m = 0.999f, c = 1e-4f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    if (s == 12345.678f) out[0] = s;
}

template <class F>
int timed(int reps, float *ms, F &&launch) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    launch();  // warm-up
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, nullptr);
    int rc = hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess ? 0 : -1;
    float t = 0.0f;
    if (!rc) rc = hipEventElapsedTime(&t, e0, e1) == hipSuccess ? 0 : -1;
    *ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" {

// Probe `which` on the current device; *rate receives the result:
//   0 HBM copy of `bytes` (read + write bytes / s); 1 HBM read of `bytes`;
//   2 random 4-byte gathers from a table of `bytes` (gathers / s);
//   3 device-scope FP32 atomic adds, random over `bytes` (adds / s);
//   4 LDS ds_add_f32, 5 LDS 64-bit integer add, 6 LDS 4-byte reads, random
//     over 32 KiB per workgroup (operations / s);
//   7 vector FP32 FMA (lane FMAs / s).
// Returns 0, or -1 on an allocation or runtime error.
int mb_run(int which, int64_t bytes, int reps, double *rate) {
    *rate = 0.0;
    // the table size must be a power of two in [4 KiB, 8 GiB] (the random
    // probes mask their indices with it)
    if (which < 0 || which > 7 || reps < 1 || bytes < 4096 || bytes > (int64_t(1) << 33) || (bytes & (bytes - 1)))
        return -1;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    const int grid = ncu * 32;
    float ms = 0.0f;
    int rc = 0;
    if (which <= 3) {
        const int64_t n4 = bytes / 16;
        float4 *a = nullptr, *b = nullptr;
        float *o = nullptr;
        if (hipMalloc((void **)&a, n4 * 16) != hipSuccess || hipMalloc((void **)&o, sizeof(float) * grid * kBlock) != hipSuccess)
            return -1;
        if (which == 0 && hipMalloc((void **)&b, n4 * 16) != hipSuccess) return -1;
        if (hipMemset(a, 0, n4 * 16) != hipSuccess) return -1;
        const uint32_t mask = (uint32_t)((bytes / 4) - 1);  // bytes: a power of two
        const int per_lane = 64;
        if (which == 0) {
            rc = timed(reps, &ms, [&] { hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, nullptr, a, b, n4); });
            *rate = 2.0 * (double)(n4 * 16) / (ms * 1e-3);
        } else if (which == 1) {
            rc = timed(reps, &ms, [&] { hipLaunchKernelGGL(k_read, dim3(grid), dim3(kBlock), 0, nullptr, a, n4, o); });
            *rate = (double)(n4 * 16) / (ms * 1e-3);
        } else if (which == 2) {
            rc = timed(reps, &ms, [&] {
                hipLaunchKernelGGL(k_gather, dim3(grid), dim3(kBlock), 0, nullptr, (const float *)a, mask, per_lane, o);
            });
            *rate = (double)grid * kBlock * per_lane / (ms * 1e-3);
        } else {
            rc = timed(reps, &ms, [&] {
                hipLaunchKernelGGL(k_atomic_f32, dim3(grid), dim3(kBlock), 0, nullptr, (float *)a, mask, per_lane);
            });
            *rate = (double)grid * kBlock * per_lane / (ms * 1e-3);
        }
        (void)hipFree(a);
        if (b) (void)hipFree(b);
        (void)hipFree(o);
    } else if (which <= 6) {
        float *o = nullptr;
        const int g2 = ncu * 4, per_lane = 256;
        if (hipMalloc((void **)&o, sizeof(float) * g2) != hipSuccess) return -1;
        auto go = [&](const void *fn) {
            int pl = per_lane;
            void *args[] = {&pl, &o};
            (void)hipLaunchKernel(fn, dim3(g2), dim3(1024), args, 0, nullptr);
        };
        const void *fn = which == 4 ? (const void *)&k_lds<0> : which == 5 ? (const void *)&k_lds<1> : (const void *)&k_lds<2>;
        rc = timed(reps, &ms, [&] { go(fn); });
        *rate = (double)g2 * 1024 * per_lane / (ms * 1e-3);
        (void)hipFree(o);
    } else {
        float *o = nullptr;
        const int iters = 4096;
        if (hipMalloc((void **)&o, sizeof(float)) != hipSuccess) return -1;
        rc = timed(reps, &ms, [&] { hipLaunchKernelGGL(k_fma, dim3(grid), dim3(kBlock), 0, nullptr, iters, o); });
        *rate = (double)grid * kBlock * iters * 8 / (ms * 1e-3);
        (void)hipFree(o);
    }
    return rc;
}

}  // extern "C"

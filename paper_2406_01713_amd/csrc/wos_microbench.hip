// wos_microbench.hip -- issue-rate microbenchmarks that pin the roofline
// denominator of the walk kernels on the device they run on:
//   0  FP32 fused multiply-add (v_fma_f32, not packed): FLOP/s
//   1  FP32 square root (v_sqrt_f32): operations/s
//   2  the 7-D sphere-distance loop of the walk kernels (sub, fma, sqrt,
//      sub, min per sphere, rows through scalar loads): sphere evaluations/s
#include <hip/hip_runtime.h>

#include "../../include/wos.h"
#include "wos_device.hpp"

namespace {

constexpr int kMbBlock = 256;
constexpr int kChains = 8;

__global__ void __launch_bounds__(kMbBlock) mb_fma(float* out, int iters, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (float)(threadIdx.x + c) * 1e-3f;
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * kMbBlock + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kMbBlock) mb_sqrt(float* out, int iters)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = 1.0f + (float)(threadIdx.x + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_sqrtf(x[c]);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * kMbBlock + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kMbBlock) mb_distance(const float* sph, int n, float* out, int iters)
{
    using namespace wos;
    float x[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) x[i] = 0.01f * (float)((threadIdx.x * 7 + i) & 255) - 1.0f;
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        const float m = spheres_min<float, 7>(fresh(to_const(sph)), n, x);
        acc += m;
        x[0] += 1e-6f * m;
    }
    out[blockIdx.x * kMbBlock + threadIdx.x] = acc;
}

}  // namespace

extern "C" int wos_microbench(int which, double* out_rate, double* out_ms)
{
    if (!out_rate || which < 0 || which > 2) return WOS_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return WOS_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return WOS_EHIP;
    const int blocks = cus * 8;  // 8 blocks of 4 waves per CU: 8 waves per SIMD
    float* out = nullptr;
    float* sph = nullptr;
    const int n_sph = 256;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)blocks * kMbBlock * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&sph, (size_t)n_sph * 8 * sizeof(float));
    if (e == hipSuccess) {
        float h[n_sph * 8];
        for (int j = 0; j < n_sph * 8; ++j) h[j] = (float)((j * 37) % 101) * 0.02f - 1.0f;
        for (int j = 0; j < n_sph; ++j) h[j * 8 + 7] = 0.05f + 0.001f * (float)j;
        e = hipMemcpy(sph, h, sizeof(h), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // about 20 ms per launch; 5 untimed launches bring the clocks up, then 5 timed
    const int iters = which == 2 ? 1024 : 131072;
    const int warm = 5, timed = 5;
    double work = 0.0;
    for (int rep = 0; rep < warm + timed && e == hipSuccess; ++rep) {
        if (rep == warm) e = hipEventRecord(e0, nullptr);
        if (which == 0)
            hipLaunchKernelGGL(mb_fma, dim3(blocks), dim3(kMbBlock), 0, nullptr, out, iters, 0.9999f, 1e-4f);
        else if (which == 1)
            hipLaunchKernelGGL(mb_sqrt, dim3(blocks), dim3(kMbBlock), 0, nullptr, out, iters);
        else
            hipLaunchKernelGGL(mb_distance, dim3(blocks), dim3(kMbBlock), 0, nullptr, sph, n_sph, out, iters);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const double lanes = (double)blocks * kMbBlock;
    if (which == 0) work = timed * lanes * iters * kChains * 2.0;  // FLOP
    else if (which == 1) work = timed * lanes * iters * kChains;   // square roots
    else work = timed * lanes * iters * (double)n_sph;             // sphere evaluations
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    (void)hipFree(sph);
    if (e != hipSuccess) return WOS_EHIP;
    *out_rate = work / (ms * 1e-3);
    if (out_ms) *out_ms = ms / timed;
    return WOS_OK;
}

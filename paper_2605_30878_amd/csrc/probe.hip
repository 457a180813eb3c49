// probe.hip -- HBM reference kernels: what plain streaming kernels reach on
// this device, so that the lattice kernels' bandwidth can be read against
// the attainable rate as well as against the published peak.  Not part of
// the time step.
//
//   kind 0  read:    every 16-byte vector of `src` loaded once
//   kind 1  copy:    dst = src, 16-byte vectors
//   kind 2  planes:  dst[k] = sum of 19 FP32 planes src[i][k], one 4-byte
//                    load per lane and plane (the access pattern of the
//                    colour-field kernel: Q plane reads and one plane write)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"

namespace {

constexpr int PROBE_BX = 256;
constexpr unsigned PROBE_GRID = 256 * 16;   // grid-stride kernels: 16 workgroups per CU

__global__ __launch_bounds__(PROBE_BX) void k_probe_read(const float4* __restrict__ src, uint64_t n4,
                                                         float* __restrict__ out) {
    float acc = 0.f;
    const uint64_t stride = (uint64_t)gridDim.x * PROBE_BX;
    for (uint64_t i = (uint64_t)blockIdx.x * PROBE_BX + threadIdx.x; i < n4; i += stride) {
        const float4 v = src[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    // the sum is kept live by a store that the zero-filled input never takes
    if (acc == 1234.5f) out[blockIdx.x] = acc;
}

__global__ __launch_bounds__(PROBE_BX) void k_probe_copy(const float4* __restrict__ src, uint64_t n4,
                                                         float4* __restrict__ dst) {
    const uint64_t stride = (uint64_t)gridDim.x * PROBE_BX;
    for (uint64_t i = (uint64_t)blockIdx.x * PROBE_BX + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(PROBE_BX) void k_probe_planes(const float* __restrict__ src, uint64_t n,
                                                           float* __restrict__ dst) {
    const uint64_t k = (uint64_t)blockIdx.x * PROBE_BX + threadIdx.x;
    if (k >= n) return;
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 19; i++) acc += src[(uint64_t)i * n + k];
    dst[k] = acc;
}

}  // namespace

extern "C" int lbm_hbm_probe(int32_t kind, const void* src, void* dst, size_t src_bytes, int32_t repeats,
                             void* hip_stream, double* ms_out) {
    if (!src || !dst || !ms_out || repeats < 1 || kind < 0 || kind > 2) return LBM_EINVAL;
    if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return LBM_EINVAL;
    const uint64_t unit = kind == 2 ? 19 * sizeof(float) : sizeof(float4);
    if (src_bytes < unit || src_bytes % unit) return LBM_EINVAL;
    const uint64_t n = src_bytes / unit;   // float4 vectors (kinds 0, 1) or plane length (kind 2)
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return LBM_EHIP;
    }
    hipError_t err = hipEventRecord(e0, s);
    for (int r = 0; r < repeats && err == hipSuccess; r++) {
        if (kind == 0)
            k_probe_read<<<PROBE_GRID, PROBE_BX, 0, s>>>((const float4*)src, n, (float*)dst);
        else if (kind == 1)
            k_probe_copy<<<PROBE_GRID, PROBE_BX, 0, s>>>((const float4*)src, n, (float4*)dst);
        else
            k_probe_planes<<<(unsigned)((n + PROBE_BX - 1) / PROBE_BX), PROBE_BX, 0, s>>>((const float*)src, n,
                                                                                          (float*)dst);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return LBM_EHIP;
    *ms_out = (double)ms / repeats;
    return LBM_OK;
}

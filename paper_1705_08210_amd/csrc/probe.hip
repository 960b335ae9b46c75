// probe.hip -- the shader clock the GPU holds under a full vector-ALU load, a
// measurement aid for the benchmark: kernel durations are compared across
// machines that run at different clocks under load.
#include "ps_internal.h"

namespace ps {

constexpr int kProbeBlocks = 2048;   // 8 workgroups per CU on 256 CUs: all resident
constexpr int kProbeChains = 8;      // independent min/add chains per lane

// Every lane runs `iters` rounds of min + add on kProbeChains independent
// chains (the instruction mix of the FP32 tile kernels).  The first lane of
// each workgroup reads the shader-clock counter (s_memtime) and the
// constant-rate 100 MHz counter (s_memrealtime) before and after.
__global__ __launch_bounds__(256) void ps_clock_probe_kernel(int64_t iters, float seed,
                                                             unsigned long long* out) {
    float a[kProbeChains], b[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
        a[c] = seed * (float)(threadIdx.x + c);
        b[c] = seed + (float)c;
    }
    __syncthreads();
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    for (int64_t k = 0; k < iters; ++k) {
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) a[c] = __builtin_fminf(a[c], b[c]) + b[c];
    }
    __syncthreads();
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) acc += a[c];
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = c1 - c0;
        out[3 * blockIdx.x + 1] = r1 - r0;
        out[3 * blockIdx.x + 2] = acc == -1.0f;   // keeps the chains live
    }
}

}  // namespace ps

using namespace ps;

extern "C" {

size_t ps_clock_probe_workspace_size(void) {
    return (size_t)kProbeBlocks * 3 * sizeof(unsigned long long);
}

ps_status ps_clock_probe(int64_t iters, void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (iters < 1) return fail(PS_ERR_ARG, "iters = %lld must be >= 1", (long long)iters);
    if (!workspace || ws_bytes < ps_clock_probe_workspace_size())
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes,
                    ps_clock_probe_workspace_size());
    if ((uintptr_t)workspace % 8) return fail(PS_ERR_ARG, "workspace is not 8-byte aligned");
    hipLaunchKernelGGL(ps_clock_probe_kernel, dim3(kProbeBlocks), dim3(256), 0, stream, iters,
                       0.5f, (unsigned long long*)workspace);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? PS_OK : fail(PS_ERR_HIP, "clock probe launch: %s",
                                          hipGetErrorString(e));
}

}  // extern "C"

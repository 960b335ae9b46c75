// reduce.hip -- on-GPU reduction of metric output before it leaves the device
// (the output handling of Section 6.5): one unsigned byte per metric, and
// thresholding into an index-ordered list of (index, value) pairs.  Both are
// HBM-bound passes over the c2 / c3 arrays.
#include "ps_internal.h"

namespace ps {

// ---------------------------------------------------------------------------
// One byte per metric: q = round-to-nearest-even(255 c), c clamped to [0, 1]
// (a single FP32 multiply and rint, so any reader can reproduce it).
// Four values per thread: one 16-byte load, one 4-byte store.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t q8(float c) {
    const float x = __builtin_rintf(__builtin_fminf(__builtin_fmaxf(c, 0.0f), 1.0f) * 255.0f);
    return (uint32_t)x;
}

__global__ __launch_bounds__(256) void ps_quantize_u8_kernel(const float* c, int64_t n,
                                                             uint8_t* q) {
    const bool vec = ((uintptr_t)c % 16 == 0) && ((uintptr_t)q % 4 == 0);
    const int64_t nq = (n + 3) / 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nq;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = 4 * t;
        if (vec && i + 4 <= n) {
            const float4 v = *(const float4*)(c + i);
            *(uint32_t*)(q + i) = q8(v.x) | (q8(v.y) << 8) | (q8(v.z) << 16) | (q8(v.w) << 24);
        } else {
            for (int64_t e = i; e < n && e < i + 4; ++e) q[e] = (uint8_t)q8(c[e]);
        }
    }
}

hipError_t launch_quantize_u8(const float* c, int64_t n, uint8_t* q, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = ((n + 3) / 4 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ps_quantize_u8_kernel, dim3((unsigned)blocks), dim3(256), 0, st, c, n, q);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Thresholding: the entries with c >= thr, in index order.  Three passes over
// tiles of kSelTile entries (256 threads x 16 consecutive entries each):
//   count  selected entries per tile;
//   scan   exclusive offsets of the tiles (one workgroup) and the total;
//   write  each thread writes its selected entries at tile offset + the
//          exclusive prefix of the thread counts before it.
// Deterministic, and the list is sorted by index.
// ---------------------------------------------------------------------------
constexpr int kSelPer = 16;
constexpr int kSelTile = 256 * kSelPer;

int64_t select_tiles(int64_t n) { return ceil_div(n, kSelTile); }

__device__ __forceinline__ int thread_count(const float* c, int64_t n, int64_t i0, float thr) {
    int k = 0;
    for (int e = 0; e < kSelPer; ++e) {
        const int64_t i = i0 + e;
        if (i < n && c[i] >= thr) ++k;
    }
    return k;
}

// Exclusive prefix of v over the 256 threads of the workgroup; the total in *tot.
__device__ __forceinline__ int block_exclusive(int v, int* sh, int* tot) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d *= 2) {   // Hillis-Steele inclusive scan
        const int add = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int incl = sh[threadIdx.x];
    *tot = sh[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void ps_select_count_kernel(const float* c, int64_t n,
                                                              float thr, int32_t* counts) {
    __shared__ int sh[256];
    const int64_t i0 = (int64_t)blockIdx.x * kSelTile + (int64_t)threadIdx.x * kSelPer;
    int tot;
    block_exclusive(thread_count(c, n, i0, thr), sh, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// One workgroup: exclusive offsets of ntiles counts, total into *count.
__global__ __launch_bounds__(1024) void ps_select_scan_kernel(const int32_t* counts,
                                                              int64_t ntiles, int64_t* offsets,
                                                              int64_t* count) {
    __shared__ int64_t part[1024];
    const int64_t per = (ntiles + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < ntiles ? lo + per : ntiles;
    int64_t sum = 0;
    for (int64_t t = lo; t < hi; ++t) sum += counts[t];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {   // 1024 partial sums: a serial scan is plenty
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        *count = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t t = lo; t < hi; ++t) {
        offsets[t] = run;
        run += counts[t];
    }
}

__global__ __launch_bounds__(256) void ps_select_write_kernel(const float* c, int64_t n,
                                                              float thr, int64_t base,
                                                              const int64_t* offsets,
                                                              int64_t* idx, float* val,
                                                              int64_t cap) {
    __shared__ int sh[256];
    const int64_t i0 = (int64_t)blockIdx.x * kSelTile + (int64_t)threadIdx.x * kSelPer;
    int tot;
    int64_t o = offsets[blockIdx.x] +
                block_exclusive(thread_count(c, n, i0, thr), sh, &tot);
    for (int e = 0; e < kSelPer; ++e) {
        const int64_t i = i0 + e;
        if (i < n && c[i] >= thr) {
            if (o < cap) {
                idx[o] = base + i;
                val[o] = c[i];
            }
            ++o;
        }
    }
}

hipError_t launch_select(const float* c, int64_t n, float thr, int64_t base, int64_t* idx,
                         float* val, int64_t cap, int64_t* count, int32_t* counts,
                         int64_t* offsets, hipStream_t st) {
    const int64_t T = select_tiles(n);
    if (T == 0) {   // nothing to select: the count is 0 (a kernel, not a memset)
        hipLaunchKernelGGL(ps_select_scan_kernel, dim3(1), dim3(1024), 0, st, counts,
                           (int64_t)0, offsets, count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(ps_select_count_kernel, dim3((unsigned)T), dim3(256), 0, st, c, n, thr,
                       counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ps_select_scan_kernel, dim3(1), dim3(1024), 0, st, counts, T, offsets,
                       count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(ps_select_write_kernel, dim3((unsigned)T), dim3(256), 0, st, c, n, thr,
                       base, offsets, idx, val, cap);
    return hipGetLastError();
}

}  // namespace ps

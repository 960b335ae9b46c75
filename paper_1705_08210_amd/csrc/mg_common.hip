// mg_common.hip -- per-vector sums, the 3-way tile prefix, and small fill
// kernels shared by the entry points.
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "mgemm_core.h"

namespace ps {

// ---------------------------------------------------------------------------
// Per-vector sums s_i = sum_q v_{i,q} in FP64 (exact integers for PS_U8),
// plus the count of entries outside the domain v >= 0 (negative, NaN, Inf).
// One wave per vector; 16-byte coalesced loads along the fields.
// ---------------------------------------------------------------------------
template <int DT>
__device__ __forceinline__ void sum_word(uint32_t w, double& acc, uint64_t& iacc, int& bad) {
    if constexpr (DT == PS_F32) {
        acc += (double)as_f32(w);
        bad += ((w & 0x7f800000u) == 0x7f800000u) | ((w >> 31) & (w != 0x80000000u));
    } else if constexpr (DT == PS_F16) {
        const h2_t h = as_h2(w);
        acc += (double)(float)h.x;
        acc += (double)(float)h.y;
        const uint32_t lo = w & 0xffffu, hi = w >> 16;
        bad += ((lo & 0x7c00u) == 0x7c00u) | ((lo >> 15) & (lo != 0x8000u));
        bad += ((hi & 0x7c00u) == 0x7c00u) | ((hi >> 15) & (hi != 0x8000u));
    } else {
        iacc += (w & 0xffu) + ((w >> 8) & 0xffu) + ((w >> 16) & 0xffu) + (w >> 24);
    }
}

// One FP64 element: its value and whether it is outside v >= 0 (negative
// other than -0, NaN or Inf).
__device__ __forceinline__ void sum_f64(uint64_t x, double& acc, int& bad) {
    acc += __builtin_bit_cast(double, x);
    bad += ((x & 0x7ff0000000000000ull) == 0x7ff0000000000000ull) |
           (int)((x >> 63) & (x != 0x8000000000000000ull));
}

template <int DT>
__device__ __forceinline__ void sum_row(const char* row, int64_t n_f, bool vec,
                                        double& acc, uint64_t& iacc, int& bad) {
    constexpr int ESZ = Ops<DT>::kEsz;
    const int lane = threadIdx.x % 64;
    const int64_t nbytes = n_f * ESZ;
    int64_t done = 0;
    if (vec) {
        const int64_t full = nbytes / 16 * 16;
        for (int64_t b = (int64_t)lane * 16; b < full; b += 64 * 16) {
            const uint4 v = *(const uint4*)(row + b);
            if constexpr (DT == PS_F64) {
                sum_f64(((uint64_t)v.y << 32) | v.x, acc, bad);
                sum_f64(((uint64_t)v.w << 32) | v.z, acc, bad);
            } else {
                sum_word<DT>(v.x, acc, iacc, bad);
                sum_word<DT>(v.y, acc, iacc, bad);
                sum_word<DT>(v.z, acc, iacc, bad);
                sum_word<DT>(v.w, acc, iacc, bad);
            }
        }
        done = full / ESZ;
    }
    if constexpr (DT == PS_F64) {   // whole 8-byte elements
        for (int64_t q = done + lane; q < n_f; q += 64)
            sum_f64(*(const uint64_t*)(row + 8 * q), acc, bad);
    } else {
        for (int64_t q = done + lane; q < n_f; q += 64) {
            uint32_t w;
            if (ESZ == 4) w = *(const uint32_t*)(row + 4 * q);
            else if (ESZ == 2) w = *(const unsigned short*)(row + 2 * q);
            else w = *(const unsigned char*)(row + q);
            sum_word<DT>(w, acc, iacc, bad);  // zero upper parts contribute 0
        }
    }
}

__device__ __forceinline__ void wave_reduce(double& acc, uint64_t& iacc, int& bad) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off);
        iacc += __shfl_xor(iacc, off);
        bad += __shfl_xor(bad, off);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void ps_sums_kernel(const void* V, int64_t n_f, int64_t n_v,
                                                      int64_t ld, double* s, int32_t* bad) {
    constexpr int ESZ = Ops<DT>::kEsz;
    const bool vec = ((uintptr_t)V % 16 == 0) && ((ld * ESZ) % 16 == 0);
    // one wave per vector, waves striding over the vectors (no block barrier)
    for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64; i < n_v;
         i += (int64_t)gridDim.x * 4) {
        const char* row = (const char*)V + i * ld * ESZ;
        double acc = 0.0;
        uint64_t iacc = 0;
        int nbad = 0;
        sum_row<DT>(row, n_f, vec, acc, iacc, nbad);
        wave_reduce(acc, iacc, nbad);
        if (threadIdx.x % 64 == 0) {
            s[i] = DT == PS_U8 ? (double)iacc : acc;
            if (bad && nbad) atomicAdd(bad, nbad);
        }
    }
}

// Sums for the problems of a batch that did not bring their own: blockIdx.y
// is the problem, need_s != 0 marks the ones to compute into p.s.
template <int DT>
__global__ __launch_bounds__(256) void ps_batched_sums_kernel(const DevProblem* probs) {
    const DevProblem pr = probs[blockIdx.y];
    if (!pr.need_s) return;
    constexpr int ESZ = Ops<DT>::kEsz;
    const bool vec = ((uintptr_t)pr.V % 16 == 0) && ((pr.ld * ESZ) % 16 == 0);
    for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64; i < pr.n_v;
         i += (int64_t)gridDim.x * 4) {
        const char* row = (const char*)pr.V + i * pr.ld * ESZ;
        double acc = 0.0;
        uint64_t iacc = 0;
        int nbad = 0;
        sum_row<DT>(row, pr.n_f, vec, acc, iacc, nbad);
        wave_reduce(acc, iacc, nbad);
        if (threadIdx.x % 64 == 0) ((double*)pr.s)[i] = DT == PS_U8 ? (double)iacc : acc;
    }
}

__global__ void ps_zero_i32_kernel(int32_t* p, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0;
}

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(ps_zero_i32_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)),
                       dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_sums(const void* V, int32_t dt, int64_t n_f, int64_t n_v, int64_t ld,
                       double* s, int32_t* bad, hipStream_t st) {
    if (bad) {
        hipError_t e = launch_zero_i32(bad, 1, st);
        if (e != hipSuccess) return e;
    }
    if (n_v == 0) return hipSuccess;
    // four vectors per block; large n_v strides (the dispatch size is 32-bit)
    const dim3 grid((unsigned)std::min<int64_t>((n_v + 3) / 4, 1 << 20));
    switch (dt) {
    case PS_F32: hipLaunchKernelGGL(ps_sums_kernel<PS_F32>, grid, dim3(256), 0, st, V, n_f, n_v, ld, s, bad); break;
    case PS_F16: hipLaunchKernelGGL(ps_sums_kernel<PS_F16>, grid, dim3(256), 0, st, V, n_f, n_v, ld, s, bad); break;
    case PS_U8:  hipLaunchKernelGGL(ps_sums_kernel<PS_U8>, grid, dim3(256), 0, st, V, n_f, n_v, ld, s, bad); break;
    case PS_F64: hipLaunchKernelGGL(ps_sums_kernel<PS_F64>, grid, dim3(256), 0, st, V, n_f, n_v, ld, s, bad); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batched_sums(const DevProblem* probs, int32_t n, int32_t dt, int64_t max_nv,
                               hipStream_t st) {
    if (n <= 0 || max_nv <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min<int64_t>((max_nv + 3) / 4, 1 << 16), (unsigned)n);
    switch (dt) {
    case PS_F32: hipLaunchKernelGGL(ps_batched_sums_kernel<PS_F32>, grid, dim3(256), 0, st, probs); break;
    case PS_F16: hipLaunchKernelGGL(ps_batched_sums_kernel<PS_F16>, grid, dim3(256), 0, st, probs); break;
    case PS_U8:  hipLaunchKernelGGL(ps_batched_sums_kernel<PS_U8>, grid, dim3(256), 0, st, probs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host tables to the device without a host wait: the bytes travel as kernel
// arguments (copied by the runtime at launch, or into the graph node at
// capture), and one workgroup writes them out.  kPutWords * 4 bytes per
// launch keeps the argument block well inside the kernel-argument limit.
// ---------------------------------------------------------------------------
constexpr int kPutWords = 448;
struct PutArgs {
    uint32_t* dst;
    int32_t nwords;
    int32_t pad;
    uint32_t w[kPutWords];
};

__global__ __launch_bounds__(256) void ps_put_kernel(PutArgs a) {
    for (int t = threadIdx.x; t < a.nwords; t += 256) a.dst[t] = a.w[t];
}

hipError_t launch_put(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes % 4) return hipErrorInvalidValue;
    const uint32_t* w = (const uint32_t*)src;
    const size_t nw = bytes / 4;
    for (size_t w0 = 0; w0 < nw; w0 += kPutWords) {
        PutArgs a;
        a.dst = (uint32_t*)dst + w0;
        a.nwords = (int32_t)std::min<size_t>(kPutWords, nw - w0);
        a.pad = 0;
        memcpy(a.w, w + w0, (size_t)a.nwords * 4);
        hipLaunchKernelGGL(ps_put_kernel, dim3(1), dim3(256), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Work list of a batch: position t lies in the last group whose start is
// <= t; inside the group, the tiles of the problem's upper triangle in
// column-major order, (0,0), (0,1), (1,1), (0,2), ...
__global__ __launch_bounds__(256) void ps_batch_expand_kernel(const BatchGroup* g, int32_t ng,
                                                              BatchTile* tiles, int64_t ntiles) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = ng;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) / 2;
            if (g[mid].start <= t) lo = mid; else hi = mid;
        }
        int64_t bi, bj;
        tri_decode(t - g[lo].start, bi, bj);
        tiles[t] = BatchTile{g[lo].prob, (int32_t)bi, (int32_t)bj, g[lo].chunk};
    }
}

hipError_t launch_batch_expand(const BatchGroup* groups, int32_t ngroups, BatchTile* tiles,
                               int64_t ntiles, hipStream_t st) {
    if (ntiles <= 0 || ngroups <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((ntiles + 255) / 256, 4096);
    hipLaunchKernelGGL(ps_batch_expand_kernel, dim3((unsigned)blocks), dim3(256), 0, st, groups,
                       ngroups, tiles, ntiles);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive prefix over the middle indices j in [jb, je) of the tile counts
// ceil(j / bm) * ceil((n_v - 1 - j) / bm); prefix has je - jb + 1 entries.
// One workgroup of 1024 threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void ps_prefix3_kernel(int64_t n_v, int64_t jb, int64_t je,
                                                          int bm, int mode, int ob,
                                                          int64_t* prefix) {
    __shared__ int64_t part[1024];
    const int64_t nj = je - jb;
    const int64_t per = (nj + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nj ? lo + per : nj;
    int64_t sum = 0;
    for (int64_t t = lo; t < hi; ++t) {
        sum += slab_tile_count(n_v, jb + t, bm, mode, ob);
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {  // 1024 partial sums: a serial scan is plenty
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t t = lo; t < hi; ++t) {
        prefix[t] = run;
        run += slab_tile_count(n_v, jb + t, bm, mode, ob);
    }
    if (hi == nj && lo < hi) prefix[nj] = run;
    if (nj == 0 && threadIdx.x == 0) prefix[0] = 0;
}

// 2-way finish from raw tile sums: for floating storage the FP32 sums of the
// field chunks are added in FP64 in a fixed order (the field-chunk split);
// for uint8 the single raw sum is sum |a - b| and n2 = (s_i + s_j - sum) / 2.
// Then the Section 2.1 ratio.  One thread per pair, colex order.
template <int DT>
__device__ __forceinline__ void finish_pairs(int64_t n_v, int32_t nchunks, const float* partial,
                                             const double* s, float* c2, void* n2,
                                             int64_t first, int64_t stride, int bm = 0,
                                             int64_t shard0 = 0, int64_t nshards = 1) {
    const int64_t np = n_v * (n_v - 1) / 2;
    for (int64_t idx = first; idx < np; idx += stride) {
        int64_t j = (int64_t)((1.0 + __builtin_sqrt(1.0 + 8.0 * (double)idx)) * 0.5);
        while (j * (j - 1) / 2 > idx) --j;
        while ((j + 1) * j / 2 <= idx) ++j;
        const int64_t i = idx - j * (j - 1) / 2;
        if (nshards > 1) {   // a tile shard: only the pairs of its tiles
            const int64_t bi = i / bm, bj = j / bm;
            if ((bj * (bj + 1) / 2 + bi) % nshards != shard0) continue;
        }
        double num;
        if constexpr (DT == PS_U8) {
            const uint32_t sad = ((const uint32_t*)partial)[idx];
            const int64_t v = ((int64_t)s[i] + (int64_t)s[j] - (int64_t)sad) / 2;
            num = (double)v;
            if (n2) ((int32_t*)n2)[idx] = (int32_t)v;
        } else {
            num = 0.0;
            for (int c = 0; c < nchunks; ++c) num += (double)partial[c * np + idx];
            if (n2) ((float*)n2)[idx] = (float)num;
        }
        if (c2) {
            const double d = s[i] + s[j];
            c2[idx] = d > 0.0 ? (float)((2.0 * num) / d) : 0.0f;
        }
    }
}

__global__ __launch_bounds__(256) void ps_finish2_kernel(Mg2Launch a, int bm) {
    finish_pairs<PS_F32>(a.n_v, a.nchunks, a.partial, a.s, a.c2, a.n2,
                         (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                         (int64_t)gridDim.x * blockDim.x, bm, a.shard0, a.nshards);
}

// Every problem of a batch (blockIdx.y = problem).
template <int DT>
__global__ __launch_bounds__(256) void ps_finish2_batched_kernel(const DevProblem* probs) {
    const DevProblem p = probs[blockIdx.y];
    if (p.n_v < 2) return;
    finish_pairs<DT>(p.n_v, p.nchunks, p.partial, p.s, p.c2, p.n2,
                     (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                     (int64_t)gridDim.x * blockDim.x);
}

hipError_t launch_finish2_batched(int32_t dt, const DevProblem* probs, int32_t n,
                                  int64_t max_pairs, hipStream_t st) {
    if (n <= 0 || max_pairs <= 0) return hipSuccess;
    int64_t blocks = (max_pairs + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    const dim3 grid((unsigned)blocks, (unsigned)n);
    switch (dt) {
    case PS_F32: hipLaunchKernelGGL(ps_finish2_batched_kernel<PS_F32>, grid, dim3(256), 0, st, probs); break;
    case PS_F16: hipLaunchKernelGGL(ps_finish2_batched_kernel<PS_F16>, grid, dim3(256), 0, st, probs); break;
    default:     hipLaunchKernelGGL(ps_finish2_batched_kernel<PS_U8>, grid, dim3(256), 0, st, probs); break;
    }
    return hipGetLastError();
}

hipError_t launch_finish2(int32_t dt, const Mg2Launch& a, hipStream_t st) {
    (void)dt;  // the split applies to floating storage only; partials are FP32
    const int64_t np = a.n_v * (a.n_v - 1) / 2;
    if (np <= 0) return hipSuccess;
    int64_t blocks = (np + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ps_finish2_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a,
                       kValuCfgs[a.cfg].bm());
    return hipGetLastError();
}

// Exclusive prefix of the column-tile counts of the flattened (colex) or the
// lex-ordered row tiles of a stage part, one workgroup per part (blockIdx.x):
// 1024 threads each own a contiguous run of row tiles; the run sums are
// scanned in LDS (Hillis-Steele, ten steps) and each thread writes its run.
struct Prefix3Part {
    int64_t jb, je;
    int lex;
    int64_t* prefix;
};
__device__ __forceinline__ int64_t prefix3_cols(int64_t n_v, int64_t jb, int64_t je, int bm,
                                                bool lex, int64_t rt) {
    return lex ? lex_col_tiles(n_v, jb, je, bm, rt) : flat_col_tiles(n_v, jb, bm, rt);
}
__global__ __launch_bounds__(1024) void ps_prefix3_flat_kernel(int64_t n_v, int bm,
                                                               Prefix3Part p0,
                                                               Prefix3Part p1) {
    __shared__ int64_t part[1024];
    const Prefix3Part p = blockIdx.x == 0 ? p0 : p1;
    const bool lex = p.lex != 0;
    const int64_t nr = lex ? lex_row_tiles(n_v, p.jb, p.je, bm) : flat_row_tiles(p.jb, p.je, bm);
    const int64_t per = (nr + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nr ? lo + per : nr;
    int64_t sum = 0;
    for (int64_t t = lo; t < hi; ++t) sum += prefix3_cols(n_v, p.jb, p.je, bm, lex, t);
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - sum;   // exclusive
    for (int64_t t = lo; t < hi; ++t) {
        p.prefix[t] = run;
        run += prefix3_cols(n_v, p.jb, p.je, bm, lex, t);
    }
    if (hi == nr && lo < hi) p.prefix[nr] = run;
    if (nr == 0 && threadIdx.x == 0) p.prefix[0] = 0;
}

hipError_t launch_prefix3_flat(int64_t n_v, int64_t jb, int64_t je, int bm, int64_t* prefix,
                               hipStream_t st, bool lex) {
    const Prefix3Part p{jb, je, lex ? 1 : 0, prefix};
    hipLaunchKernelGGL(ps_prefix3_flat_kernel, dim3(1), dim3(1024), 0, st, n_v, bm, p, p);
    return hipGetLastError();
}

hipError_t launch_prefix3_split(int64_t n_v, int64_t jb, int64_t js, int64_t je, int bm,
                                int64_t* prefix0, int64_t* prefix1, hipStream_t st) {
    const Prefix3Part p0{jb, js, 0, prefix0}, p1{js, je, 1, prefix1};
    const bool has0 = js > jb, has1 = je > js;
    if (!has0 && !has1) return hipSuccess;
    if (has0 && has1)
        hipLaunchKernelGGL(ps_prefix3_flat_kernel, dim3(2), dim3(1024), 0, st, n_v, bm, p0, p1);
    else
        hipLaunchKernelGGL(ps_prefix3_flat_kernel, dim3(1), dim3(1024), 0, st, n_v, bm,
                           has0 ? p0 : p1, has0 ? p0 : p1);
    return hipGetLastError();
}

int64_t flat_tiles(int64_t n_v, int64_t jb, int64_t je, int bm) {
    int64_t t = 0;
    const int64_t nr = flat_row_tiles(jb, je, bm);
    for (int64_t rt = 0; rt < nr; ++rt) t += flat_col_tiles(n_v, jb, bm, rt);
    return t;
}

int64_t lex_tiles(int64_t n_v, int64_t jb, int64_t je, int bm) {
    int64_t t = 0;
    const int64_t nr = lex_row_tiles(n_v, jb, je, bm);
    for (int64_t rt = 0; rt < nr; ++rt) t += lex_col_tiles(n_v, jb, je, bm, rt);
    return t;
}

hipError_t launch_prefix3(int64_t n_v, int64_t jb, int64_t je, int bm, int mode, int ob,
                          int64_t* prefix, hipStream_t st) {
    hipLaunchKernelGGL(ps_prefix3_kernel, dim3(1), dim3(1024), 0, st, n_v, jb, je, bm, mode, ob,
                       prefix);
    return hipGetLastError();
}

hipError_t launch_mg3_prefix(const Mg3Launch& a, hipStream_t st) {
    const int bm = kValuCfgs[a.cfg].bm();
    if (a.mode == kSlabFlat) return launch_prefix3_flat(a.n_v, a.j_begin, a.j_end, bm, a.prefix, st);
    if (a.mode == kSlabSplit)
        return launch_prefix3_split(a.n_v, a.j_begin, a.js, a.j_end, bm, a.prefix, a.prefix1, st);
    return hipErrorInvalidValue;   // the slices run kSlabFlat or kSlabSplit only
}

}  // namespace ps

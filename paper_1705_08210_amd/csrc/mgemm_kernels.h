// mgemm_kernels.h -- the VALU kernels built on mgemm_core.h, templated on the
// storage type.  Each per-type translation unit (mg_f32.hip, mg_f16.hip,
// mg_u8.hip) includes this once and instantiates the launchers for its type.
#pragma once

#include "mgemm_core.h"

namespace ps {

template <int DT>
__device__ __forceinline__ bool rows_vec_ok(const void* V, int64_t ld) {
    return ((uintptr_t)V % 16 == 0) && ((ld * Ops<DT>::kEsz) % 16 == 0);
}

// ---------------------------------------------------------------------------
// 2-way: one workgroup per tile of the upper triangle of N2 = V^T o_min V
// (Section 3.1; tiles strictly below the diagonal are never visited, the
// symmetry reduction of Section 2.1).
// ---------------------------------------------------------------------------
// Raw pair sums of one field chunk, colex order, as 32-bit patterns.
template <int DT, int TM, int TN>
__device__ __forceinline__ void store_pairs_raw(const typename Ops<DT>::Acc (&acc)[TM][TN],
                                                int64_t row0, int64_t col0, int64_t n_v,
                                                uint32_t* dst) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int lx = lane % 8, ly = lane / 8;
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int64_t i = row0 + lane_row<TM>(wave, lx, r);
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            const int64_t j = col0 + lane_col<TN>(wave, ly, c);
            if (j >= n_v || i >= j) continue;
            dst[j * (j - 1) / 2 + i] = __builtin_bit_cast(uint32_t, acc[r][c]);
        }
    }
}

template <int DT, int TM, int BKW>
__global__ __launch_bounds__(kThreads, PS_MIN_WAVES) void ps_mg2_kernel(Mg2Launch a, int64_t ntiles,
                                                                      int64_t item0) {
    using Acc = typename Ops<DT>::Acc;
    constexpr int BM = 16 * TM;
    using Word = typename Ops<DT>::Word;
    __shared__ __attribute__((aligned(16))) Word As[BKW * (BM + 4)];
    __shared__ __attribute__((aligned(16))) Word Bs[BKW * (BM + 4)];
    // work item = (field chunk, tile), chunk-major; item0: this launch's first
    const int64_t w = item0 + xcd_remap(blockIdx.x, gridDim.x);
    if (w >= ntiles * a.nchunks) return;
    const int64_t chunk = w / ntiles;
    const int64_t t = a.nshards > 1 ? a.shard0 + (w % ntiles) * a.nshards : w % ntiles;
    int64_t bi, bj;
    tri_decode(t, bi, bj);   // column-major: measured faster here than grouped order
    const int64_t row0 = bi * BM, col0 = bj * BM;
    const int wave = threadIdx.x / 64;
    const int64_t r_lo = row0 + (wave & 1) * 8 * TM;
    const int64_t c_lo = col0 + (wave >> 1) * 8 * TM;
    const int64_t c_hi = c_lo + 8 * TM;  // exclusive
    // some (i, j) with i < j, both < n_v, in this wave's quadrant?
    const bool active = r_lo < a.n_v && c_lo < a.n_v && r_lo + 1 < c_hi;
    const int64_t ldb = a.ld * Ops<DT>::kEsz;
    const int64_t nbytes = a.n_f * Ops<DT>::kEsz;
    const int64_t kt0 = a.nchunks > 1 ? chunk * a.chunk_tiles : 0;
    const int64_t kt1 = a.nchunks > 1 ? kt0 + a.chunk_tiles : -1;
    Acc acc[TM][TM];
    run_tile<DT, TM, TM, BKW, false>((const char*)a.V, ldb, nbytes,
                                              rows_vec_ok<DT>(a.V, a.ld), row0, a.n_v,
                                              col0, a.n_v, nullptr, active, As, Bs, acc,
                                              kt0, kt1);
    if (!active) return;
    if constexpr (DT != PS_F64) {   // FP64 sums are never split over field chunks
        if (a.nchunks > 1) {
            store_pairs_raw<DT, TM, TM>(acc, row0, col0, a.n_v,
                                        (uint32_t*)a.partial + chunk * (a.n_v * (a.n_v - 1) / 2));
            return;
        }
    }
    epilogue2<DT, TM, TM>(acc, row0, col0, a.n_v, a.s, a.c2, a.n2);
}

// ---------------------------------------------------------------------------
// 3-way slices B_j = X_j^T o_min V, X_j = min(V, v_j) (Section 3.2),
// restricted to i < j < k: with j the middle index the rectangle i < j, k > j
// holds every triple once.  The tiles are the split tiling (kSlabSplit) of
// the pairs (i, j) or (j, k) against the single vectors k or i.
// ---------------------------------------------------------------------------

// 3-way, first half of the epilogue: the slice sums (n3' for the floating
// and binary types) are stored as 32-bit patterns at the triple's packed
// index; ps_c3_finish_kernel turns them into c3 in place.  Keeping Eq. 1 out
// of the tile kernel keeps its register footprint (and so its occupancy)
// that of the bare min-product.
// uint8 slices accumulate sum_q |x_q - y_q| (v_sad_u8) for the staged pair
// row x = min(v_a, v_b) against a single vector y; the slices store
// n3' = sum_q min(x_q, y_q) = (n2(a, b) + s_y - SAD) / 2 instead, from the
// pair's numerator and the single vector's sum, so the finish need not know
// which pair was staged.
__device__ __forceinline__ uint32_t u8_min_sum(uint32_t sad, int32_t n2_pair, double s_single) {
    return (uint32_t)(((int64_t)n2_pair + (int64_t)s_single - (int64_t)sad) / 2);
}

// 3-way over pair rows (kSlabFlat, and part 0 of kSlabSplit): one workgroup
// per (row tile of BM consecutive pairs (i, j) in colex order, column tile of
// BM k's from the row tile's first j + 1, field chunk).  The A operand row of
// pair (i, j) is X_j's column i, min(v_i, v_j), formed while staging; entries
// with k <= j are computed by waves that also hold wanted ones and never
// stored.  Part 1 of kSlabSplit: row tiles of lex pairs (j, k) against
// column tiles of i (store_slice_lex).
template <int DT, int TM>
__device__ __forceinline__ void store_slice_flat(const typename Ops<DT>::Acc (&acc)[TM][TM],
                                                 int64_t p0, int64_t pend, int64_t col0,
                                                 const Mg3Launch& a, uint32_t* out) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int lx = lane % 8, ly = lane / 8;
    const int64_t obase = slab_offset(a.n_v, a.j_begin);
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int64_t p = p0 + lane_row<TM>(wave, lx, r);
        if (p >= pend) continue;
        const int64_t j = pair_j(p);
        const int64_t i = p - j * (j - 1) / 2;
        // index of (i, j, k) = off(j) - off(jb) + (k - j - 1) j + i
        const int64_t base = slab_offset(a.n_v, j) - obase - (j + 1) * j + i;
        int32_t nij = 0;   // the staged pair (i, j), colex index p
        if constexpr (DT == PS_U8) nij = ((const int32_t*)a.n2)[p];
#pragma unroll
        for (int c = 0; c < TM; ++c) {
            const int64_t k = col0 + lane_col<TM>(wave, ly, c);
            if (k >= a.n_v || k <= j) continue;
            if constexpr (DT == PS_F64)
                ((double*)out)[base + k * j] = acc[r][c];
            else if constexpr (DT == PS_U8)
                out[base + k * j] = u8_min_sum(acc[r][c], nij, a.s[k]);
            else
                out[base + k * j] = __builtin_bit_cast(uint32_t, acc[r][c]);
        }
    }
}

// The lex-ordered rows of kSlabSplit: row q is the pair (j, k) (lex_pair),
// its A operand row min(v_j, v_k); columns are i from col0; entries with
// i >= j are computed by waves that also hold wanted ones and never stored.
template <int DT, int TM>
__device__ __forceinline__ void store_slice_lex(const typename Ops<DT>::Acc (&acc)[TM][TM],
                                                int64_t q0, int64_t qend, int64_t col0,
                                                const Mg3Launch& a, uint32_t* out) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int lx = lane % 8, ly = lane / 8;
    const int64_t obase = slab_offset(a.n_v, a.j_begin);
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int64_t q = q0 + lane_row<TM>(wave, lx, r);
        if (q >= qend) continue;
        int64_t j, k;
        lex_pair(a.n_v, q, j, k);
        // index of (i, j, k) = off(j) - off(jb) + (k - j - 1) j + i
        const int64_t base = slab_offset(a.n_v, j) - obase + (k - j - 1) * j;
        int32_t njk = 0;   // the staged pair (j, k)
        if constexpr (DT == PS_U8) njk = ((const int32_t*)a.n2)[k * (k - 1) / 2 + j];
#pragma unroll
        for (int c = 0; c < TM; ++c) {
            const int64_t i = col0 + lane_col<TM>(wave, ly, c);
            if (i >= j) continue;
            if constexpr (DT == PS_F64)
                ((double*)out)[base + i] = acc[r][c];
            else if constexpr (DT == PS_U8)
                out[base + i] = u8_min_sum(acc[r][c], njk, a.s[i]);
            else
                out[base + i] = __builtin_bit_cast(uint32_t, acc[r][c]);
        }
    }
}

template <int DT, int TM, int BKW>
__global__ __launch_bounds__(kThreads, PS_MIN_WAVES) void ps_mg3f_kernel(Mg3Launch a,
                                                                       int64_t item0) {
    using Acc = typename Ops<DT>::Acc;
    constexpr int BM = 16 * TM;
    using Word = typename Ops<DT>::Word;
    using SA = Stager<BM, BKW, Word>;
    __shared__ __attribute__((aligned(16))) Word As[BKW * (BM + 4)];
    __shared__ __attribute__((aligned(16))) Word Bs[BKW * (BM + 4)];
    const int64_t w = item0 + xcd_remap(blockIdx.x, gridDim.x);
    if (w >= a.ntiles * a.nchunks) return;
    const int64_t chunk = w / a.ntiles, tw = w % a.ntiles;
    // kSlabSplit: tiles past ntiles0 are the lex-ordered part's
    const bool split = a.mode == kSlabSplit;
    const bool lexp = split && tw >= a.ntiles0;
    const int64_t t = lexp ? tw - a.ntiles0 : tw;
    const int64_t je0 = split ? a.js : a.j_end;   // end of the colex part
    const int64_t* pre = lexp ? a.prefix1 : a.prefix;
    // row tile: largest rt with pre[rt] <= t
    int64_t lo = 0;
    int64_t hi = lexp ? lex_row_tiles(a.n_v, a.js, a.j_end, BM) : flat_row_tiles(a.j_begin, je0, BM);
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    const int wave = threadIdx.x / 64;
    // this wave's quadrant: rows from rq, columns [cq, cq + 8 TM); it holds a
    // wanted entry iff (colex) its smallest j is below its largest k, or
    // (lex) its smallest i is below its largest j
    int64_t r0, rend, col0;
    bool active;
    if (!lexp) {
        rend = je0 * (je0 - 1) / 2;
        r0 = a.j_begin * (a.j_begin - 1) / 2 + lo * BM;
        col0 = pair_j(r0) + 1 + (t - pre[lo]) * BM;
        const int64_t rq = r0 + (wave & 1) * 8 * TM;
        const int64_t cq = col0 + (wave >> 1) * 8 * TM;
        const int64_t kq = cq + 8 * TM - 1 < a.n_v - 1 ? cq + 8 * TM - 1 : a.n_v - 1;
        active = rq < rend && cq < a.n_v && pair_j(rq) < kq;
    } else {
        rend = lex_first(a.n_v, a.j_end);
        r0 = lex_first(a.n_v, a.js) + lo * BM;
        col0 = (t - pre[lo]) * BM;
        const int64_t rq = r0 + (wave & 1) * 8 * TM;
        const int64_t cq = col0 + (wave >> 1) * 8 * TM;
        int64_t jz, kz;
        lex_pair(a.n_v, rq + 8 * TM - 1 < rend ? rq + 8 * TM - 1 : rend - 1, jz, kz);
        active = rq < rend && cq < jz;
    }
    const int64_t ldb = a.ld * Ops<DT>::kEsz;
    const int64_t nbytes = a.n_f * Ops<DT>::kEsz;
    int64_t aoff[SA::kCh], xoff[SA::kCh];
#pragma unroll
    for (int c = 0; c < SA::kCh; ++c) {
        const int64_t r = r0 + (threadIdx.x + c * kThreads) % BM;
        if (!lexp) {
            const int64_t j = r < rend ? pair_j(r) : 0;
            aoff[c] = r < rend ? (r - j * (j - 1) / 2) * ldb : -1;
            xoff[c] = j * ldb;
        } else {
            int64_t j, k;
            lex_pair(a.n_v, r < rend ? r : rend - 1, j, k);
            aoff[c] = r < rend ? j * ldb : -1;
            xoff[c] = k * ldb;
        }
    }
    Acc acc[TM][TM];
    const int64_t kt0 = a.nchunks > 1 ? chunk * a.chunk_tiles : 0;
    const int64_t kt1 = a.nchunks > 1 ? kt0 + a.chunk_tiles : -1;
    run_tile_flat<DT, TM, TM, BKW>((const char*)a.V, ldb, nbytes, rows_vec_ok<DT>(a.V, a.ld),
                                   aoff, xoff, col0, a.n_v, active, As, Bs, acc, kt0, kt1);
    if (active) {
        uint32_t* dst = DT == PS_F64 ? (uint32_t*)a.partial   // stage doubles, never split
                        : a.nchunks > 1
                            ? (uint32_t*)a.partial +
                                  chunk * (slab_offset(a.n_v, a.j_end) - slab_offset(a.n_v, a.j_begin))
                            : (uint32_t*)a.c3;
        if (lexp)
            store_slice_lex<DT, TM>(acc, r0, rend, col0, a, dst);
        else
            store_slice_flat<DT, TM>(acc, r0, rend, col0, a, dst);
    }
}

// 3-way, second half of the epilogue (Eq. 1, Section 2.2): one workgroup per
// slice j; the triples of the slice are contiguous in the j-slab layout, with
// i fastest.  n3 = ((n2(i,j) + n2(i,k)) + n2(j,k)) - n3', d3 = (s_i + s_j) + s_k,
// c3 = (3 n3) / (2 d3) in FP64, rounded once to FP32.
// Outputs per workgroup of the finish: 256 threads x 8.  Work items are
// (slab, range of kFinishRange consecutive outputs), found through a slab
// prefix of the range counts, so every workgroup has the same work whatever
// the slab sizes.
constexpr int kFinishRange = 2048;

template <int DT>
__global__ __launch_bounds__(256) void ps_c3_finish_kernel(Mg3Launch a, int64_t nitems,
                                                           int64_t item0) {
    using N2T = typename std::conditional<
        DT == PS_U8 || DT == PS_B1, int32_t,
        typename std::conditional<DT == PS_F64, double, float>::type>::type;
    const int64_t b = item0 + blockIdx.x;
    if (b >= nitems) return;
    int64_t lo = 0, hi = a.j_end - a.j_begin;   // slab holding range b (see ps_mg3_kernel)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (a.prefix[mid] <= b) lo = mid; else hi = mid;
    }
    const int64_t j = a.j_begin + lo;
    const N2T* N2 = (const N2T*)a.n2;
    const int64_t n_v = a.n_v;
    const int64_t base = slab_offset(n_v, j) - slab_offset(n_v, a.j_begin);
    const int64_t cnt = (n_v - 1 - j) * j;
    const double sj = a.s[j];
    const int64_t nj = j * (j - 1) / 2;
    uint32_t* io = (uint32_t*)a.c3;
    const int64_t stage = slab_offset(n_v, a.j_end) - slab_offset(n_v, a.j_begin);
    const int64_t t0 = (b - a.prefix[lo]) * kFinishRange;
    const bool small = cnt <= 0xffffffffLL;   // 32-bit division suffices
#pragma unroll 4
    for (int e = 0; e < kFinishRange / 256; ++e) {
        const int64_t t = t0 + e * 256 + threadIdx.x;
        if (t >= cnt) break;
        int64_t kk, i;   // t = (k - j - 1) j + i
        if (small) {
            const uint32_t q = (uint32_t)t / (uint32_t)j;
            kk = q;
            i = (int64_t)((uint32_t)t - q * (uint32_t)j);
        } else {
            kk = t / j;
            i = t - kk * j;
        }
        const int64_t k = j + 1 + kk;
        const uint32_t raw = (a.nchunks > 1 || DT == PS_F64) ? 0u : io[base + t];
        const double nij = (double)N2[nj + i];
        const double nik = (double)N2[k * (k - 1) / 2 + i];
        const double njk = (double)N2[k * (k - 1) / 2 + j];
        const double sk = a.s[k];
        double n3p;
        if constexpr (DT == PS_U8) {
            n3p = (double)(int32_t)raw;   // the slices store n3' (u8_min_sum), never split
        } else if constexpr (DT == PS_B1) {
            n3p = (double)raw;   // popcount(v_i AND v_j AND v_k), never split
        } else if constexpr (DT == PS_F64) {
            n3p = ((const double*)a.partial)[base + t];   // FP64 raw sums, never split
        } else if (a.nchunks > 1) {  // chunks of the field split, in FP64
            n3p = 0.0;
            for (int c = 0; c < a.nchunks; ++c) n3p += (double)a.partial[c * stage + base + t];
        } else {
            n3p = (double)__builtin_bit_cast(float, raw);
        }
        const double n3 = ((nij + nik) + njk) - n3p;
        const double d3 = (a.s[i] + sj) + sk;
        io[base + t] = __builtin_bit_cast(uint32_t,
                                          d3 > 0.0 ? (float)((3.0 * n3) / (2.0 * d3)) : 0.0f);
    }
}

// The finish after the slice launches of a: its slab prefix (over output
// ranges) reuses a.prefix, which the slice launches before it on the stream
// have finished reading.
template <int DT>
hipError_t go_c3_finish(const Mg3Launch& a, hipStream_t st) {
    if (a.j_end <= a.j_begin) return hipSuccess;
    hipError_t e = launch_prefix3(a.n_v, a.j_begin, a.j_end, kFinishRange, kSlabRange, 0,
                                  a.prefix, st);
    if (e != hipSuccess) return e;
    const int64_t n = slab_tiles(a.n_v, a.j_begin, a.j_end, kFinishRange, kSlabRange, 0);
    if (n == 0) return hipSuccess;
    return launch_items(n, 256, 1, [&](unsigned grid, int64_t item0) {
        hipLaunchKernelGGL(ps_c3_finish_kernel<DT>, dim3(grid), dim3(256), 0, st, a, n, item0);
    });
}

// ---------------------------------------------------------------------------
// Batched 2-way: one launch over (problem, tile, field chunk) items of many
// problems.  The host packs the (problem, field chunk) groups onto the 8
// XCDs by cost and lists each XCD's groups longest first; an XCD's blocks
// take its list in order as slots free up (greedy longest-first within the
// XCD), and an XCD works through whole groups, so the rows a tile column
// shares stay in that XCD's L2.  A persistent loop over an atomic work
// counter measured the same schedule but needed ~70 more registers (2
// instead of 4 waves per SIMD).
// ---------------------------------------------------------------------------
template <int DT, int TM, int BKW>
__global__ __launch_bounds__(kThreads, PS_MIN_WAVES) void ps_mgb_kernel(MgBatchLaunch a,
                                                                      int64_t item0) {
    using Acc = typename Ops<DT>::Acc;
    constexpr int BM = 16 * TM;
    using Word = typename Ops<DT>::Word;
    __shared__ __attribute__((aligned(16))) Word As[BKW * (BM + 4)];
    __shared__ __attribute__((aligned(16))) Word Bs[BKW * (BM + 4)];
    // block b runs on XCD b % kXcds: its position b / kXcds in that XCD's list
    const int64_t b = item0 + blockIdx.x;
    const int x = (int)(b % kXcds);
    const int64_t r = b / kXcds;
    if (r >= a.xcd_len[x]) return;
    const int64_t t = a.xcd_start[x] + r;
    const int wave = threadIdx.x / 64;
    const BatchTile bt = a.tiles[t];
    const DevProblem p = a.probs[bt.prob];
    const int64_t row0 = (int64_t)bt.bi * BM, col0 = (int64_t)bt.bj * BM;
    const int64_t r_lo = row0 + (wave & 1) * 8 * TM;
    const int64_t c_lo = col0 + (wave >> 1) * 8 * TM;
    const int64_t c_hi = c_lo + 8 * TM;
    const bool active = r_lo < p.n_v && c_lo < p.n_v && r_lo + 1 < c_hi;
    const int64_t kt0 = p.nchunks > 1 ? (int64_t)bt.chunk * a.chunk_tiles : 0;
    const int64_t kt1 = p.nchunks > 1 ? kt0 + a.chunk_tiles : -1;
    Acc acc[TM][TM];
    run_tile<DT, TM, TM, BKW, false>((const char*)p.V, p.ld * Ops<DT>::kEsz,
                                     p.n_f * Ops<DT>::kEsz, rows_vec_ok<DT>(p.V, p.ld), row0,
                                     p.n_v, col0, p.n_v, nullptr, active, As, Bs, acc, kt0, kt1);
    // raw sums only: ps_finish2_batched_kernel forms n2 and c2 of every problem
    if (active)
        store_pairs_raw<DT, TM, TM>(acc, row0, col0, p.n_v,
                                    (uint32_t*)p.partial +
                                        (int64_t)bt.chunk * (p.n_v * (p.n_v - 1) / 2));
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

template <int DT, int TM, int BKW>
hipError_t go_mg2(const Mg2Launch& a, hipStream_t st) {
    const int64_t T = shard_tiles(tri_tiles(a.n_v, 16 * TM), a.shard0, a.nshards);
    if (T == 0) return hipSuccess;
    return launch_items(T * a.nchunks, kThreads, kXcds, [&](unsigned grid, int64_t item0) {
        hipLaunchKernelGGL((ps_mg2_kernel<DT, TM, BKW>), dim3(grid), dim3(kThreads), 0, st, a,
                           T, item0);
    });
}

template <int DT, int TM, int BKW>
hipError_t go_mg3(const Mg3Launch& a, hipStream_t st) {
    if (a.ntiles == 0) return hipSuccess;
    if (a.mode != kSlabFlat && a.mode != kSlabSplit) return hipErrorInvalidValue;
    return launch_items(a.ntiles * a.nchunks, kThreads, kXcds, [&](unsigned grid, int64_t item0) {
        hipLaunchKernelGGL((ps_mg3f_kernel<DT, TM, BKW>), dim3(grid), dim3(kThreads), 0, st, a,
                           item0);
    });
}

// The slice launch of a.  dispatch(cfg, go) runs go with the compiled tile
// configuration cfg.
template <int DT, class Dispatch>
hipError_t go_mg3_all(const Mg3Launch& a, Dispatch dispatch, hipStream_t st) {
    return dispatch(a.cfg, [&](auto tm, auto bkw) {
        return go_mg3<DT, decltype(tm)::value, decltype(bkw)::value>(a, st);
    });
}

template <int DT, int TM, int BKW>
hipError_t go_mgb(const MgBatchLaunch& a, hipStream_t st) {
    if (a.ntiles == 0) return hipSuccess;
    int64_t longest = 0;
    for (int x = 0; x < kXcds; ++x) longest = a.xcd_len[x] > longest ? a.xcd_len[x] : longest;
    return launch_items(kXcds * longest, kThreads, kXcds, [&](unsigned grid, int64_t item0) {
        hipLaunchKernelGGL((ps_mgb_kernel<DT, TM, BKW>), dim3(grid), dim3(kThreads), 0, st, a,
                           item0);
    });
}

}  // namespace ps

// mgemm_core.h -- device core of the VALU min-product ("modified GEMM",
// Section 3.1 of the paper) kernels: one workgroup computes one output tile
//   acc[r][c] = sum_q op(A[row r, q], B[col c, q])
// where both operands are vectors of V (field-contiguous rows) and
//   PS_F32: op = min,                      FP32 accumulation
//   PS_F16: op = packed FP16 min, summed by a dot product with (1, 1) into FP32
//   PS_U8 : op = |a - b| summed four bytes at a time (v_sad_u8); the pair
//           numerator follows from min(a,b) = (a + b - |a-b|) / 2.
//   PS_B1 : binary fields, 32 per word; op = popcount(a AND b).
//   PS_F64: op = FP64 min, FP64 accumulation, on 64-bit words.
// For the 3-way slices (Section 3.2) the A operand is X_j = min(V, v_j),
// formed while the field tile is staged into LDS.
//
// Layout of the work: 256 threads = 2x2 waves.  Lane (lx, ly) of a wave owns
// the rows {g*32 + lx*4 + e} and columns {g*32 + ly*4 + e} (e < 4) of the
// wave's quadrant, so every LDS operand read is one 16-byte ds_read_b128.
// A wave whose quadrant holds no wanted output (below the diagonal, outside
// the tetrahedron, past n_v) skips the arithmetic but still helps stage.
#pragma once

#include "ps_internal.h"

#ifndef PS_UNROLL_PLAIN
#define PS_UNROLL_PLAIN 4
#endif
#ifndef PS_MIN_WAVES
#define PS_MIN_WAVES 2     // waves per SIMD the tile kernels are compiled for
#endif

namespace ps {

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float as_f32(uint32_t x) { return __builtin_bit_cast(float, x); }
__device__ __forceinline__ uint32_t as_u32(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ h2_t as_h2(uint32_t x) { return __builtin_bit_cast(h2_t, x); }

// ---------------------------------------------------------------------------
// Word-level arithmetic per storage type.
// ---------------------------------------------------------------------------
template <int DT> struct Ops;

template <> struct Ops<PS_F32> {
    using Acc = float;
    using Word = uint32_t;
    static constexpr int kEsz = 4;
    __device__ __forceinline__ static float step(float acc, uint32_t a, uint32_t b) {
        return acc + __builtin_fminf(as_f32(a), as_f32(b));
    }
    __device__ __forceinline__ static uint32_t xmin(uint32_t a, uint32_t b) {
        return as_u32(__builtin_fminf(as_f32(a), as_f32(b)));
    }
};

template <> struct Ops<PS_F16> {
    using Acc = float;
    using Word = uint32_t;
    static constexpr int kEsz = 2;
    __device__ __forceinline__ static float step(float acc, uint32_t a, uint32_t b) {
        const h2_t one = {(_Float16)1.0f, (_Float16)1.0f};
        return __builtin_amdgcn_fdot2(__builtin_elementwise_min(as_h2(a), as_h2(b)),
                                      one, acc, false);
    }
    __device__ __forceinline__ static uint32_t xmin(uint32_t a, uint32_t b) {
        return __builtin_bit_cast(uint32_t,
                                  __builtin_elementwise_min(as_h2(a), as_h2(b)));
    }
};

template <> struct Ops<PS_U8> {
    using Acc = uint32_t;
    using Word = uint32_t;
    static constexpr int kEsz = 1;
    __device__ __forceinline__ static uint32_t step(uint32_t acc, uint32_t a, uint32_t b) {
        return __builtin_amdgcn_sad_u8(a, b, acc);
    }
    // bytewise min through two packed 16-bit mins
    __device__ __forceinline__ static uint32_t xmin(uint32_t a, uint32_t b) {
        const uint32_t m = 0x00ff00ffu;
        u16x2_t lo = __builtin_elementwise_min(__builtin_bit_cast(u16x2_t, a & m),
                                               __builtin_bit_cast(u16x2_t, b & m));
        u16x2_t hi = __builtin_elementwise_min(__builtin_bit_cast(u16x2_t, (a >> 8) & m),
                                               __builtin_bit_cast(u16x2_t, (b >> 8) & m));
        return __builtin_bit_cast(uint32_t, lo) | (__builtin_bit_cast(uint32_t, hi) << 8);
    }
};

// Binary fields packed 32 to a word (the BITS path): min is AND, and a word
// pair contributes the population count of its AND (v_and + v_bcnt).
template <> struct Ops<PS_B1> {
    using Acc = uint32_t;
    using Word = uint32_t;
    static constexpr int kEsz = 4;   // the kernels' "element" is one packed word
    __device__ __forceinline__ static uint32_t step(uint32_t acc, uint32_t a, uint32_t b) {
        return acc + (uint32_t)__builtin_popcount(a & b);
    }
    __device__ __forceinline__ static uint32_t xmin(uint32_t a, uint32_t b) { return a & b; }
};

// FP64 data: one element per 64-bit word, FP64 min and add.
template <> struct Ops<PS_F64> {
    using Acc = double;
    using Word = uint64_t;
    static constexpr int kEsz = 8;
    __device__ __forceinline__ static double step(double acc, uint64_t a, uint64_t b) {
        return acc + __builtin_fmin(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b));
    }
    __device__ __forceinline__ static uint64_t xmin(uint64_t a, uint64_t b) {
        return __builtin_bit_cast(uint64_t, __builtin_fmin(__builtin_bit_cast(double, a),
                                                           __builtin_bit_cast(double, b)));
    }
};

// X_j staging of one 16-byte chunk: each word replaced by its min with the
// matching word of v_j.
template <int DT>
__device__ __forceinline__ uint4 xmin_chunk(uint4 v, uint4 x) {
    if constexpr (sizeof(typename Ops<DT>::Word) == 8) {
        const uint64_t lo = Ops<DT>::xmin(((uint64_t)v.y << 32) | v.x, ((uint64_t)x.y << 32) | x.x);
        const uint64_t hi = Ops<DT>::xmin(((uint64_t)v.w << 32) | v.z, ((uint64_t)x.w << 32) | x.z);
        return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    } else {
        return make_uint4(Ops<DT>::xmin(v.x, x.x), Ops<DT>::xmin(v.y, x.y),
                          Ops<DT>::xmin(v.z, x.z), Ops<DT>::xmin(v.w, x.w));
    }
}

// ---------------------------------------------------------------------------
// Staging of one field tile of BM rows into registers, then into LDS laid out
// word-major: S[w * (BM + 4) + row], words of 4 bytes (8 for FP64).  Chunks
// are 16 bytes; chunk index runs row-fastest so the transposing LDS writes of
// a wave hit distinct banks.
// ---------------------------------------------------------------------------
template <int BM, int BKW, typename Word = uint32_t>
struct Stager {
    static constexpr int kWpc = 16 / (int)sizeof(Word);  // words per chunk
    static constexpr int kCpr = BKW / kWpc;              // chunks per row
    static constexpr int kCh = BM * kCpr / kThreads;     // chunks per thread
    static constexpr int kLd = BM + 4;                   // LDS row pitch (words)
    static_assert(BM * kCpr % kThreads == 0, "tile not divisible");
    uint4 r[kCh];

    // Load the 16-byte chunk that straddles the end of the fields, element by
    // element (zero fill past the end).
    template <int ESZ>
    __device__ __forceinline__ static uint4 load_slow(const char* p, int64_t nbytes_left) {
        union {
            uint4 v;
            unsigned char b[16];
            unsigned short h[8];
            uint32_t w[4];
            uint64_t d[2];
        } u;
        u.v = make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 16 / ESZ; ++e) {
            if ((int64_t)e * ESZ < nbytes_left) {
                if (ESZ == 8) u.d[e] = *(const uint64_t*)(p + 8 * e);
                else if (ESZ == 4) u.w[e] = *(const uint32_t*)(p + 4 * e);
                else if (ESZ == 2) u.h[e] = *(const unsigned short*)(p + 2 * e);
                else u.b[e] = *(const unsigned char*)(p + e);
            }
        }
        return u.v;
    }

    // A whole 16-byte chunk of a row that is not 16-byte aligned: four
    // 32-bit loads when 4-byte aligned (always for FP32), else element loads.
    // (Two aligned 16-byte loads shifted into place measured 35% slower on
    // the batched workload: twice the bytes through the L1.)
    template <int ESZ>
    __device__ __forceinline__ static uint4 load_unaligned(const char* p) {
        if (ESZ >= 4 || (uintptr_t)p % 4 == 0) {
            const uint32_t* w = (const uint32_t*)p;
            return make_uint4(w[0], w[1], w[2], w[3]);
        }
        return load_slow<ESZ>(p, 16);
    }

    // VEC: rows are 16-byte aligned.  A compile-time choice, taken once per
    // tile loop (run_tile): with both forms in one loop the compiler merges
    // them into the 32-bit loads, which then serve aligned rows too.
    template <int ESZ, bool VEC>
    __device__ __forceinline__ static uint4 load_chunk(const char* row_base, int64_t b0,
                                                       int64_t nbytes) {
        if (b0 + 16 <= nbytes)
            return VEC ? *(const uint4*)(row_base + b0) : load_unaligned<ESZ>(row_base + b0);
        if (b0 < nbytes) return load_slow<ESZ>(row_base + b0, nbytes - b0);
        return make_uint4(0, 0, 0, 0);
    }

    // rows [row0, row0 + BM) of V, valid below row_end; field-tile byte
    // offset kb0; nbytes = n_f * element size; ldb = row pitch in bytes.
    // XJ: replace each word by min(word, word of row xrow) (X_j staging).
    template <int DT, bool XJ, bool VEC>
    __device__ __forceinline__ void load(const char* Vb, int64_t ldb, int64_t row0,
                                         int64_t row_end, int64_t kb0, int64_t nbytes,
                                         const char* xrow) {
        constexpr int ESZ = Ops<DT>::kEsz;
#pragma unroll
        for (int c = 0; c < kCh; ++c) {
            const int idx = threadIdx.x + c * kThreads;
            const int row = idx % BM;
            const int ch = idx / BM;
            const int64_t grow = row0 + row;
            const int64_t b0 = kb0 + ch * 16;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (grow < row_end) v = load_chunk<ESZ, VEC>(Vb + grow * ldb, b0, nbytes);
            if (XJ) v = xmin_chunk<DT>(v, load_chunk<ESZ, VEC>(xrow, b0, nbytes));
            r[c] = v;
        }
    }

    // Rows given per chunk (the flattened 3-way rows): roff[c] is the byte
    // offset of chunk c's row (< 0: no row, zero fill) and, with XJ, xoff[c]
    // the offset of the row v_j it is min-ed with.
    template <int DT, bool XJ, bool VEC>
    __device__ __forceinline__ void load_rows(const char* Vb, const int64_t (&roff)[kCh],
                                              const int64_t (&xoff)[kCh], int64_t kb0,
                                              int64_t nbytes) {
        constexpr int ESZ = Ops<DT>::kEsz;
#pragma unroll
        for (int c = 0; c < kCh; ++c) {
            const int ch = (threadIdx.x + c * kThreads) / BM;
            const int64_t b0 = kb0 + ch * 16;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (roff[c] >= 0) {
                v = load_chunk<ESZ, VEC>(Vb + roff[c], b0, nbytes);
                if (XJ) v = xmin_chunk<DT>(v, load_chunk<ESZ, VEC>(Vb + xoff[c], b0, nbytes));
            }
            r[c] = v;
        }
    }

    __device__ __forceinline__ void store(Word* S) const {
#pragma unroll
        for (int c = 0; c < kCh; ++c) {
            const int idx = threadIdx.x + c * kThreads;
            const int row = idx % BM;
            const int ch = idx / BM;
            Word* w = S + (ch * kWpc) * kLd + row;
            if constexpr (sizeof(Word) == 8) {
                w[0] = ((uint64_t)r[c].y << 32) | r[c].x;
                w[kLd] = ((uint64_t)r[c].w << 32) | r[c].z;
            } else {
                w[0] = r[c].x;
                w[kLd] = r[c].y;
                w[2 * kLd] = r[c].z;
                w[3 * kLd] = r[c].w;
            }
        }
    }
};

// Rows/columns of a lane's micro-tile element (r, c) relative to the tile.
template <int TM>
__device__ __forceinline__ int lane_row(int wave, int lx, int r) {
    return (wave & 1) * (8 * TM) + (r / 4) * 32 + lx * 4 + (r % 4);
}
template <int TN>
__device__ __forceinline__ int lane_col(int wave, int ly, int c) {
    return (wave >> 1) * (8 * TN) + (c / 4) * 32 + ly * 4 + (c % 4);
}

// ---------------------------------------------------------------------------
// One output tile.  acc receives the sums for the lane's micro-tile.
//   A rows [a_row0, a_row0 + BM) valid below a_end (optionally X_j-staged
//   against row xj), B rows [b_row0, b_row0 + BN) valid below b_end.
//   active: whether this wave does the arithmetic.
//   [kt0, kt1): the field tiles summed (kt1 < 0: all of them).
// ---------------------------------------------------------------------------
template <int DT, int TM, int TN, int BKW, bool XJ, bool VEC>
__device__ __forceinline__ void run_tile_body(const char* Vb, int64_t ldb, int64_t nbytes,
                                              int64_t a_row0, int64_t a_end, int64_t b_row0,
                                              int64_t b_end, const char* xrow, bool active,
                                              typename Ops<DT>::Word* As,
                                              typename Ops<DT>::Word* Bs,
                                              typename Ops<DT>::Acc (&acc)[TM][TN],
                                              int64_t kt0, int64_t kt1) {
    using Acc = typename Ops<DT>::Acc;
    using Word = typename Ops<DT>::Word;
    constexpr int BM = 16 * TM, BN = 16 * TN;
    using SA = Stager<BM, BKW, Word>;
    using SB = Stager<BN, BKW, Word>;
    constexpr int kV = (int)sizeof(Word) / 4;   // 16-byte reads per 4 consecutive words
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int lx = lane % 8, ly = lane / 8;
    const int ar = (wave & 1) * (8 * TM) + lx * 4;   // first A row of the lane
    const int bc = (wave >> 1) * (8 * TN) + ly * 4;  // first B column

#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[r][c] = Acc(0);

    const int64_t tile_bytes = (int64_t)BKW * (int64_t)sizeof(Word);
    const int64_t nk_all = (nbytes + tile_bytes - 1) / tile_bytes;
    const int64_t nk = kt1 < 0 || kt1 > nk_all ? nk_all : kt1;
    // 2-way tiles prefetch the next field tile into registers while
    // computing; the 3-way slices (which also stage v_j) load each tile just
    // before staging it and rely on the other resident workgroups to cover
    // the latency.
    constexpr bool kPrefetch = !XJ;
    SA sa;
    SB sb;
    if (kPrefetch && kt0 < nk) {
        const int64_t kb = kt0 * tile_bytes;
        sa.template load<DT, XJ, VEC>(Vb, ldb, a_row0, a_end, kb, nbytes, xrow);
        sb.template load<DT, false, VEC>(Vb, ldb, b_row0, b_end, kb, nbytes, nullptr);
    }
    for (int64_t kt = kt0; kt < nk; ++kt) {
        if (!kPrefetch) {
            const int64_t kb = kt * tile_bytes;
            sa.template load<DT, XJ, VEC>(Vb, ldb, a_row0, a_end, kb, nbytes, xrow);
            sb.template load<DT, false, VEC>(Vb, ldb, b_row0, b_end, kb, nbytes, nullptr);
        }
        __syncthreads();  // previous tile's LDS reads are done
        sa.store(As);
        sb.store(Bs);
        __syncthreads();
        if (kPrefetch && kt + 1 < nk) {  // prefetch the next field tile into registers
            const int64_t kb = (kt + 1) * tile_bytes;
            sa.template load<DT, XJ, VEC>(Vb, ldb, a_row0, a_end, kb, nbytes, xrow);
            sb.template load<DT, false, VEC>(Vb, ldb, b_row0, b_end, kb, nbytes, nullptr);
        }
        if (!active) continue;
        constexpr int kUnroll = DT == PS_U8 ? PS_UNROLL_PLAIN / 2 : PS_UNROLL_PLAIN;
#pragma unroll kUnroll
        for (int w = 0; w < BKW; ++w) {
            Word a[TM], b[TN];
#pragma unroll
            for (int g = 0; g < TM / 4; ++g)
#pragma unroll
                for (int h = 0; h < kV; ++h)
                    ((uint4*)&a[4 * g])[h] = ((const uint4*)&As[w * SA::kLd + ar + g * 32])[h];
#pragma unroll
            for (int g = 0; g < TN / 4; ++g)
#pragma unroll
                for (int h = 0; h < kV; ++h)
                    ((uint4*)&b[4 * g])[h] = ((const uint4*)&Bs[w * SB::kLd + bc + g * 32])[h];
#pragma unroll
            for (int r = 0; r < TM; ++r)
#pragma unroll
                for (int c = 0; c < TN; ++c)
                    acc[r][c] = Ops<DT>::step(acc[r][c], a[r], b[c]);
        }
    }
}

// One output tile; the row alignment picks the staging loads once for the
// whole field loop (see Stager::load_chunk).
template <int DT, int TM, int TN, int BKW, bool XJ>
__device__ __forceinline__ void run_tile(const char* Vb, int64_t ldb, int64_t nbytes,
                                         bool vec, int64_t a_row0, int64_t a_end,
                                         int64_t b_row0, int64_t b_end, const char* xrow,
                                         bool active, typename Ops<DT>::Word* As,
                                         typename Ops<DT>::Word* Bs,
                                         typename Ops<DT>::Acc (&acc)[TM][TN],
                                         int64_t kt0 = 0, int64_t kt1 = -1) {
    if (vec)
        run_tile_body<DT, TM, TN, BKW, XJ, true>(Vb, ldb, nbytes, a_row0, a_end, b_row0, b_end,
                                                 xrow, active, As, Bs, acc, kt0, kt1);
    else
        run_tile_body<DT, TM, TN, BKW, XJ, false>(Vb, ldb, nbytes, a_row0, a_end, b_row0,
                                                  b_end, xrow, active, As, Bs, acc, kt0, kt1);
}

// run_tile for the flattened 3-way slices: the A rows are given per staged
// chunk (aoff / xoff as in Stager::load_rows; X_j formed per row), the B rows
// are [b_row0, b_row0 + BN) valid below b_end.  The X_j rows of each field
// tile are loaded just before they are staged (the other resident
// workgroups cover the latency); the B rows are prefetched where registers
// allow (below).
template <int DT, int TM, int TN, int BKW, bool VEC>
__device__ __forceinline__ void run_tile_flat_body(
    const char* Vb, int64_t ldb, int64_t nbytes,
    const int64_t (&aoff)[Stager<16 * TM, BKW, typename Ops<DT>::Word>::kCh],
    const int64_t (&xoff)[Stager<16 * TM, BKW, typename Ops<DT>::Word>::kCh], int64_t b_row0,
    int64_t b_end, bool active, typename Ops<DT>::Word* As, typename Ops<DT>::Word* Bs,
    typename Ops<DT>::Acc (&acc)[TM][TN], int64_t kt0, int64_t kt1) {
    using Acc = typename Ops<DT>::Acc;
    using Word = typename Ops<DT>::Word;
    constexpr int BM = 16 * TM, BN = 16 * TN;
    using SA = Stager<BM, BKW, Word>;
    using SB = Stager<BN, BKW, Word>;
    constexpr int kV = (int)sizeof(Word) / 4;
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int lx = lane % 8, ly = lane / 8;
    const int ar = (wave & 1) * (8 * TM) + lx * 4;
    const int bc = (wave >> 1) * (8 * TN) + ly * 4;

#pragma unroll
    for (int r = 0; r < TM; ++r)
#pragma unroll
        for (int c = 0; c < TN; ++c) acc[r][c] = Acc(0);

    const int64_t tile_bytes = (int64_t)BKW * (int64_t)sizeof(Word);
    const int64_t nk_all = (nbytes + tile_bytes - 1) / tile_bytes;
    const int64_t nk = kt1 < 0 || kt1 > nk_all ? nk_all : kt1;
    // The plain B rows of the next field tile are prefetched into registers
    // while this one is consumed, for the FP32 / FP16 tiles that stage two
    // B chunks per thread (measured on sparse_4096x1024, FP32: 128 x 128
    // tiles with 16-word field tiles 26.5 -> 25.5 ms, 64 x 64 28.7 -> 28.3
    // ms; the 128 x 128 tiles with 32-word field tiles stage four, lose a
    // wave per SIMD to the extra registers and ran 28.1 -> 33.5 ms).
    constexpr bool kPrefetchB = (DT == PS_F32 || DT == PS_F16) && SB::kCh <= 2;
    SA sa;
    SB sb;
    if (kPrefetchB && kt0 < nk)
        sb.template load<DT, false, VEC>(Vb, ldb, b_row0, b_end, kt0 * tile_bytes, nbytes,
                                         nullptr);
    for (int64_t kt = kt0; kt < nk; ++kt) {
        const int64_t kb = kt * tile_bytes;
        sa.template load_rows<DT, true, VEC>(Vb, aoff, xoff, kb, nbytes);
        if (!kPrefetchB)
            sb.template load<DT, false, VEC>(Vb, ldb, b_row0, b_end, kb, nbytes, nullptr);
        __syncthreads();  // previous tile's LDS reads are done
        sa.store(As);
        sb.store(Bs);
        __syncthreads();
        if (kPrefetchB && kt + 1 < nk)
            sb.template load<DT, false, VEC>(Vb, ldb, b_row0, b_end, kb + tile_bytes, nbytes,
                                             nullptr);
        if (!active) continue;
        constexpr int kUnroll = DT == PS_U8 ? PS_UNROLL_PLAIN / 2 : PS_UNROLL_PLAIN;
#pragma unroll kUnroll
        for (int w = 0; w < BKW; ++w) {
            Word a[TM], b[TN];
#pragma unroll
            for (int g = 0; g < TM / 4; ++g)
#pragma unroll
                for (int h = 0; h < kV; ++h)
                    ((uint4*)&a[4 * g])[h] = ((const uint4*)&As[w * SA::kLd + ar + g * 32])[h];
#pragma unroll
            for (int g = 0; g < TN / 4; ++g)
#pragma unroll
                for (int h = 0; h < kV; ++h)
                    ((uint4*)&b[4 * g])[h] = ((const uint4*)&Bs[w * SB::kLd + bc + g * 32])[h];
#pragma unroll
            for (int r = 0; r < TM; ++r)
#pragma unroll
                for (int c = 0; c < TN; ++c)
                    acc[r][c] = Ops<DT>::step(acc[r][c], a[r], b[c]);
        }
    }
}

template <int DT, int TM, int TN, int BKW>
__device__ __forceinline__ void run_tile_flat(
    const char* Vb, int64_t ldb, int64_t nbytes, bool vec,
    const int64_t (&aoff)[Stager<16 * TM, BKW, typename Ops<DT>::Word>::kCh],
    const int64_t (&xoff)[Stager<16 * TM, BKW, typename Ops<DT>::Word>::kCh], int64_t b_row0,
    int64_t b_end, bool active, typename Ops<DT>::Word* As, typename Ops<DT>::Word* Bs,
    typename Ops<DT>::Acc (&acc)[TM][TN], int64_t kt0 = 0, int64_t kt1 = -1) {
    if (vec)
        run_tile_flat_body<DT, TM, TN, BKW, true>(Vb, ldb, nbytes, aoff, xoff, b_row0, b_end,
                                                  active, As, Bs, acc, kt0, kt1);
    else
        run_tile_flat_body<DT, TM, TN, BKW, false>(Vb, ldb, nbytes, aoff, xoff, b_row0, b_end,
                                                   active, As, Bs, acc, kt0, kt1);
}

// Block index -> work index so that each XCD receives one contiguous run of
// the work list (blocks are dealt to the XCDs round-robin by hardware).
// Needs gridDim.x % kXcds == 0; returns an index in [0, gridDim.x).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t grid) {
    const int64_t per = grid / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Upper-triangle tile t (column-major: (0,0), (0,1), (1,1), (0,2), ...).
__device__ __forceinline__ void tri_decode(int64_t t, int64_t& bi, int64_t& bj) {
    int64_t j = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    bj = j;
    bi = t - j * (j + 1) / 2;
}

// ---------------------------------------------------------------------------
// Epilogues.
// ---------------------------------------------------------------------------

// 2-way: c2 = 2 n2 / (s_i + s_j) in FP64 (Section 2.1), rounded once to FP32;
// optional raw numerators.  Output (i, j), i < j, at colex j(j-1)/2 + i.
template <int DT, int TM, int TN>
__device__ __forceinline__ void epilogue2(const typename Ops<DT>::Acc (&acc)[TM][TN],
                                          int64_t row0, int64_t col0, int64_t n_v,
                                          const double* __restrict__ s, float* c2,
                                          void* n2) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int lx = lane % 8, ly = lane / 8;
    double sc[TN];
#pragma unroll
    for (int c = 0; c < TN; ++c) {
        const int64_t j = col0 + lane_col<TN>(wave, ly, c);
        sc[c] = j < n_v ? s[j] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < TM; ++r) {
        const int64_t i = row0 + lane_row<TM>(wave, lx, r);
        if (i >= n_v) continue;
        const double si = s[i];
#pragma unroll
        for (int c = 0; c < TN; ++c) {
            const int64_t j = col0 + lane_col<TN>(wave, ly, c);
            if (j >= n_v || i >= j) continue;
            const int64_t idx = j * (j - 1) / 2 + i;
            double num;
            if constexpr (DT == PS_U8) {
                const int64_t v = ((int64_t)si + (int64_t)sc[c] - (int64_t)acc[r][c]) / 2;
                num = (double)v;
                if (n2) ((int32_t*)n2)[idx] = (int32_t)v;
            } else if constexpr (DT == PS_B1) {
                num = (double)acc[r][c];
                if (n2) ((int32_t*)n2)[idx] = (int32_t)acc[r][c];
            } else if constexpr (DT == PS_F64) {
                num = acc[r][c];
                if (n2) ((double*)n2)[idx] = acc[r][c];
            } else {
                num = (double)acc[r][c];
                if (n2) ((float*)n2)[idx] = acc[r][c];
            }
            if (c2) {
                const double d = si + sc[c];
                c2[idx] = d > 0.0 ? (float)((2.0 * num) / d) : 0.0f;
            }
        }
    }
}

}  // namespace ps

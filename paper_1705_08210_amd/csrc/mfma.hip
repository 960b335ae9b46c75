// mfma.hip -- 2-way numerators on the matrix cores for integer-level data.
//
// For integer values 0 <= v <= L,
//   min(a, b) = sum_{t=1..L} [a >= t] [b >= t],
// so with the 0/1 "thermometer" planes T_t = [V >= t] the pair numerators are
//   n2(i, j) = sum_t sum_q T_t[i, q] T_t[j, q],
// a dense int8 contraction over K = L * n_f, exact in int32.  This is the
// paper's min-product (Section 3.1) recast so that the matrix cores can run
// it.
//
// Two operand formats, one kernel structure:
//   int8: one plane value per byte, v_mfma_i32_32x32x32_i8, int32 sums;
//   fp4 : two plane values per byte (e2m1: 0 -> 0x0, 1 -> 0x2),
//         v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales, FP32 sums
//         (exact: every partial sum is an integer below 2^24).
// Kernels:
//   ps_thermo_expand_kernel  V (uint8, n_v x ld) -> planes P, row length
//                            L * kpad fields, kpad = n_f rounded up to whole
//                            field tiles; HBM-bound, one pass.
//   ps_mfma2_kernel          upper-triangle tiles of P P^T, FP64 epilogue
//                            (int8: operands staged through registers);
//   ps_mfma2_dma_kernel      the same with operands loaded straight into LDS
//                            (fp4);
//   ps_mfma3_kernel          3-way slices: (P_i AND P_j) P_k^T over the
//                            rectangles i < j < k, raw n3' out.
#include <type_traits>

#include "ps_internal.h"

namespace ps {

typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef int v16i_t __attribute__((ext_vector_type(16)));
typedef float v16f_t __attribute__((ext_vector_type(16)));

enum { kFmtI8 = 0, kFmtF4 = 1 };
__host__ __device__ constexpr int fields_per_byte(int fmt) { return fmt == kFmtF4 ? 2 : 1; }

constexpr int kMB = kMfmaTile;   // output tile rows and columns
constexpr int kPad = 16;      // LDS row padding: b128 reads of 32 rows spread over the banks
constexpr int kTileBytes = 128;   // plane rows are padded to whole multiples of this

// Field-tile depth in plane bytes.  A deeper tile gives each staged load
// more MFMA work to hide behind; int8 with 8 waves fits 128 bytes (two
// 147 KB LDS buffers, no spills), the fp4 and 4-wave variants run out of
// registers there and keep 64.
template <int FMT, int WN>
__host__ __device__ constexpr int mfma_mk() { return (FMT == kFmtI8 && WN == 2) ? 128 : 64; }
#ifndef PS_MFMA_GROUP
#define PS_MFMA_GROUP 4
#endif
constexpr int kGroup = PS_MFMA_GROUP;   // tile columns per L2-sharing group (grouped_tri_decode;
                                        // 4 measured 1-2% faster than 1, 2, 8, 16, 32)

// Fields of one plane row, padded to whole kTileBytes-byte field tiles
// (a multiple of every variant's tile depth; >= 1 tile).
static int64_t plane_fields(int64_t n_f, int fmt) {
    const int64_t q = (int64_t)kTileBytes * fields_per_byte(fmt);
    const int64_t kpad = (n_f + q - 1) / q * q;
    return kpad > 0 ? kpad : q;
}

int64_t mfma_row_bytes(int64_t n_f, int levels, int fmt) {
    return (int64_t)levels * (plane_fields(n_f, fmt) / fields_per_byte(fmt));
}

size_t mfma_workspace_bytes(int64_t n_f, int64_t n_v, int levels, int fmt, int wide) {
    if (mfma_fused(n_f, levels, fmt, wide)) return 0;
    return (size_t)n_v * (size_t)mfma_row_bytes(n_f, levels, fmt);
}

// ---------------------------------------------------------------------------
// Thermometer planes.  One thread per 16 fields of one vector.  For byte
// values v <= 127, (v | 0x80) - t keeps bit 7 iff v >= t and never borrows
// across bytes, so four bytes are thresholded per 32-bit operation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ge_bytes(uint32_t x, uint32_t t) {
    return (((x | 0x80808080u) - t * 0x01010101u) >> 7) & 0x01010101u;
}

// fp4 packing of four 0/1 bytes (one word of ge_bytes) into four nibbles
__device__ __forceinline__ uint32_t nibbles_e2m1(uint32_t m) {
    return ((m & 0x1u) << 1) | ((m & 0x100u) >> 3) | ((m & 0x10000u) >> 7) |
           ((m & 0x1000000u) >> 11);
}

// One thread per 32 fields of one vector; kpad is a multiple of 128.
template <int FMT>
__global__ __launch_bounds__(256) void ps_thermo_expand_kernel(const uint8_t* V, int64_t n_f,
                                                               int64_t n_v, int64_t ld,
                                                               int levels, int64_t kpad,
                                                               int8_t* P) {
    constexpr int FPB = fields_per_byte(FMT);
    const int64_t nch = kpad / 32;
    const int64_t total = n_v * nch;
    const int64_t plane_bytes = kpad / FPB;
    const bool vec = ((uintptr_t)V % 16 == 0) && (ld % 16 == 0);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / nch, ch = t % nch;
        const int64_t q0 = ch * 32;
        const uint8_t* src = V + row * ld + q0;
        union { uint4 v[2]; uint32_t w[8]; uint8_t b[32]; } u;
        if (vec && q0 + 32 <= n_f) {
            u.v[0] = *(const uint4*)src;
            u.v[1] = *(const uint4*)(src + 16);
        } else {
            u.v[0] = u.v[1] = make_uint4(0, 0, 0, 0);
            for (int e = 0; e < 32; ++e)
                if (q0 + e < n_f) u.b[e] = src[e];
        }
        int8_t* dst = P + row * (int64_t)levels * plane_bytes + q0 / FPB;
        for (int lev = 1; lev <= levels; ++lev) {
            int8_t* d = dst + (int64_t)(lev - 1) * plane_bytes;
            if constexpr (FMT == kFmtI8) {
                uint4 o0, o1;
                o0.x = ge_bytes(u.w[0], lev); o0.y = ge_bytes(u.w[1], lev);
                o0.z = ge_bytes(u.w[2], lev); o0.w = ge_bytes(u.w[3], lev);
                o1.x = ge_bytes(u.w[4], lev); o1.y = ge_bytes(u.w[5], lev);
                o1.z = ge_bytes(u.w[6], lev); o1.w = ge_bytes(u.w[7], lev);
                *(uint4*)d = o0;
                *(uint4*)(d + 16) = o1;
            } else {
                uint4 o;
                o.x = nibbles_e2m1(ge_bytes(u.w[0], lev)) | (nibbles_e2m1(ge_bytes(u.w[1], lev)) << 16);
                o.y = nibbles_e2m1(ge_bytes(u.w[2], lev)) | (nibbles_e2m1(ge_bytes(u.w[3], lev)) << 16);
                o.z = nibbles_e2m1(ge_bytes(u.w[4], lev)) | (nibbles_e2m1(ge_bytes(u.w[5], lev)) << 16);
                o.w = nibbles_e2m1(ge_bytes(u.w[6], lev)) | (nibbles_e2m1(ge_bytes(u.w[7], lev)) << 16);
                *(uint4*)d = o;
            }
        }
    }
}

struct MfmaArgs {
    const int8_t* P;
    int64_t kp;           // plane-row length in bytes (levels * kpad), multiple of the tile depth
    int64_t n_v;
    const double* s;
    float* c2;
    int32_t* n2;
    int64_t nb, ntiles;
    // 3-way
    int64_t j_begin, j_end;
    const int64_t* prefix;
    uint32_t* c3;
    int64_t item0;        // first work item of this launch
    int32_t mode, ob;     // 3-way tile set (slab_tile_count) and its outer tile edge
};

// Wave w owns j rows [(w%2)*128, +128) and i columns [(w/2)*32*WN, +32*WN)
// of the 256 x 256 tile: 4 x WN blocks of 32 x 32.  WN = 2: 8 waves, 128
// accumulator registers, 2 waves per SIMD; WN = 4: 4 waves, 256 accumulator
// registers (AGPRs), one wave per SIMD, a third less LDS traffic per MAC.
// The 128 x 128 tile (TB = 128, 3-way slab edges) halves the wave rows: 4
// waves of 2 x 2 blocks, two workgroups per CU.
template <int WN, int TB = kMB>
__host__ __device__ constexpr int mfma_threads() { return 64 * 2 * (TB / (32 * WN)); }

// Epilogue of one wave's 4 x WN blocks of 32 x 32 (Section 2.1): n2 exact,
// c2 = 2 n2 / (s_i + s_j) in FP64, rounded once to FP32, d = 0 gives 0.
template <int WN, typename AccT>
__device__ __forceinline__ void mfma_epilogue(const AccT (&acc)[4][WN], const MfmaArgs& a,
                                              int64_t i0, int64_t j0, int wr, int wc,
                                              int lane) {
    // D[row][col] of a 32x32 block: col = lane % 32, row = (r/4)*8 + (lane/32)*4 + r%4;
    // rows are j, columns are i, so 32 lanes store 32 consecutive i of one j
    const int64_t ib = i0 + wc + (lane % 32);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t j = j0 + wr + m * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
            if (j >= a.n_v) continue;
            const double sj = a.s[j];
            const int64_t base = j * (j - 1) / 2;
#pragma unroll
            for (int n = 0; n < WN; ++n) {
                const int64_t i = ib + n * 32;
                if (i >= j) continue;
                const int32_t num = (int32_t)acc[m][n][r];   // exact in either format
                if (a.n2) a.n2[base + i] = num;
                if (a.c2) {
                    const double d = a.s[i] + sj;
                    a.c2[base + i] = d > 0.0 ? (float)((2.0 * (double)num) / d) : 0.0f;
                }
            }
        }
    }
}

// Dword 3 of a raw buffer descriptor on gfx950: 32-bit data format, offset
// addressing, no swizzle (loads past num_records return zero).
constexpr int kRsrcWord3 = 0x00020000;

// Accumulator type of a format.
template <int FMT>
using mfma_acc_t = typename std::conditional<FMT == kFmtF4, v16f_t, v16i_t>::type;

// LDS of the register-staged tile: two buffers for each of the two operands.
template <int FMT, int WN, int TB = kMB>
constexpr int mfma_lds_bytes() { return 4 * TB * (mfma_mk<FMT, WN>() + kPad); }

// Main loop of one register-staged TB x TB tile: A rows a0 .. a0+TB-1 and
// B rows b0 .. b0+TB-1 of the planes (rows at or past n_v read as zero); with
// MASK every B chunk is ANDed with the same chunk of plane row `mrow` (the
// 3-way X_j operand: [v_i >= t] AND [v_j >= t] = [min(v_i, v_j) >= t]).
// Field tile kt+1 is written from registers into the second LDS buffer while
// tile kt is consumed, one barrier per field tile; tile kt+2 is loaded into
// registers meanwhile (a second register set, loading two tiles ahead, was
// measured slower on int8).  The loads are buffer loads with 32-bit offsets
// (measured 12% faster on int8 than 64-bit addresses with row tests).  Waves
// that are not `active` take part in staging and barriers only.
template <int FMT, int WN, bool MASK, int TB = kMB>
__device__ __forceinline__ void mfma_tile(const MfmaArgs& a, int64_t a0, int64_t b0,
                                          const int8_t* mrow, bool active, int wr, int wc,
                                          mfma_acc_t<FMT> (&acc)[TB / 64][WN], int8_t* lds) {
    constexpr int WM = TB / 64;                    // 32-row blocks per wave
    constexpr int kMThreads = mfma_threads<WN, TB>();
    constexpr int kMK = mfma_mk<FMT, WN>();
    constexpr int kPitch = kMK + kPad;
    constexpr int kRowChunks = kMK / 16;           // 16-byte chunks per tile row
    constexpr int kStage = TB * kRowChunks / kMThreads;   // 16-byte chunks per thread per operand
    static_assert(TB * kRowChunks % kMThreads == 0, "staging must divide evenly");
    static_assert(kMThreads % kRowChunks == 0, "a thread's chunks share one column");
    // two buffers per operand: [A0 | B0 | A1 | B1], each TB * kPitch bytes
    auto As = [&](int buf) { return lds + (2 * buf) * (TB * kPitch); };
    auto Bs = [&](int buf) { return lds + (2 * buf + 1) * (TB * kPitch); };
    const int lane = threadIdx.x % 64;

#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = (mfma_acc_t<FMT>){};

    // staging: TB rows x kMK bytes per operand, kRowChunks threads per row.
    // Buffer resources over the tile's A and B rows (the host checks that 256
    // plane rows span < 2^31 bytes): rows at or past n_v lie past num_records,
    // where buffer loads return zero without a memory access.
    auto rsrc = [&](int64_t r0) {
        const int64_t rows = r0 < a.n_v ? (a.n_v - r0 < TB ? a.n_v - r0 : TB) : 0;
        return __builtin_amdgcn_make_buffer_rsrc((void*)(a.P + (rows > 0 ? r0 : 0) * a.kp),
                                                 (short)0, (int)(rows * a.kp), kRsrcWord3);
    };
    const __amdgpu_buffer_rsrc_t rsa = rsrc(a0), rsb = rsrc(b0);
    uint4 ra[kStage], rb[kStage];
    const int ch = threadIdx.x % kRowChunks;   // the same for all of a thread's chunks
    constexpr int kRowStep = kMThreads / kRowChunks;   // rows between a thread's chunks
    const int kp = (int)a.kp;
    const int voff = (threadIdx.x / kRowChunks) * kp + ch * 16;
    auto load = [&](int64_t k0) {
        uint4 mk = make_uint4(0, 0, 0, 0);
        if constexpr (MASK) mk = *(const uint4*)(mrow + k0 + ch * 16);
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
            const int off = voff + c * kRowStep * kp + (int)k0;
            const v4u_t va = __builtin_amdgcn_raw_buffer_load_b128(rsa, off, 0, 0);
            const v4u_t vb = __builtin_amdgcn_raw_buffer_load_b128(rsb, off, 0, 0);
            ra[c] = make_uint4(va[0], va[1], va[2], va[3]);
            rb[c] = make_uint4(vb[0], vb[1], vb[2], vb[3]);
            if constexpr (MASK) {
                rb[c].x &= mk.x;
                rb[c].y &= mk.y;
                rb[c].z &= mk.z;
                rb[c].w &= mk.w;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
            const int row = (threadIdx.x + c * kMThreads) / kRowChunks;
            *(uint4*)(As(buf) + row * kPitch + ch * 16) = ra[c];
            *(uint4*)(Bs(buf) + row * kPitch + ch * 16) = rb[c];
        }
    };

    const int64_t nk = a.kp / kMK;
    // prologue: tile 0 staged, tile 1 in registers
    load(0);
    store(0);
    __syncthreads();
    if (nk > 1) load(kMK);
    const int fr = lane % 32, fk = (lane / 32) * 16;
    // One field tile kt: consume buffer cur, write tile kt+1 from the
    // registers into buffer cur^1, barrier, start loading tile kt+2.
    auto step = [&](int64_t kt, int cur) {
        const int8_t* A = As(cur);
        const int8_t* B = Bs(cur);
#pragma unroll
        for (int ks = 0; ks < kMK / 32; ++ks) {
            v4i_t fa[WM], fb[WN];
#pragma unroll
            for (int m = 0; m < WM; ++m)
                fa[m] = *(const v4i_t*)(A + (wr + m * 32 + fr) * kPitch + ks * 32 + fk);
#pragma unroll
            for (int n = 0; n < WN; ++n)
                fb[n] = *(const v4i_t*)(B + (wc + n * 32 + fr) * kPitch + ks * 32 + fk);
#pragma unroll
            for (int m = 0; m < WM; ++m)
#pragma unroll
                for (int n = 0; n < WN; ++n) {
                    if constexpr (FMT == kFmtI8) {
                        acc[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[m], fb[n],
                                                                          acc[m][n], 0, 0, 0);
                    } else {  // 64 e2m1 values per row per k-step, unit (2^0) scales
                        const v8i_t xa = {fa[m].x, fa[m].y, fa[m].z, fa[m].w, 0, 0, 0, 0};
                        const v8i_t xb = {fb[n].x, fb[n].y, fb[n].z, fb[n].w, 0, 0, 0, 0};
                        acc[m][n] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            xa, xb, acc[m][n], 4, 4, 0, 127, 0, 127);
                    }
                }
        }
        // tile kt+1 into the other buffer (after the last tile the write is
        // stale and never read; unconditional, so it joins this block)
        store(cur ^ 1);
        // schedule (measured 5% faster on int8): the next k-step's fragment
        // reads between the MFMAs of this one, the staging writes of the
        // next field tile between the MFMAs of the last k-step
        if constexpr (FMT == kFmtI8 && WN == 2 && kMK == 128) {
            constexpr int R = WM + WN, M = WM * WN, W = 2 * kStage;   // per k-step / tile
            static_assert(M >= R && W % M == 0, "schedule pattern");
            __builtin_amdgcn_sched_group_barrier(0x100, R, 0);
#pragma unroll
            for (int ks = 0; ks < kMK / 32 - 1; ++ks) {
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                if constexpr (M > R) __builtin_amdgcn_sched_group_barrier(0x008, M - R, 0);
            }
#pragma unroll
            for (int i = 0; i < M; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x200, W / M, 0);
            }
        }
        __syncthreads();   // kt+1 visible; everyone is done reading kt
        if (kt + 2 < nk) load((kt + 2) * kMK);
    };
    // Active and idle waves run separate loops with the same barriers: a
    // branch around the MFMAs inside one loop makes the compiler copy every
    // accumulator at the join on each iteration.
    if (active) {
        for (int64_t kt = 0; kt < nk; ++kt) step(kt, (int)(kt & 1));
    } else {
        for (int64_t kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) store((int)(kt & 1) ^ 1);
            __syncthreads();
            if (kt + 2 < nk) load((kt + 2) * kMK);
        }
    }
}

template <int FMT, int WN>
__global__ __launch_bounds__(mfma_threads<WN>(), 1) void ps_mfma2_kernel(MfmaArgs a) {
    __shared__ __attribute__((aligned(16))) int8_t lds[mfma_lds_bytes<FMT, WN>()];
    const int64_t t = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                      blockIdx.x / kXcds;
    if (t >= a.ntiles) return;
    int64_t bi, bj;
    grouped_tri_decode<kGroup>(t, a.nb, bi, bj);
    const int64_t i0 = bi * kMB, j0 = bj * kMB;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * 128;        // j offset of the wave's block (A rows)
    const int wc = (wave / 2) * 32 * WN;    // i offset (B rows)
    // some i < j with both < n_v among rows j0+wr.. and columns i0+wc..?
    const bool active = (i0 + wc < a.n_v) && (j0 + wr < a.n_v) && (i0 + wc + 1 < j0 + wr + 128);
    mfma_acc_t<FMT> acc[4][WN];
    mfma_tile<FMT, WN, false>(a, j0, i0, nullptr, active, wr, wc, acc, lds);
    if (!active) return;
    mfma_epilogue<WN>(acc, a, i0, j0, wr, wc, lane);
}

// ---------------------------------------------------------------------------
// 3-way slices on the matrix cores (Section 3.2 with the thermometer
// identity).  For slab j, n3'(i, j, k) = sum over plane bytes of
// (P_i AND P_j) P_k, since [a >= t][b >= t][c >= t] = [min(a, b, c) >= t].
// A work item is (slab j, tile of i, tile of k > j), enumerated through the
// slab prefix of the tile counts.  A rows are k and B rows are i, masked with
// P_j while staging, so the lane index of the MFMA output runs along i and 32
// lanes store 32 consecutive entries of the j-slab layout.  The exact integer
// n3' is stored as int32 bits; the integer 3-way finish applies Eq. 1.
// Two launches cover each slab rectangle: TB = 256 over its whole 256 x 256
// tiles, TB = 128 over the rest (two workgroups per CU, so one workgroup's
// waves that lie outside the rectangle leave their SIMD to the other's).
// ---------------------------------------------------------------------------
template <int FMT, int TB>
__global__ __launch_bounds__((mfma_threads<2, TB>()), kMB / TB) void ps_mfma3_kernel(MfmaArgs a) {
    constexpr int WN = 2, WM = TB / 64;
    __shared__ __attribute__((aligned(16))) int8_t lds[mfma_lds_bytes<FMT, WN, TB>()];
    const int64_t t = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                      blockIdx.x / kXcds;
    if (t >= a.ntiles) return;
    // slab j: largest jj with prefix[jj] <= t (the slab holding tile t; slabs
    // without tiles in this tile set repeat their prefix and are passed)
    int64_t lo = 0, hi = a.j_end - a.j_begin;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (a.prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const int64_t j = a.j_begin + lo;
    int64_t i0, k0;
    slab_tile_origin(a.n_v, j, t - a.prefix[lo], TB, a.mode, a.ob, i0, k0);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * (TB / 2);   // k offset of the wave's block (A rows)
    const int wc = (wave / 2) * 32 * WN;    // i offset (B rows)
    const bool active = (k0 + wr < a.n_v) && (i0 + wc < j);
    mfma_acc_t<FMT> acc[WM][WN];
    mfma_tile<FMT, WN, true, TB>(a, k0, i0, a.P + j * a.kp, active, wr, wc, acc, lds);
    if (!active) return;
    const int64_t base = slab_offset(a.n_v, j) - slab_offset(a.n_v, a.j_begin);
    const int64_t ib = i0 + wc + (lane % 32);
#pragma unroll
    for (int m = 0; m < WM; ++m) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t k = k0 + wr + m * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
            if (k >= a.n_v) continue;
            uint32_t* row = a.c3 + base + (k - j - 1) * j;
#pragma unroll
            for (int n = 0; n < WN; ++n) {
                const int64_t i = ib + n * 32;
                if (i < j) row[i] = (uint32_t)(int32_t)acc[m][n][r];   // exact in either format
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fused thermometer operands (int8).  The tiles hold V's own bytes and the
// level planes are formed in registers from the LDS fragments, so V is read
// once (no plane pass, no plane workspace) and a staged byte serves every
// level: the LDS and L2 traffic per multiply-add drop by the number of
// levels.  Two ways to form [v >= t] four bytes at a time:
//   kLvPerm (levels <= 7): v_perm_b32 with v's bytes as selectors into an
//     8-byte table whose byte k is [k >= t]; one instruction per word, both
//     operands 0/1, int32 sums exact up to 2^31.
//   kLvSub (levels 8..127): bytes staged as x = v | 0x80; x - t never
//     borrows across bytes and has bit 7 set exactly when v >= t.  A
//     fragments become -128 [v >= t] (sub, and), B fragments [v >= t] (sub,
//     shift, and); the sums are -128 min(a, b) summed, exact while
//     levels * n_f < 2^24.
// For the 3-way slices the B rows are min(v_i, v_j) bytewise, formed while
// staging ([min(a, b) >= t] = [a >= t][b >= t]).
// ---------------------------------------------------------------------------
constexpr int kLvMK = 128;   // fields per field tile (one byte each)
enum { kLvPerm = 0, kLvSub = 1 };

__host__ __device__ constexpr int lv_mode(int levels) { return levels <= 7 ? kLvPerm : kLvSub; }

struct LvArgs {
    const uint8_t* V;
    int64_t ld, n_f, n_v;
    int levels;
    int group;            // 2-way: block columns per tile-order group
    int64_t nk;           // field tiles
    const double* s;
    float* c2;
    int32_t* n2;
    int64_t nb, ntiles;
    // 3-way
    int64_t j_begin, j_end;
    const int64_t* prefix;
    uint32_t* c3;
    int64_t item0;
    int32_t mode, ob;
};

// Bytewise unsigned min of two words whose bytes all have bit 7 set.  Per
// byte, a - (b AND 0x7f) = 0x80 + (a7 - b7) lies in [1, 255], so bit 7 says
// a >= b and nothing borrows; the flags widen to 0xff bytes.
__device__ __forceinline__ uint32_t bytemin_hi(uint32_t a, uint32_t b) {
    const uint32_t ge = (a - (b & 0x7f7f7f7fu)) & 0x80808080u;
    const uint32_t m = ge | (ge - (ge >> 7));
    return (b & m) | (a & ~m);
}

// 16 bytes at byte offset `off` of a buffer: one b128 load when rows are
// 16-byte aligned, else byte loads.
template <bool ALIGNED>
__device__ __forceinline__ uint4 lv_load16(__amdgpu_buffer_rsrc_t rs, int off) {
    if constexpr (ALIGNED) {
        const v4u_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        return make_uint4(v[0], v[1], v[2], v[3]);
    } else {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            uint32_t x = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                x |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, off + 4 * e + b, 0, 0)
                     << (8 * b);
            w[e] = x;
        }
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Bytes of fields at or past n_f (nvalid = n_f - first field of the chunk)
// cleared; kLvSub also ORs every byte with 0x80.
template <int MODE>
__device__ __forceinline__ uint4 lv_prep(uint4 v, int nvalid) {
    if (nvalid < 16) {
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = nvalid - 4 * e;
            w[e] &= k >= 4 ? 0xffffffffu : k <= 0 ? 0u : (1u << (8 * k)) - 1u;
        }
        v = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if constexpr (MODE == kLvSub)
        v = make_uint4(v.x | 0x80808080u, v.y | 0x80808080u, v.z | 0x80808080u,
                       v.w | 0x80808080u);
    return v;
}

// Bytewise min of staged words (the 3-way X_j rows).
template <int MODE>
__device__ __forceinline__ uint32_t lv_min(uint32_t a, uint32_t b) {
    if constexpr (MODE == kLvSub) return bytemin_hi(a, b);
    return bytemin_hi(a | 0x80808080u, b | 0x80808080u) & 0x7f7f7f7fu;
}

// Level t of a fragment.
__device__ __forceinline__ v4i_t lv_perm(v4i_t f, uint32_t hi, uint32_t lo) {
    v4i_t r;   // byte k of {hi, lo} for each selector byte k = v (0..7)
    r.x = (int)__builtin_amdgcn_perm(hi, lo, (uint32_t)f.x);
    r.y = (int)__builtin_amdgcn_perm(hi, lo, (uint32_t)f.y);
    r.z = (int)__builtin_amdgcn_perm(hi, lo, (uint32_t)f.z);
    r.w = (int)__builtin_amdgcn_perm(hi, lo, (uint32_t)f.w);
    return r;
}
__device__ __forceinline__ v4i_t lv_suba(v4i_t f, uint32_t tt) {   // -128 [v >= t]
    v4i_t r;
    r.x = (int)(((uint32_t)f.x - tt) & 0x80808080u);
    r.y = (int)(((uint32_t)f.y - tt) & 0x80808080u);
    r.z = (int)(((uint32_t)f.z - tt) & 0x80808080u);
    r.w = (int)(((uint32_t)f.w - tt) & 0x80808080u);
    return r;
}
__device__ __forceinline__ v4i_t lv_subb(v4i_t f, uint32_t tt) {   // [v >= t]
    v4i_t r;
    r.x = (int)((((uint32_t)f.x - tt) >> 7) & 0x01010101u);
    r.y = (int)((((uint32_t)f.y - tt) >> 7) & 0x01010101u);
    r.z = (int)((((uint32_t)f.z - tt) >> 7) & 0x01010101u);
    r.w = (int)((((uint32_t)f.w - tt) >> 7) & 0x01010101u);
    return r;
}

// Main loop of one fused TB x TB tile: A rows a0 .. a0+TB-1 and B rows
// b0 .. b0+TB-1 of V (rows at or past n_v read as zero through the buffer
// bound); with MASK the B rows are min-ed with row mj.  Staging as in
// mfma_tile: tile kt+1 goes from registers into the second LDS buffer while
// tile kt is consumed, one barrier per field tile.  Inside a field tile the
// fragments of k-step ks+1 are read while k-step ks runs; the compiler
// interleaves the level transforms with the multiply-adds (measured: up to
// about six independent VALU instructions per 32x32x32 MFMA run beside the
// matrix core at no cost with two waves per SIMD, and an explicit
// sched_group_barrier interleave of the transforms was 20% slower).  LC > 0
// fixes the number of levels at compile time (0: a.levels at run time).  The
// sums come out as counts.
template <int WN, bool MASK, bool ALIGNED, int LC, int MODE, int TB = kMB>
__device__ __forceinline__ void lv_tile(const LvArgs& a, int64_t a0, int64_t b0, int64_t mj,
                                        bool active, int wr, int wc,
                                        v16i_t (&acc)[TB / 64][WN], int8_t* lds) {
    constexpr int WM = TB / 64;
    constexpr int kMThreads = mfma_threads<WN, TB>();
    constexpr int kMK = kLvMK;
    constexpr int KS = kMK / 32;                   // k-steps per field tile
    constexpr int kPitch = kMK + kPad;
    constexpr int kRowChunks = kMK / 16;
    constexpr int kStage = TB * kRowChunks / kMThreads;
    constexpr int kRowStep = kMThreads / kRowChunks;
    static_assert(TB * kRowChunks % kMThreads == 0, "staging must divide evenly");
    auto As = [&](int buf) { return lds + (2 * buf) * (TB * kPitch); };
    auto Bs = [&](int buf) { return lds + (2 * buf + 1) * (TB * kPitch); };
    const int lane = threadIdx.x % 64;
    const int L = LC > 0 ? LC : a.levels;

#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = (v16i_t){};

    // the host checks 256 * ld + 256 < 2^31, so a tile's rows take 32-bit offsets
    auto rsrc = [&](int64_t r0) {
        const int64_t rows = r0 < a.n_v ? (a.n_v - r0 < TB ? a.n_v - r0 : TB) : 0;
        return __builtin_amdgcn_make_buffer_rsrc((void*)(a.V + (rows > 0 ? r0 : 0) * a.ld),
                                                 (short)0, (int)(rows * a.ld), kRsrcWord3);
    };
    const __amdgpu_buffer_rsrc_t rsa = rsrc(a0), rsb = rsrc(b0);
    __amdgpu_buffer_rsrc_t rsm;
    if constexpr (MASK)
        rsm = __builtin_amdgcn_make_buffer_rsrc((void*)(a.V + mj * a.ld), (short)0, (int)a.n_f,
                                                kRsrcWord3);
    uint4 ra[kStage], rb[kStage];
    const int ch = threadIdx.x % kRowChunks;
    const int ldi = (int)a.ld;
    const int voff = (threadIdx.x / kRowChunks) * ldi + ch * 16;
    auto load = [&](int64_t kt) {
        const int f0 = (int)kt * kMK + ch * 16;
        const int nvalid = (int)a.n_f - f0;
        uint4 mk = make_uint4(0, 0, 0, 0);
        if constexpr (MASK) mk = lv_prep<MODE>(lv_load16<ALIGNED>(rsm, f0), nvalid);
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
            const int off = voff + c * kRowStep * ldi + (int)kt * kMK;
            ra[c] = lv_prep<MODE>(lv_load16<ALIGNED>(rsa, off), nvalid);
            rb[c] = lv_prep<MODE>(lv_load16<ALIGNED>(rsb, off), nvalid);
            if constexpr (MASK) {
                rb[c].x = lv_min<MODE>(rb[c].x, mk.x);
                rb[c].y = lv_min<MODE>(rb[c].y, mk.y);
                rb[c].z = lv_min<MODE>(rb[c].z, mk.z);
                rb[c].w = lv_min<MODE>(rb[c].w, mk.w);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
            const int row = (threadIdx.x + c * kMThreads) / kRowChunks;
            *(uint4*)(As(buf) + row * kPitch + ch * 16) = ra[c];
            *(uint4*)(Bs(buf) + row * kPitch + ch * 16) = rb[c];
        }
    };

    const int64_t nk = a.nk;
    load(0);
    store(0);
    __syncthreads();
    if (nk > 1) load(1);
    const int fr = lane % 32, fk = (lane / 32) * 16;
    auto frag = [&](const int8_t* A, const int8_t* B, int ks, v4i_t (&fa)[WM], v4i_t (&fb)[WN]) {
#pragma unroll
        for (int m = 0; m < WM; ++m)
            fa[m] = *(const v4i_t*)(A + (wr + m * 32 + fr) * kPitch + ks * 32 + fk);
#pragma unroll
        for (int n = 0; n < WN; ++n)
            fb[n] = *(const v4i_t*)(B + (wc + n * 32 + fr) * kPitch + ks * 32 + fk);
    };
    auto level = [&](const v4i_t (&fa)[WM], const v4i_t (&fb)[WN], int t) {
        v4i_t xa[WM], xb[WN];
        if constexpr (MODE == kLvPerm) {
            // table byte k = [k >= t], k = 0..7
            const uint32_t lo = t <= 3 ? 0x01010101u << (8 * t) : 0u;
            const uint32_t hi = t <= 4 ? 0x01010101u : 0x01010101u << (8 * (t - 4));
#pragma unroll
            for (int m = 0; m < WM; ++m) xa[m] = lv_perm(fa[m], hi, lo);
#pragma unroll
            for (int n = 0; n < WN; ++n) xb[n] = lv_perm(fb[n], hi, lo);
        } else {
            const uint32_t tt = (uint32_t)t * 0x01010101u;
#pragma unroll
            for (int m = 0; m < WM; ++m) xa[m] = lv_suba(fa[m], tt);
#pragma unroll
            for (int n = 0; n < WN; ++n) xb[n] = lv_subb(fb[n], tt);
        }
#pragma unroll
        for (int m = 0; m < WM; ++m)
#pragma unroll
            for (int n = 0; n < WN; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[m], xb[n], acc[m][n], 0, 0,
                                                                  0);
    };
    auto step = [&](int64_t kt, int cur) {
        const int8_t* A = As(cur);
        const int8_t* B = Bs(cur);
        v4i_t fa[2][WM], fb[2][WN];
        frag(A, B, 0, fa[0], fb[0]);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks + 1 < KS) frag(A, B, ks + 1, fa[(ks + 1) & 1], fb[(ks + 1) & 1]);
#pragma unroll(LC > 0 ? LC : 1)
            for (int t = 1; t <= L; ++t) level(fa[ks & 1], fb[ks & 1], t);
        }
        // tile kt+1 into the other buffer (after the last tile the write is
        // stale and never read; unconditional, so it joins this block)
        store(cur ^ 1);
        __syncthreads();   // kt+1 visible; everyone is done reading kt
        if (kt + 2 < nk) load(kt + 2);
    };
    if (active) {
        for (int64_t kt = 0; kt < nk; ++kt) step(kt, (int)(kt & 1));
    } else {
        for (int64_t kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) store((int)(kt & 1) ^ 1);
            __syncthreads();
            if (kt + 2 < nk) load(kt + 2);
        }
    }
    if constexpr (MODE == kLvSub) {   // -128 * count -> count
#pragma unroll
        for (int m = 0; m < WM; ++m)
#pragma unroll
            for (int n = 0; n < WN; ++n)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[m][n][r] = -acc[m][n][r] >> 7;
    }
}

template <int WN, bool ALIGNED, int LC, int MODE>
__global__ __launch_bounds__(mfma_threads<WN>(), 1) void ps_mfma2_lv_kernel(LvArgs a) {
    __shared__ __attribute__((aligned(16))) int8_t lds[4 * kMB * (kLvMK + kPad)];
    const int64_t t = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                      blockIdx.x / kXcds;
    if (t >= a.ntiles) return;
    int64_t bi, bj;
    grouped_tri_decode_rt(t, a.nb, a.group, bi, bj);
    const int64_t i0 = bi * kMB, j0 = bj * kMB;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * 128;        // j offset of the wave's block (A rows)
    const int wc = (wave / 2) * 32 * WN;    // i offset (B rows)
    const bool active = (i0 + wc < a.n_v) && (j0 + wr < a.n_v) && (i0 + wc + 1 < j0 + wr + 128);
    v16i_t acc[4][WN];
    lv_tile<WN, false, ALIGNED, LC, MODE>(a, j0, i0, 0, active, wr, wc, acc, lds);
    if (!active) return;
    MfmaArgs e{};
    e.n_v = a.n_v;
    e.s = a.s;
    e.c2 = a.c2;
    e.n2 = a.n2;
    mfma_epilogue<WN>(acc, e, i0, j0, wr, wc, lane);
}

template <int TB, bool ALIGNED, int LC, int MODE>
__global__ __launch_bounds__((mfma_threads<2, TB>()), kMB / TB) void ps_mfma3_lv_kernel(
    LvArgs a) {
    constexpr int WN = 2, WM = TB / 64;
    __shared__ __attribute__((aligned(16))) int8_t lds[4 * TB * (kLvMK + kPad)];
    const int64_t t = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                      blockIdx.x / kXcds;
    if (t >= a.ntiles) return;
    int64_t lo = 0, hi = a.j_end - a.j_begin;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (a.prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const int64_t j = a.j_begin + lo;
    int64_t i0, k0;
    slab_tile_origin(a.n_v, j, t - a.prefix[lo], TB, a.mode, a.ob, i0, k0);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * (TB / 2);   // k offset of the wave's block (A rows)
    const int wc = (wave / 2) * 32 * WN;    // i offset (B rows)
    const bool active = (k0 + wr < a.n_v) && (i0 + wc < j);
    v16i_t acc[WM][WN];
    lv_tile<WN, true, ALIGNED, LC, MODE, TB>(a, k0, i0, j, active, wr, wc, acc, lds);
    if (!active) return;
    // Eq. 1 on exact integers: n3 = n2(i,j) + n2(i,k) + n2(j,k) - n3', then
    // c3 = 3 n3 / (2 (s_i + s_j + s_k)) in FP64, rounded once to FP32 (d = 0
    // gives 0).  Every operand is an integer below 2^53, so the FP64 quotient
    // is the correctly rounded one whatever the order of the sums.  The
    // operands of a 32-row block are loaded together before any of its
    // stores (the stores could alias them for all the compiler knows, which
    // would otherwise serialise one load round trip per row).
    const int64_t base = slab_offset(a.n_v, j) - slab_offset(a.n_v, a.j_begin);
    const int64_t ib = i0 + wc + (lane % 32);
    const double* __restrict__ S = a.s;
    const int32_t* __restrict__ N2 = a.n2;
    float* __restrict__ c3 = (float*)a.c3;
    const double sj = S[j];
    const int64_t cj = j * (j - 1) / 2;   // n2(i, j) = N2[cj + i], i < j
    double si[WN];
    int64_t nij[WN];
#pragma unroll
    for (int n = 0; n < WN; ++n) {
        const int64_t i = ib + n * 32;
        si[n] = i < j ? S[i] : 0.0;
        nij[n] = i < j ? N2[cj + i] : 0;
    }
    // rows of the accumulators in batches of RB: the loads of batch b+1 are
    // issued before batch b is computed and stored (two register sets)
    constexpr int RB = 4, NB = WM * 16 / RB;
    struct Batch {
        double sk[RB];
        int32_t njk[RB], nik[RB][WN];
    };
    auto row_k = [&](int b, int q) {   // k of row q of batch b
        const int m = b / (16 / RB), r = (b % (16 / RB)) * RB + q;
        return k0 + wr + m * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
    };
    auto load_batch = [&](int b, Batch& o) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            int64_t k = row_k(b, q);
            if (k >= a.n_v) k = a.n_v - 1;   // loaded but not stored
            const int64_t ck = k * (k - 1) / 2;   // n2(x, k) = N2[ck + x], x < k
            o.sk[q] = S[k];
            o.njk[q] = N2[ck + j];
#pragma unroll
            for (int n = 0; n < WN; ++n) {
                const int64_t i = ib + n * 32;
                o.nik[q][n] = N2[ck + (i < j ? i : 0)];
            }
        }
    };
    auto store_batch = [&](int b, const Batch& o) {
        const int m = b / (16 / RB);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = (b % (16 / RB)) * RB + q;
            const int64_t k = row_k(b, q);
            if (k >= a.n_v) continue;
            float* row = c3 + base + (k - j - 1) * j;
#pragma unroll
            for (int n = 0; n < WN; ++n) {
                const int64_t i = ib + n * 32;
                if (i >= j) continue;
                const int64_t n3 =
                    nij[n] + (int64_t)o.nik[q][n] + (int64_t)o.njk[q] - (int64_t)acc[m][n][r];
                const double d3 = (si[n] + sj) + o.sk[q];
                row[i] = d3 > 0.0 ? (float)((3.0 * (double)n3) / (2.0 * d3)) : 0.0f;
            }
        }
    };
    Batch bt[2];
    load_batch(0, bt[0]);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) load_batch(b + 1, bt[(b + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        store_batch(b, bt[b & 1]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

static LvArgs lv_args(const MfmaLaunch& m) {
    LvArgs a{};
    a.V = (const uint8_t*)m.V;
    a.ld = m.ld;
    a.n_f = m.n_f;
    a.n_v = m.n_v;
    a.levels = m.levels;
    a.group = m.group >= 1 && m.group <= 64 ? m.group : kGroup;
    a.nk = (m.n_f + kLvMK - 1) / kLvMK;
    if (a.nk < 1) a.nk = 1;
    a.s = m.s;
    a.c2 = m.c2;
    a.n2 = (int32_t*)m.n2;
    return a;
}

static bool lv_aligned(const MfmaLaunch& m) {
    return (uintptr_t)m.V % 16 == 0 && m.ld % 16 == 0;
}

template <bool ALIGNED, int LC, int MODE>
static hipError_t go_mfma2_lv(const MfmaLaunch& m, hipStream_t st) {
    LvArgs a = lv_args(m);
    a.nb = (m.n_v + kMB - 1) / kMB;
    a.ntiles = a.nb * (a.nb + 1) / 2;
    return launch_items(a.ntiles, mfma_threads<2>(), kXcds, [&](unsigned grid, int64_t item0) {
        LvArgs b = a;
        b.item0 = item0;
        hipLaunchKernelGGL((ps_mfma2_lv_kernel<2, ALIGNED, LC, MODE>), dim3(grid),
                           dim3(mfma_threads<2>()), 0, st, b);
    });
}

template <bool ALIGNED, int LC, int MODE>
static hipError_t go_mfma3_lv(const MfmaLaunch& m, hipStream_t st) {
    constexpr int kEdge = kMB / 2;
    hipError_t e = launch_prefix3(m.n_v, m.j_begin, m.j_end, kMB, kSlabFull, kMB, m.prefix, st);
    if (e == hipSuccess)
        e = launch_prefix3(m.n_v, m.j_begin, m.j_end, kEdge, kSlabEdge, kMB, m.edge_prefix, st);
    if (e != hipSuccess) return e;
    LvArgs a = lv_args(m);   // a.n2: the pair numerators of Eq. 1
    a.j_begin = m.j_begin;
    a.j_end = m.j_end;
    a.c3 = (uint32_t*)m.c3;
    a.prefix = m.prefix;
    a.mode = kSlabFull;
    a.ob = kMB;
    a.ntiles = slab_tiles(m.n_v, m.j_begin, m.j_end, kMB, kSlabFull, kMB);
    const int64_t T2 = slab_tiles(m.n_v, m.j_begin, m.j_end, kEdge, kSlabEdge, kMB);
    if (a.ntiles > 0)
        e = launch_items(a.ntiles, mfma_threads<2>(), kXcds, [&](unsigned grid, int64_t item0) {
            LvArgs b = a;
            b.item0 = item0;
            hipLaunchKernelGGL((ps_mfma3_lv_kernel<kMB, ALIGNED, LC, MODE>), dim3(grid),
                               dim3(mfma_threads<2>()), 0, st, b);
        });
    if (e != hipSuccess || T2 == 0) return e;
    a.ntiles = T2;
    a.prefix = m.edge_prefix;
    a.mode = kSlabEdge;
    return launch_items(T2, mfma_threads<2, kEdge>(), kXcds, [&](unsigned grid, int64_t item0) {
        LvArgs b = a;
        b.item0 = item0;
        hipLaunchKernelGGL((ps_mfma3_lv_kernel<kEdge, ALIGNED, LC, MODE>), dim3(grid),
                           dim3(mfma_threads<2, kEdge>()), 0, st, b);
    });
}

// The fused launch for m: 16-byte row loads when V and its stride allow;
// table lookups for levels <= 7 (three levels unrolled and scheduled at
// compile time, the common case), the subtraction form above.
template <int WAY, bool AL>
static hipError_t go_lv_al(const MfmaLaunch& m, hipStream_t st) {
    if (WAY == 2) {
        if (m.levels == 3) return go_mfma2_lv<AL, 3, kLvPerm>(m, st);
        if (m.levels <= 7) return go_mfma2_lv<AL, 0, kLvPerm>(m, st);
        return go_mfma2_lv<AL, 0, kLvSub>(m, st);
    }
    if (m.levels == 3) return go_mfma3_lv<AL, 3, kLvPerm>(m, st);
    if (m.levels <= 7) return go_mfma3_lv<AL, 0, kLvPerm>(m, st);
    return go_mfma3_lv<AL, 0, kLvSub>(m, st);
}

template <int WAY>
static hipError_t go_lv(const MfmaLaunch& m, hipStream_t st) {
    return lv_aligned(m) ? go_lv_al<WAY, true>(m, st) : go_lv_al<WAY, false>(m, st);
}

// ---------------------------------------------------------------------------
// LDS-direct variant (used for fp4): field tiles go from global memory
// straight into LDS (global_load_lds_dwordx4: one wave instruction fills
// 1 KB of LDS, lane l at byte 16 l), so no registers hold staged data and
// the 128-byte tile fits the fp4 kernel without spills.  Two buffers: tile
// kt+1 loads while tile kt is consumed.  Rows are kDmaMK bytes, unpadded;
// 16-byte chunk c of row r sits at chunk position c ^ dma_swz(r).  Rows past
// n_v load row n_v - 1 (their outputs are never stored).
// Measured on the int8 planes the register-staged kernel above is faster
// (it is kept for int8); on fp4 this one is.
// ---------------------------------------------------------------------------
constexpr int kDmaMK = 128;

// Chunk swizzle of row r: for every chunk c, the 16-byte slots of any 8
// consecutive rows are distinct modulo 128 bytes and those of any 16
// consecutive rows distinct modulo 256 bytes, so fragment reads are free of
// bank conflicts whether the LDS serves 8 or 16 lanes of a b128 read at once.
// Rows r and r + 32 share a swizzle.
__device__ __forceinline__ int dma_swz(int r) { return (r % 8) ^ ((r / 8) % 2); }

// Tile hand-over between the waves of a workgroup: this wave's LDS reads are
// done and all of its tile loads have landed, then the barrier.  The empty
// asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void tile_sync() {
    // vmcnt 0, expcnt unconstrained (7), lgkmcnt 0
    __builtin_amdgcn_s_waitcnt(0x7 << 4);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int FMT, int WN>
__global__ __launch_bounds__(mfma_threads<WN>(), 1) void ps_mfma2_dma_kernel(MfmaArgs a) {
    constexpr int MK = kDmaMK;
    constexpr int kWaves = mfma_threads<WN>() / 64;
    constexpr int R = MK / 16;                 // chunks per row
    constexpr int RB = 1024 / MK;              // rows per wave instruction
    constexpr int NBW = kMB / RB / kWaves;     // instructions per wave per operand per tile
    constexpr int kStageBytes = kMB * MK;
    static_assert(NBW >= 1 && kMB % (RB * kWaves) == 0, "stage split");
    using AccT = typename std::conditional<FMT == kFmtF4, v16f_t, v16i_t>::type;
    __shared__ __attribute__((aligned(1024))) int8_t As[2 * kStageBytes];   // j rows
    __shared__ __attribute__((aligned(1024))) int8_t Bs[2 * kStageBytes];   // i rows
    const int64_t t = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                      blockIdx.x / kXcds;
    if (t >= a.ntiles) return;
    int64_t bi, bj;
    grouped_tri_decode<kGroup>(t, a.nb, bi, bj);
    const int64_t i0 = bi * kMB, j0 = bj * kMB;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * 128;
    const int wc = (wave / 2) * 32 * WN;
    const bool active = (i0 + wc < a.n_v) && (j0 + wr < a.n_v) && (i0 + wc + 1 < j0 + wr + 128);

    AccT acc[4][WN];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = (AccT){};

    // per-lane source rows and chunk offsets of this wave's loads
    const int8_t* srcA[NBW];
    const int8_t* srcB[NBW];
#pragma unroll
    for (int u = 0; u < NBW; ++u) {
        const int row = (wave + kWaves * u) * RB + lane / R;
        const int c = (lane % R) ^ dma_swz(row);
        const int64_t gj = j0 + row < a.n_v ? j0 + row : a.n_v - 1;
        const int64_t gi = i0 + row < a.n_v ? i0 + row : a.n_v - 1;
        srcA[u] = a.P + gj * a.kp + c * 16;
        srcB[u] = a.P + gi * a.kp + c * 16;
    }
    auto issue = [&](int64_t kt, int buf) {
        const int64_t k0 = kt * MK;
#pragma unroll
        for (int u = 0; u < NBW; ++u) {
            const int blk = (wave + kWaves * u) * 1024;
            __builtin_amdgcn_global_load_lds((const void*)(srcA[u] + k0),
                                             (void*)(As + buf * kStageBytes + blk), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(srcB[u] + k0),
                                             (void*)(Bs + buf * kStageBytes + blk), 16, 0, 0);
        }
    };

    const int64_t nk = a.kp / MK;
    issue(0, 0);
    const int fr = lane % 32, hk = lane / 32;
    const int sw = dma_swz(fr);   // swizzle of rows wr + m*32 + fr and wc + n*32 + fr
    if (active) {
        for (int64_t kt = 0; kt < nk; ++kt) {
            const int cur = (int)(kt & 1);
            tile_sync();   // tile kt in LDS everywhere; tile kt-1 no longer read
            if (kt + 1 < nk) issue(kt + 1, cur ^ 1);
            const int8_t* A = As + cur * kStageBytes;
            const int8_t* B = Bs + cur * kStageBytes;
            // fragments of k-step ks+1 are read into the other register set
            // while k-step ks runs (scheduled below; measured 4% faster)
            v4i_t fa[2][4], fb[2][WN];
            auto frag = [&](int ks, int sl) {
                const int co = ((ks * 2 + hk) ^ sw) * 16;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    fa[sl][m] = *(const v4i_t*)(A + (wr + m * 32 + fr) * MK + co);
#pragma unroll
                for (int n = 0; n < WN; ++n)
                    fb[sl][n] = *(const v4i_t*)(B + (wc + n * 32 + fr) * MK + co);
            };
            frag(0, 0);
#pragma unroll
            for (int ks = 0; ks < MK / 32; ++ks) {
                if (ks + 1 < MK / 32) frag(ks + 1, (ks + 1) & 1);
                const int sl = ks & 1;
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < WN; ++n) {
                        if constexpr (FMT == kFmtI8) {
                            acc[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                fa[sl][m], fb[sl][n], acc[m][n], 0, 0, 0);
                        } else {
                            const v8i_t xa = {fa[sl][m].x, fa[sl][m].y, fa[sl][m].z,
                                              fa[sl][m].w, 0, 0, 0, 0};
                            const v8i_t xb = {fb[sl][n].x, fb[sl][n].y, fb[sl][n].z,
                                              fb[sl][n].w, 0, 0, 0, 0};
                            acc[m][n] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                xa, xb, acc[m][n], 4, 4, 0, 127, 0, 127);
                        }
                    }
            }
            if constexpr (WN == 2) {
                __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
                for (int ks = 0; ks < MK / 32 - 1; ++ks) {
#pragma unroll
                    for (int i = 0; i < 6; ++i) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                    }
                    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
            }
        }
    } else {
        for (int64_t kt = 0; kt < nk; ++kt) {
            tile_sync();
            if (kt + 1 < nk) issue(kt + 1, (int)(kt & 1) ^ 1);
        }
        return;   // the last tile_sync waited for every load of this wave
    }

    mfma_epilogue<WN>(acc, a, i0, j0, wr, wc, lane);
}

// Thermometer planes of V into m.planes (when m.expand); returns the plane-row
// length in bytes through kp.
template <int FMT>
static hipError_t expand_planes(const MfmaLaunch& m, int64_t& kp, hipStream_t st) {
    const int64_t kpad = plane_fields(m.n_f, FMT);
    kp = (int64_t)m.levels * kpad / fields_per_byte(FMT);
    if (!m.expand) return hipSuccess;
    const int64_t total = m.n_v * (kpad / 32);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ps_thermo_expand_kernel<FMT>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const uint8_t*)m.V, m.n_f, m.n_v, m.ld, m.levels, kpad, m.planes);
    return hipGetLastError();
}

template <int FMT, int WN>
static hipError_t go_mfma2(const MfmaLaunch& m, hipStream_t st) {
    int64_t kp = 0;
    hipError_t e = expand_planes<FMT>(m, kp, st);
    if (e != hipSuccess) return e;
    const int64_t nb = (m.n_v + kMB - 1) / kMB;
    const int64_t T = nb * (nb + 1) / 2;
    MfmaArgs a{m.planes, kp, m.n_v, m.s, m.c2, (int32_t*)m.n2, nb, T, 0, 0, nullptr, nullptr, 0};
    return launch_items(T, mfma_threads<WN>(), kXcds, [&](unsigned grid, int64_t item0) {
        MfmaArgs b = a;
        b.item0 = item0;
        if constexpr (FMT == kFmtF4 && WN == 2)
            hipLaunchKernelGGL((ps_mfma2_dma_kernel<FMT, WN>), dim3(grid),
                               dim3(mfma_threads<WN>()), 0, st, b);
        else
            hipLaunchKernelGGL((ps_mfma2_kernel<FMT, WN>), dim3(grid), dim3(mfma_threads<WN>()),
                               0, st, b);
    });
}

template <int FMT>
static hipError_t go_mfma3(const MfmaLaunch& m, hipStream_t st) {
    int64_t kp = 0;
    hipError_t e = expand_planes<FMT>(m, kp, st);
    if (e != hipSuccess) return e;
    // whole 256-wide tiles of each slab rectangle, then 128-wide edge tiles
    constexpr int kEdge = kMB / 2;
    e = launch_prefix3(m.n_v, m.j_begin, m.j_end, kMB, kSlabFull, kMB, m.prefix, st);
    if (e == hipSuccess)
        e = launch_prefix3(m.n_v, m.j_begin, m.j_end, kEdge, kSlabEdge, kMB, m.edge_prefix, st);
    if (e != hipSuccess) return e;
    const int64_t T1 = slab_tiles(m.n_v, m.j_begin, m.j_end, kMB, kSlabFull, kMB);
    const int64_t T2 = slab_tiles(m.n_v, m.j_begin, m.j_end, kEdge, kSlabEdge, kMB);
    MfmaArgs a{m.planes, kp, m.n_v, m.s, nullptr, nullptr, 0, T1, m.j_begin, m.j_end, m.prefix,
               (uint32_t*)m.c3, 0, kSlabFull, kMB};
    if (T1 > 0)
        e = launch_items(T1, mfma_threads<2>(), kXcds, [&](unsigned grid, int64_t item0) {
            MfmaArgs b = a;
            b.item0 = item0;
            hipLaunchKernelGGL((ps_mfma3_kernel<FMT, kMB>), dim3(grid), dim3(mfma_threads<2>()),
                               0, st, b);
        });
    if (e != hipSuccess || T2 == 0) return e;
    a.ntiles = T2;
    a.prefix = m.edge_prefix;
    a.mode = kSlabEdge;
    return launch_items(T2, mfma_threads<2, kEdge>(), kXcds, [&](unsigned grid, int64_t item0) {
        MfmaArgs b = a;
        b.item0 = item0;
        hipLaunchKernelGGL((ps_mfma3_kernel<FMT, kEdge>), dim3(grid),
                           dim3(mfma_threads<2, kEdge>()), 0, st, b);
    });
}

hipError_t launch_mfma3(const MfmaLaunch& m, hipStream_t st) {
    if (m.n_v < 3 || m.j_end <= m.j_begin) return hipSuccess;
    if (mfma_fused(m.n_f, m.levels, m.fmt, 0)) return go_lv<3>(m, st);
    return m.fmt == kFmtF4 ? go_mfma3<kFmtF4>(m, st) : go_mfma3<kFmtI8>(m, st);
}

hipError_t launch_mfma2(const MfmaLaunch& m, hipStream_t st) {
    if (m.n_v < 2) return hipSuccess;
    if (mfma_fused(m.n_f, m.levels, m.fmt, m.wide)) return go_lv<2>(m, st);
    if (m.wide)
        return m.fmt == kFmtF4 ? go_mfma2<kFmtF4, 4>(m, st) : go_mfma2<kFmtI8, 4>(m, st);
    return m.fmt == kFmtF4 ? go_mfma2<kFmtF4, 2>(m, st) : go_mfma2<kFmtI8, 2>(m, st);
}

}  // namespace ps

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

// n / d correctly rounded, for integers 0 <= n < 2^24 and 1 <= d < 2^24 held
// in floats (the FP32 quotients of Section 2.1 and Eq. 1): the reciprocal
// refinement and the two remainder corrections of the IEEE division
// sequence, without its range scaling and special-case fix-up.  No
// operand, reciprocal, partial quotient or remainder here is denormal,
// infinite or needs scaling, so those steps are identities and the result
// is the sequence's own, the correctly rounded quotient.
__device__ __forceinline__ float div_u24(float n, float d) {
    const float y0 = __builtin_amdgcn_rcpf(d);
    const float y = __builtin_fmaf(__builtin_fmaf(-d, y0, 1.0f), y0, y0);
    const float q0 = n * y;
    const float q1 = __builtin_fmaf(__builtin_fmaf(-d, q0, n), y, q0);
    return __builtin_fmaf(__builtin_fmaf(-d, q1, n), y, q1);
}

// Epilogue of one wave's 4 x WN blocks of 32 x 32 (Section 2.1): n2 exact,
// c2 = 2 n2 / (s_i + s_j) in FP64, rounded once to FP32, d = 0 gives 0.
// F32: the same value from the FP32 division of the exact integers (both
// below 2^24: 2 L n_f < 2^24 for L levels): the FP64 quotient lies more
// than 2^-48 (relative) from every FP32 rounding boundary, so rounding it
// to FP32 gives the correctly rounded FP32 quotient.
template <int WN, bool F32 = false, typename AccT>
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
                    if constexpr (F32) {
                        const float q = div_u24((float)(2 * num), d > 0.0 ? (float)d : 1.0f);
                        a.c2[base + i] = d > 0.0 ? q : 0.0f;
                    } else {
                        a.c2[base + i] = d > 0.0 ? (float)((2.0 * (double)num) / d) : 0.0f;
                    }
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
// Kernels: ps_mfma2_lvd_kernel (2-way, rows 16-byte aligned and n_f a
// multiple of 64: stages go straight into LDS), ps_mfma2_lv_kernel (2-way,
// any rows: staged through registers, fields past n_f cleared),
// ps_mfma3_lvsd_kernel (3-way split tiling, 1..7 levels on aligned rows
// with n_f a multiple of 64: plain rows straight into LDS, pair rows through
// registers), ps_mfma3_lvs_kernel (3-way split tiling, any rows and levels)
// and ps_mfma3_lv_kernel (3-way per-slab tiles).
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
    int32_t f32div;       // the quotient's operands are integers below 2^24 (FP32 division)
    // split 3-way tiling, part p = 0, 1: its tiles, row tiles, the prefix of
    // their column-tile counts, and its pairs [r_begin, r_end) (colex indices
    // for the (i, j) part, lex indices for the (j, k) part); tiles
    // [0, nt[0]) of a launch are part 0's, the next nt[1] part 1's
    int64_t nt[2], nrt[2], r_begin[2], r_end[2];
    const int64_t* pre[2];
};

// Bytewise min of a and b given d, a word whose byte k has bit 7 set exactly
// where byte k of a is at least byte k of b: the flags widen to 0xff bytes
// with one byte permute (selectors 8-11 replicate bit 7 of bytes 1, 3, 5, 7
// of {d, d << 8}, which are d's bytes 0, 2, 1, 3), then one bit-field insert.
__device__ __forceinline__ uint32_t bytemin_flags(uint32_t d, uint32_t a, uint32_t b) {
    const uint32_t m = __builtin_amdgcn_perm(d, d << 8, 0x0B090A08u);
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

// Bytewise min of staged words (the 3-way pair rows).  kLvSub bytes all have
// bit 7 set: a - (b AND 0x7f) is 0x80 + (a7 - b7) per byte, in [1, 255]; the
// other modes' bytes are below 128: (a OR 0x80) - b is 0x80 + a - b per byte,
// in [1, 255].  Either way nothing borrows and bit 7 says a >= b.
template <int MODE>
__device__ __forceinline__ uint32_t lv_min(uint32_t a, uint32_t b) {
    if constexpr (MODE == kLvSub) return bytemin_flags(a - (b & 0x7f7f7f7fu), a, b);
    return bytemin_flags((a | 0x80808080u) - b, a, b);
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

// Staging geometry of a fused tile: each of THREADS threads stages kStage
// 16-byte chunks of an operand of ROWS rows per field tile, chunk ch of rows
// row(0) + c kRowStep.
template <int THREADS, int ROWS>
struct LvGeom {
    static constexpr int kMThreads = THREADS;
    static constexpr int kRows = ROWS;
    static constexpr int kRowChunks = kLvMK / 16;
    static constexpr int kStage = ROWS * kRowChunks / THREADS;
    static constexpr int kRowStep = THREADS / kRowChunks;
    static_assert(ROWS * kRowChunks % THREADS == 0, "staging must divide evenly");
    __device__ static int ch() { return threadIdx.x % kRowChunks; }
    __device__ static int row(int c) { return threadIdx.x / kRowChunks + c * kRowStep; }
};
template <int WN, int TB>
using LvGeomW = LvGeom<mfma_threads<WN, TB>(), TB>;

// Row sources of the staging.  LvRows: TB consecutive rows of V from r0 (rows
// at or past n_v read as zero through the buffer bound); with MASK each row
// is min-ed bytewise with row mj (the 3-way X_j rows).  The host checks
// 256 ld + 256 < 2^31, so a tile's rows take 32-bit offsets.
template <class G, bool ALIGNED, int MODE, bool MASK>
struct LvRows {
    using Geom = G;
    static constexpr int TB = G::kRows;
    __amdgpu_buffer_rsrc_t rs, rm;
    int voff, step;
    uint4 mk;
    __device__ LvRows(const LvArgs& a, int64_t r0, int64_t mj) {
        const int64_t rows = r0 < a.n_v ? (a.n_v - r0 < TB ? a.n_v - r0 : TB) : 0;
        rs = __builtin_amdgcn_make_buffer_rsrc((void*)(a.V + (rows > 0 ? r0 : 0) * a.ld),
                                               (short)0, (int)(rows * a.ld), kRsrcWord3);
        if constexpr (MASK)
            rm = __builtin_amdgcn_make_buffer_rsrc((void*)(a.V + mj * a.ld), (short)0,
                                                   (int)a.n_f, kRsrcWord3);
        voff = G::row(0) * (int)a.ld + G::ch() * 16;
        step = G::kRowStep * (int)a.ld;
    }
    // once per field tile (ko: its first field); nvalid = n_f - this chunk's first field
    __device__ void prep(int ko, int nvalid) {
        if constexpr (MASK) mk = lv_prep<MODE>(lv_load16<ALIGNED>(rm, ko + G::ch() * 16), nvalid);
    }
    __device__ uint4 load(int c, int ko, int nvalid) const {
        uint4 v = lv_prep<MODE>(lv_load16<ALIGNED>(rs, voff + c * step + ko), nvalid);
        if constexpr (MASK) {
            v.x = lv_min<MODE>(v.x, mk.x);
            v.y = lv_min<MODE>(v.y, mk.y);
            v.z = lv_min<MODE>(v.z, mk.z);
            v.w = lv_min<MODE>(v.w, mk.w);
        }
        return v;
    }
};

// LvPairs: row r of the tile is a pair of rows (x, y) of V, staged as
// min(v_x, v_y) (the 3-way rows X_y's column x, or X_x's column y).  The
// rows come through one buffer resource over all of V (the host checks
// n_v ld + 256 < 2^31); pair(r, x, y) gives each staged row's pair.
template <class G, bool ALIGNED, int MODE>
struct LvPairs {
    using Geom = G;
    __amdgpu_buffer_rsrc_t rs;
    int ox[G::kStage], oy[G::kStage];
    template <class F>
    __device__ LvPairs(const LvArgs& a, F pair) {
        rs = __builtin_amdgcn_make_buffer_rsrc((void*)a.V, (short)0, (int)(a.n_v * a.ld),
                                               kRsrcWord3);
#pragma unroll
        for (int c = 0; c < G::kStage; ++c) {
            int64_t x, y;
            pair(G::row(c), x, y);
            ox[c] = (int)(x * a.ld) + G::ch() * 16;
            oy[c] = (int)(y * a.ld) + G::ch() * 16;
        }
    }
    __device__ void prep(int, int) {}
    __device__ uint4 load(int c, int ko, int nvalid) const {
        const uint4 x = lv_prep<MODE>(lv_load16<ALIGNED>(rs, ox[c] + ko), nvalid);
        const uint4 y = lv_prep<MODE>(lv_load16<ALIGNED>(rs, oy[c] + ko), nvalid);
        return make_uint4(lv_min<MODE>(x.x, y.x), lv_min<MODE>(x.y, y.y),
                          lv_min<MODE>(x.z, y.z), lv_min<MODE>(x.w, y.w));
    }
};

// Main loop of one fused TB x TB tile: the A operand's rows (output rows)
// from source sa, the B operand's (output columns) from sb.  Staging as in
// mfma_tile: tile kt+1 goes from registers into the second LDS buffer while
// tile kt is consumed, one barrier per field tile.  Inside a field tile the
// fragments of k-step ks+1 are read while k-step ks runs; the compiler
// interleaves the level transforms with the multiply-adds (measured: up to
// about six independent VALU instructions per 32x32x32 MFMA run beside the
// matrix core at no cost with two waves per SIMD, and an explicit
// sched_group_barrier interleave of the transforms was 20% slower).  LC > 0
// fixes the number of levels at compile time (0: a.levels at run time).  The
// sums come out as counts.
template <int WN, bool ALIGNED, int LC, int MODE, int TB, class SA, class SB>
__device__ __forceinline__ void lv_tile(const LvArgs& a, SA& sa, SB& sb, bool active, int wr,
                                        int wc, v16i_t (&acc)[TB / 64][WN], int8_t* lds) {
    using G = LvGeomW<WN, TB>;
    constexpr int WM = TB / 64;
    constexpr int kMK = kLvMK;
    constexpr int KS = kMK / 32;                   // k-steps per field tile
    constexpr int kPitch = kMK + kPad;
    constexpr int kStage = G::kStage;
    constexpr int kMThreads = G::kMThreads;
    constexpr int kRowChunks = G::kRowChunks;
    auto As = [&](int buf) { return lds + (2 * buf) * (TB * kPitch); };
    auto Bs = [&](int buf) { return lds + (2 * buf + 1) * (TB * kPitch); };
    const int lane = threadIdx.x % 64;
    const int L = LC > 0 ? LC : a.levels;

#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = (v16i_t){};

    uint4 ra[kStage], rb[kStage];
    const int ch = G::ch();
    auto load = [&](int64_t kt) {
        const int ko = (int)kt * kMK;
        const int nvalid = (int)a.n_f - ko - ch * 16;
        sa.prep(ko, nvalid);
        sb.prep(ko, nvalid);
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
            ra[c] = sa.load(c, ko, nvalid);
            rb[c] = sb.load(c, ko, nvalid);
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

// Main loop of a half tile with one LDS buffer, two workgroups per CU:
// the A operand's 256 rows and the B operand's 128, four waves of 128 x 64.
// Field tile kt+1 is loaded into registers while kt is consumed from LDS,
// then a barrier, the registers go to LDS, and a barrier; the other
// workgroup on the CU keeps the matrix cores busy across this one's
// barriers and epilogue.
template <int WN, bool ALIGNED, int LC, int MODE, class SA, class SB>
__device__ __forceinline__ void lv_tile_sb(const LvArgs& a, SA& sa, SB& sb, bool active, int wr,
                                           int wc, v16i_t (&acc)[4][WN], int8_t* lds) {
    using GA = typename SA::Geom;
    using GB = typename SB::Geom;
    constexpr int WM = 4;
    constexpr int KS = kLvMK / 32;
    constexpr int kPitch = kLvMK + kPad;
    int8_t* As = lds;
    int8_t* Bs = lds + GA::kRows * kPitch;
    const int lane = threadIdx.x % 64;
    const int L = LC > 0 ? LC : a.levels;
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = (v16i_t){};
    uint4 ra[GA::kStage], rb[GB::kStage];
    const int ch = GA::ch();
    auto load = [&](int64_t kt) {
        const int ko = (int)kt * kLvMK;
        const int nvalid = (int)a.n_f - ko - ch * 16;
        sa.prep(ko, nvalid);
        sb.prep(ko, nvalid);
#pragma unroll
        for (int c = 0; c < GA::kStage; ++c) ra[c] = sa.load(c, ko, nvalid);
#pragma unroll
        for (int c = 0; c < GB::kStage; ++c) rb[c] = sb.load(c, ko, nvalid);
    };
    auto store = [&]() {
#pragma unroll
        for (int c = 0; c < GA::kStage; ++c)
            *(uint4*)(As + GA::row(c) * kPitch + ch * 16) = ra[c];
#pragma unroll
        for (int c = 0; c < GB::kStage; ++c)
            *(uint4*)(Bs + GB::row(c) * kPitch + ch * 16) = rb[c];
    };
    const int fr = lane % 32, fk = (lane / 32) * 16;
    auto frag = [&](int ks, v4i_t (&fa)[WM], v4i_t (&fb)[WN]) {
#pragma unroll
        for (int m = 0; m < WM; ++m)
            fa[m] = *(const v4i_t*)(As + (wr + m * 32 + fr) * kPitch + ks * 32 + fk);
#pragma unroll
        for (int n = 0; n < WN; ++n)
            fb[n] = *(const v4i_t*)(Bs + (wc + n * 32 + fr) * kPitch + ks * 32 + fk);
    };
    auto level = [&](const v4i_t (&fa)[WM], const v4i_t (&fb)[WN], int t) {
        v4i_t xa[WM], xb[WN];
        if constexpr (MODE == kLvPerm) {
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
    const int64_t nk = a.nk;
    load(0);
    store();
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load(kt + 1);
        if (active) {
            v4i_t fa[2][WM], fb[2][WN];
            frag(0, fa[0], fb[0]);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks + 1 < KS) frag(ks + 1, fa[(ks + 1) & 1], fb[(ks + 1) & 1]);
#pragma unroll(LC > 0 ? LC : 1)
                for (int t = 1; t <= L; ++t) level(fa[ks & 1], fb[ks & 1], t);
            }
        }
        __syncthreads();   // everyone is done reading field tile kt
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }
    if constexpr (MODE == kLvSub) {
#pragma unroll
        for (int m = 0; m < WM; ++m)
#pragma unroll
            for (int n = 0; n < WN; ++n)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[m][n][r] = -acc[m][n][r] >> 7;
    }
}

// 2-way half tiles: work item t2 is half t2 % 2 (output columns 0-127 or
// 128-255) of 256 x 256 tile t2 / 2, four waves, two workgroups per CU.
// Register staging with the fields past n_f cleared: the launch for rows
// that are not 16-byte aligned or n_f not a multiple of kLvdMK.
template <int WN, bool ALIGNED, int LC, int MODE>
__global__ __launch_bounds__(256, 2) void ps_mfma2_lv_kernel(LvArgs a) {
    __shared__ __attribute__((aligned(16))) int8_t lds[(kMB + kMB / 2) * (kLvMK + kPad)];
    const int64_t t2 = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                       blockIdx.x / kXcds;
    if (t2 >= 2 * a.ntiles) return;
    int64_t bi, bj;
    grouped_tri_decode_rt(t2 / 2, a.nb, a.group, bi, bj);
    const int64_t i0 = bi * kMB + (t2 % 2) * (kMB / 2), j0 = bj * kMB;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * 128;        // j offset of the wave's block (A rows)
    const int wc = (wave / 2) * 32 * WN;    // i offset (B rows)
    const bool active = (i0 + wc < a.n_v) && (j0 + wr < a.n_v) && (i0 + wc + 1 < j0 + wr + 128);
    v16i_t acc[4][WN];
    LvRows<LvGeom<256, kMB>, ALIGNED, MODE, false> sa(a, j0, 0);
    LvRows<LvGeom<256, kMB / 2>, ALIGNED, MODE, false> sb(a, i0, 0);
    lv_tile_sb<WN, ALIGNED, LC, MODE>(a, sa, sb, active, wr, wc, acc, lds);
    if (!active) return;
    MfmaArgs e{};
    e.n_v = a.n_v;
    e.s = a.s;
    e.c2 = a.c2;
    e.n2 = a.n2;
    if (a.f32div)
        mfma_epilogue<WN, true>(acc, e, i0, j0, wr, wc, lane);
    else
        mfma_epilogue<WN>(acc, e, i0, j0, wr, wc, lane);
}

// Eq. 1 on exact integers for one 3-way tile (rows k0 .. k0+TB-1, columns
// i0 .. i0+TB-1 of slab j): n3 = n2(i,j) + n2(i,k) + n2(j,k) - n3', then
// c3 = 3 n3 / (2 (s_i + s_j + s_k)), rounded once to FP32, 0 where the
// denominator is 0.  The operands are integers; F32 is taken when
// 6 levels n_f < 2^24, so numerator and denominator are exact FP32 integers
// and the correctly rounded FP32 quotient equals the FP32 rounding of the
// FP64 quotient (double rounding through 53 bits is innocuous for a
// quotient of 24-bit operands); otherwise the quotient is taken in FP64 and
// rounded to FP32.  The numerator is summed modulo 2^32 (the intermediate
// sum can pass 2^31; n3 itself is below 2^31).
//
// 2 s_k and n2(j, k) of the tile's rows are staged in LDS once; n2(i, k)
// comes through a buffer resource over the tile's rows of the pair table,
// and the stores through one over the tile's rows of the slab: rows past
// n_v and columns i >= j fall outside (loads read 0, stores are dropped),
// so no branch guards an element.  Loads run one batch of rows ahead of the
// arithmetic and stores.
template <int TB, bool F32>
__device__ __forceinline__ void lv3_epilogue(const LvArgs& a, const v16i_t (&acc)[TB / 64][2],
                                             int64_t j, int64_t k0, int64_t i0, int wr, int wc,
                                             bool active, int8_t* lds) {
    using R = typename std::conditional<F32, float, double>::type;
    constexpr int WN = 2, WM = TB / 64;
    const int lane = threadIdx.x % 64;
    const double* __restrict__ S = a.s;
    const int32_t* __restrict__ N2 = a.n2;
    R* rs2 = (R*)lds;                        // 2 s_k
    int32_t* rnj = (int32_t*)(lds + TB * sizeof(R));   // n2(j, k)
    const int64_t kend = k0 + TB < a.n_v ? k0 + TB : a.n_v;   // rows of the tile below n_v
    if (threadIdx.x < TB) {
        const int64_t k = k0 + threadIdx.x;
        const bool in = k < kend;
        rs2[threadIdx.x] = in ? (R)(2.0 * S[k]) : (R)0;
        rnj[threadIdx.x] = in ? N2[k * (k - 1) / 2 + j] : 0;
    }
    __syncthreads();
    if (!active) return;
    // pair-table rows k0 .. kend-1: entry (k, x) at element k (k-1)/2 - c(k0) + x
    const int64_t ck0 = k0 * (k0 - 1) / 2;
    const __amdgpu_buffer_rsrc_t rn2 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(N2 + ck0), (short)0, (int)((kend * (kend - 1) / 2 - ck0) * 4), kRsrcWord3);
    // slab rows k0 .. kend-1: triple (i, j, k) at element (k - k0) j + i
    const int64_t base = slab_offset(a.n_v, j) - slab_offset(a.n_v, a.j_begin) + (k0 - j - 1) * j;
    const __amdgpu_buffer_rsrc_t rc3 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.c3 + base), (short)0, (int)((kend - k0) * j * 4), kRsrcWord3);
    const int jj = (int)j, ki = (int)k0;
    const R sj = (R)S[j];
    const int64_t cj = j * (j - 1) / 2;   // n2(i, j) = N2[cj + i], i < j
    R ls2[WN];            // 2 (s_i + s_j)
    uint32_t nij[WN];     // n2(i, j)
    int ioff[WN];         // byte offset of column i; out of range when i >= j
    int icol[WN];         // column i (pair-table offset within a row)
#pragma unroll
    for (int n = 0; n < WN; ++n) {
        const int64_t i = i0 + wc + n * 32 + lane % 32;
        const bool vi = i < j;
        ls2[n] = vi ? (R)2 * ((R)S[i] + sj) : (R)0;
        nij[n] = vi ? (uint32_t)N2[cj + i] : 0u;
        icol[n] = (int)i;
        ioff[n] = vi ? (int)i * 4 : (int)0x80000000;
    }
    // row q of batch b: accumulator row r of block m, tile row dk
    constexpr int RB = 8, NB = WM * 16 / RB;
    auto row_dk = [&](int b, int q) {
        const int m = b / (16 / RB), r = (b % (16 / RB)) * RB + q;
        return wr + m * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
    };
    auto load_batch = [&](int b, uint32_t (&o)[RB][WN]) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int dk = row_dk(b, q);
            // c(k0 + dk) - c(k0) = dk (dk + 2 k0 - 1) / 2
            const int roff = (int)(((uint32_t)dk * (uint32_t)(dk + 2 * ki - 1)) >> 1);
#pragma unroll
            for (int n = 0; n < WN; ++n)
                o[q][n] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                    rn2, (roff + icol[n]) * 4, 0, 0);
        }
    };
    auto store_batch = [&](int b, const uint32_t (&o)[RB][WN]) {
        const int m = b / (16 / RB);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = (b % (16 / RB)) * RB + q;
            const int dk = row_dk(b, q);
            const R rk = rs2[dk];
            const uint32_t njk = (uint32_t)rnj[dk];
            const int soff = dk * jj * 4;
#pragma unroll
            for (int n = 0; n < WN; ++n) {
                const uint32_t n3 = nij[n] + njk + o[q][n] - (uint32_t)acc[m][n][r];
                // denominators are even integers: d = 0 or d >= 2; the
                // quotient is formed unconditionally (no branch) and d = 0
                // selects 0
                const R d = ls2[n] + rk;
                const R dd = d > (R)0 ? d : (R)1;
                float q;
                if constexpr (F32)
                    q = div_u24((float)(3u * n3), dd);
                else
                    q = (float)((3.0 * (double)n3) / dd);
                const float c = d > (R)0 ? q : 0.0f;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, c), rc3,
                                                      (int)((uint32_t)soff + (uint32_t)ioff[n]),
                                                      0, 0);
            }
        }
    };
    uint32_t bt[2][RB][WN];
    load_batch(0, bt[0]);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) load_batch(b + 1, bt[(b + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        store_batch(b, bt[b & 1]);
        __builtin_amdgcn_sched_barrier(0);
    }
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
    LvRows<LvGeomW<WN, TB>, ALIGNED, MODE, false> sa(a, k0, 0);
    LvRows<LvGeomW<WN, TB>, ALIGNED, MODE, true> sb(a, i0, j);
    lv_tile<WN, ALIGNED, LC, MODE, TB>(a, sa, sb, active, wr, wc, acc, lds);
    // The main loop ended on a barrier after its last LDS read, so the LDS is
    // free: the per-row operands of Eq. 1 for the tile's TB rows k go there
    // (every wave takes part in the staging and its barrier).
    if (a.f32div)
        lv3_epilogue<TB, true>(a, acc, j, k0, i0, wr, wc, active, lds);
    else
        lv3_epilogue<TB, false>(a, acc, j, k0, i0, wr, wc, active, lds);
}


// ---------------------------------------------------------------------------
// Split tiling of the fused 3-way slices (split3): every tile is a whole
// 256 x 256 tile of pairs x single vectors, so no slab edge needs narrower
// tiles.  Part 0: output columns are the colex pairs (i, j), j < js, staged
// as min(v_i, v_j); output rows are k from the row tile's smallest j + 1.
// Part 1: output rows are the lex pairs (j, k), j >= js, staged as
// min(v_j, v_k); output columns are i from 0 below the row tile's largest j.
// Entries outside i < j < k < n_v are computed by waves that also hold wanted
// ones and are never stored (a wave with none skips the multiply-adds).
// ---------------------------------------------------------------------------

// Part 0 epilogue (Eq. 1 as in lv3_epilogue): a lane's two columns are pairs
// (i, j) with their own j, so n2(j, k) is gathered per element like n2(i, k);
// 2 s_k of the tile's rows is staged in LDS.  Stores go through a buffer
// resource from the tile's first entry (0, jmin, k0) to the end of the last
// pair's slab; an element outside i < j < k < n_v gets an offset past it.
template <bool F32>
__device__ __forceinline__ void lvs_epilogue0(const LvArgs& a, const v16i_t (&acc)[4][2],
                                              int64_t p0, int64_t k0, int wr, int wc,
                                              bool active, int8_t* lds) {
    using R = typename std::conditional<F32, float, double>::type;
    constexpr int TB = kMB, WN = 2, WM = 4;
    const int lane = threadIdx.x % 64;
    const int64_t n = a.n_v;
    const double* __restrict__ S = a.s;
    const int32_t* __restrict__ N2 = a.n2;
    R* rs2 = (R*)lds;   // 2 s_k
    if (threadIdx.x < TB) {
        const int64_t k = k0 + threadIdx.x;
        rs2[threadIdx.x] = k < n ? (R)(2.0 * S[k]) : (R)0;
    }
    __syncthreads();
    if (!active) return;
    const int64_t pe = a.r_end[0];
    const int64_t jmin = pair_j(p0);
    const int64_t jlast = pair_j(p0 + TB - 1 < pe ? p0 + TB - 1 : pe - 1);
    const int64_t ob = slab_offset(n, a.j_begin);
    const int64_t base0 = slab_offset(n, jmin) - ob + (k0 - jmin - 1) * jmin;
    const __amdgpu_buffer_rsrc_t rc3 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.c3 + base0), (short)0, (int)((slab_offset(n, jlast + 1) - ob - base0) * 4),
        kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rn2 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)N2, (short)0, (int)(n * (n - 1) / 2 * 4), kRsrcWord3);
    R ls2[WN];            // 2 (s_i + s_j)
    uint32_t nij[WN];     // n2(i, j)
    int ii[WN], jj[WN];   // the column's pair; jj = n_v when past the part
    uint32_t sb[WN];      // entry (i, j, k) - base0 = sb + k j (mod 2^32)
#pragma unroll
    for (int nn = 0; nn < WN; ++nn) {
        const int64_t p = p0 + wc + nn * 32 + lane % 32;
        const bool vp = p < pe;
        const int64_t pp = vp ? p : pe - 1;
        const int64_t j = pair_j(pp), i = pp - j * (j - 1) / 2;
        ls2[nn] = (R)2 * ((R)S[i] + (R)S[j]);
        nij[nn] = (uint32_t)N2[pp];
        ii[nn] = (int)i;
        jj[nn] = vp ? (int)j : (int)n;
        sb[nn] = (uint32_t)(slab_offset(n, j) - ob - base0 - (j + 1) * j + i);
    }
    constexpr int RB = 4, NB = WM * 16 / RB;
    auto row_dk = [&](int b, int q) {
        const int m = b / (16 / RB), r = (b % (16 / RB)) * RB + q;
        return wr + m * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
    };
    struct Batch {
        uint32_t nik[RB][WN], njk[RB][WN];
    };
    const int kb = (int)k0;
    auto load_batch = [&](int b, Batch& o) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const uint32_t k = (uint32_t)(kb + row_dk(b, q));
            const uint32_t ck = (k * (k - 1)) >> 1;   // k < 2^16: the table is below 2^31 bytes
#pragma unroll
            for (int nn = 0; nn < WN; ++nn) {
                o.nik[q][nn] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                    rn2, (int)((ck + (uint32_t)ii[nn]) * 4), 0, 0);
                o.njk[q][nn] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                    rn2, (int)((ck + (uint32_t)jj[nn]) * 4), 0, 0);
            }
        }
    };
    auto store_batch = [&](int b, const Batch& o) {
        const int m = b / (16 / RB);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = (b % (16 / RB)) * RB + q;
            const int dk = row_dk(b, q);
            const int k = kb + dk;
            const R rk = rs2[dk];
#pragma unroll
            for (int nn = 0; nn < WN; ++nn) {
                const bool ok = k > jj[nn] && k < (int)n;
                const uint32_t n3 = nij[nn] + o.nik[q][nn] + o.njk[q][nn] - (uint32_t)acc[m][nn][r];
                const R d = ls2[nn] + rk;
                const R dd = d > (R)0 ? d : (R)1;
                float qv;
                if constexpr (F32)
                    qv = div_u24((float)(3u * n3), dd);
                else
                    qv = (float)((3.0 * (double)n3) / dd);
                const float c = d > (R)0 ? qv : 0.0f;
                const uint32_t off = ok ? (sb[nn] + __umul24((uint32_t)k, (uint32_t)jj[nn])) * 4u
                                        : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, c), rc3,
                                                      (int)off, 0, 0);
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

// Part 1 epilogue (TB rows): a row is a pair (j, k); its 2 (s_j + s_k), n2(j, k), the
// pair-table offsets of rows j and k, j and its output row offset are staged
// in LDS once per tile; n2(i, j) and n2(i, k) are gathered per element
// (contiguous in i).  Stores from the tile's first pair's entry i = 0 to the
// end of the last pair's slab; columns i >= j get an offset past it.
template <bool F32, int TB>
__device__ __forceinline__ void lvs_epilogue1(const LvArgs& a, const v16i_t (&acc)[4][2],
                                              int64_t q0, int64_t i0, int wr, int wc,
                                              bool active, int8_t* lds) {
    using R = typename std::conditional<F32, float, double>::type;
    constexpr int WN = 2, WM = 4;   // TB rows (pairs) from q0
    const int lane = threadIdx.x % 64;
    const int64_t n = a.n_v;
    const double* __restrict__ S = a.s;
    const int32_t* __restrict__ N2 = a.n2;
    const int64_t qe = a.r_end[1];
    const int64_t ob = slab_offset(n, a.j_begin);
    int64_t jf, kf, jl, kl;
    lex_pair(n, q0 < qe ? q0 : qe - 1, jf, kf);   // (a half past the part stores nothing)
    lex_pair(n, q0 + TB - 1 < qe ? q0 + TB - 1 : qe - 1, jl, kl);
    const int64_t base0 = slab_offset(n, jf) - ob + (kf - jf - 1) * jf;
    int4* rowi = (int4*)lds;                         // {c(j), c(k), j, output row offset}
    R* rs2 = (R*)(lds + TB * sizeof(int4));           // 2 (s_j + s_k)
    int32_t* rnj = (int32_t*)(lds + TB * (sizeof(int4) + sizeof(R)));   // n2(j, k)
    if (threadIdx.x < TB) {
        const int64_t q = q0 + threadIdx.x;
        const bool vq = q < qe;
        int64_t j, k;
        lex_pair(n, vq ? q : qe - 1, j, k);
        const int64_t cj = j * (j - 1) / 2, ck = k * (k - 1) / 2;
        rowi[threadIdx.x] = make_int4((int)cj, (int)ck, vq ? (int)j : 0,
                                      (int)(slab_offset(n, j) - ob + (k - j - 1) * j - base0));
        rs2[threadIdx.x] = (R)2 * ((R)S[j] + (R)S[k]);
        rnj[threadIdx.x] = N2[ck + j];
    }
    __syncthreads();
    if (!active) return;
    const __amdgpu_buffer_rsrc_t rc3 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.c3 + base0), (short)0, (int)((slab_offset(n, jl + 1) - ob - base0) * 4),
        kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rn2 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)N2, (short)0, (int)(n * (n - 1) / 2 * 4), kRsrcWord3);
    R ls[WN];        // 2 s_i
    int ii[WN];
#pragma unroll
    for (int nn = 0; nn < WN; ++nn) {
        const int64_t i = i0 + wc + nn * 32 + lane % 32;
        ls[nn] = (R)(2.0 * S[i < n ? i : n - 1]);
        ii[nn] = (int)i;
    }
    constexpr int RB = 4, NB = WM * 16 / RB;
    auto row_dk = [&](int b, int q) {
        const int m = b / (16 / RB), r = (b % (16 / RB)) * RB + q;
        return wr + m * 32 + (r / 4) * 8 + (lane / 32) * 4 + (r % 4);
    };
    struct Batch {
        uint32_t nij[RB][WN], nik[RB][WN];
        int4 ri[RB];
    };
    auto load_batch = [&](int b, Batch& o) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int4 ri = rowi[row_dk(b, q)];
            o.ri[q] = ri;
#pragma unroll
            for (int nn = 0; nn < WN; ++nn) {
                o.nij[q][nn] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                    rn2, (int)(((uint32_t)ri.x + (uint32_t)ii[nn]) * 4), 0, 0);
                o.nik[q][nn] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                    rn2, (int)(((uint32_t)ri.y + (uint32_t)ii[nn]) * 4), 0, 0);
            }
        }
    };
    auto store_batch = [&](int b, const Batch& o) {
        const int m = b / (16 / RB);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = (b % (16 / RB)) * RB + q;
            const int dk = row_dk(b, q);
            const R rr = rs2[dk];
            const uint32_t njk = (uint32_t)rnj[dk];
            const int4 ri = o.ri[q];
#pragma unroll
            for (int nn = 0; nn < WN; ++nn) {
                const bool ok = ii[nn] < ri.z;
                const uint32_t n3 = o.nij[q][nn] + o.nik[q][nn] + njk - (uint32_t)acc[m][nn][r];
                const R d = ls[nn] + rr;
                const R dd = d > (R)0 ? d : (R)1;
                float qv;
                if constexpr (F32)
                    qv = div_u24((float)(3u * n3), dd);
                else
                    qv = (float)((3.0 * (double)n3) / dd);
                const float c = d > (R)0 ? qv : 0.0f;
                const uint32_t off =
                    ok ? ((uint32_t)ri.w + (uint32_t)ii[nn]) * 4u : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, c), rc3,
                                                      (int)off, 0, 0);
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

// Half h of tile t of part PART of the split tiling: part 0's output columns
// (pairs) 128 h .. 128 h + 127, part 1's output rows (pairs) likewise; four
// waves of 128 x 64, two workgroups per CU (the epilogue and barriers of
// one overlap the other's multiply-adds).
template <int PART, bool ALIGNED, int LC, int MODE>
__device__ __forceinline__ void lvs_tile(const LvArgs& a, int64_t t, int h, int8_t* lds) {
    constexpr int TB = kMB, WN = 2;
    constexpr int HB = TB / 2;   // output columns of a half tile
    using GA = LvGeom<256, TB>;
    using GB = LvGeom<256, HB>;
    // row tile: the largest rt with prefix[rt] <= t
    const int64_t* pre = a.pre[PART];
    int64_t lo = 0, hi = a.nrt[PART];
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    const int64_t ct = t - pre[lo];
    const int64_t n = a.n_v;
    const int64_t r0 = a.r_begin[PART] + lo * TB, re = a.r_end[PART];
    const int wave = threadIdx.x / 64;
    const int wr = (wave % 2) * (TB / 2);   // the wave's output rows
    const int wl = (wave / 2) * 32 * WN;    // its output columns in the half (LDS rows)
    const int wc = h * HB + wl;             // ... in the tile
    v16i_t acc[4][WN];
    if constexpr (PART == 0) {
        const int64_t k0 = pair_j(r0) + 1 + ct * TB;
        const int64_t pq = r0 + wc;
        const int64_t kq = k0 + wr + TB / 2 - 1 < n - 1 ? k0 + wr + TB / 2 - 1 : n - 1;
        const bool active = k0 + wr < n && pq < re && pair_j(pq) < kq;
        LvRows<GA, ALIGNED, MODE, false> sa(a, k0, 0);
        LvPairs<GB, ALIGNED, MODE> sb(a, [&](int r, int64_t& x, int64_t& y) {
            const int64_t p = r0 + h * HB + r < re ? r0 + h * HB + r : re - 1;
            y = pair_j(p);
            x = p - y * (y - 1) / 2;
        });
        lv_tile_sb<WN, ALIGNED, LC, MODE>(a, sa, sb, active, wr, wl, acc, lds);
        if (a.f32div)
            lvs_epilogue0<true>(a, acc, r0, k0, wr, wc, active, lds);
        else
            lvs_epilogue0<false>(a, acc, r0, k0, wr, wc, active, lds);
    } else {
        // the halves split the rows (pairs), so no pair row is staged twice;
        // the four waves take 64 of the 256 columns each
        const int64_t i0 = ct * TB;
        const int64_t qa = r0 + h * HB;
        const int64_t qz = qa + HB - 1 < re ? qa + HB - 1 : re - 1;
        const int wi = wave * 32 * WN;
        int64_t jz, kz;
        lex_pair(n, qz, jz, kz);
        const bool active = qa < re && i0 + wi < jz;
        LvPairs<LvGeom<256, HB>, ALIGNED, MODE> sa(a, [&](int r, int64_t& x, int64_t& y) {
            lex_pair(n, qa + r < re ? qa + r : re - 1, x, y);
        });
        LvRows<LvGeom<256, TB>, ALIGNED, MODE, false> sb(a, i0, 0);
        lv_tile_sb<WN, ALIGNED, LC, MODE>(a, sa, sb, active, 0, wi, acc, lds);
        if (a.f32div)
            lvs_epilogue1<true, HB>(a, acc, qa, i0, 0, wi, active, lds);
        else
            lvs_epilogue1<false, HB>(a, acc, qa, i0, 0, wi, active, lds);
    }
}

// Both parts in one launch (one tail instead of two): work item t2 is half
// t2 % 2 of tile t2 / 2; tiles [0, nt[0]) are part 0's, the rest part 1's.
template <bool ALIGNED, int LC, int MODE>
__global__ __launch_bounds__(256, 2) void ps_mfma3_lvs_kernel(LvArgs a) {
    __shared__ __attribute__((aligned(16))) int8_t lds[(kMB + kMB / 2) * (kLvMK + kPad)];
    const int64_t t2 = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                       blockIdx.x / kXcds;
    if (t2 >= 2 * a.ntiles) return;
    const int64_t t = t2 / 2;
    const int h = (int)(t2 % 2);
    if (t < a.nt[0])
        lvs_tile<0, ALIGNED, LC, MODE>(a, t, h, lds);
    else
        lvs_tile<1, ALIGNED, LC, MODE>(a, t - a.nt[0], h, lds);
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

// 2-way half tiles with LDS-direct staging (rows 16-byte aligned, n_f a
// multiple of kLvdMK): stages of kLvdMK fields of the tile's 384 rows (256 j
// rows, then 128 i rows) go from global memory straight into a ring of
// kLvdStages LDS slots (global_load_lds_dwordx4: one wave instruction fills
// 1 KB, 16 rows of 64 bytes, lane l at byte 16 l), two stages ahead of the
// multiply-adds, so no registers hold staged data and the fragment reads of
// the next k-step are in flight while a k-step runs.  16-byte chunk c of
// row r sits at chunk position c ^ lvd_swz(r).  Rows past n_v load row
// n_v - 1 (their outputs are never stored).  One barrier per stage.
constexpr int kLvdMK = 64;
constexpr int kLvdStages = 3;

// Chunk swizzle of 64-byte rows: for every chunk c, the slots of any 8
// consecutive rows are distinct modulo 128 bytes and those of any 16
// consecutive rows distinct modulo 256 bytes (b128 fragment reads free of
// bank conflicts whether the LDS serves 8 or 16 lanes at once); rows r and
// r + 32 share a swizzle.
__device__ __forceinline__ int lvd_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// This wave's stage loads but the N most recent have landed and its LDS
// accesses are done, then the barrier; the empty asm statements keep the
// compiler from moving memory accesses across.
template <int N>
__device__ __forceinline__ void lvd_sync() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (0x7 << 4) | ((N >> 4) << 14));   // lgkmcnt 0
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One kLvdMK-field stage of a wave's 128 x 64 block: A rows wr + 0..127 and
// B rows wc + 0..63 of LDS regions of 64-byte rows in the lvd_swz layout
// (wr, wc multiples of 32); the fragments of the second k-step are read
// while the first runs.  mid() (the loads of a later stage) is issued
// between the two k-steps, behind the first one's multiply-adds, so that
// neither the stage's first fragment reads nor its first multiply-adds wait
// behind the load issue (measured against issuing at the top of the stage:
// 2-way 7.96 -> 7.74 ms, 3-way 1.75 -> 1.71 ms; after the first fragment
// reads, 3-way 1.79 -> 1.75 ms and the 2-way unchanged).
template <int LC, int MODE, class MID>
__device__ __forceinline__ void lvd_stage(const int8_t* A, const int8_t* B, int wr, int wc, int L,
                                          v16i_t (&acc)[4][2], MID mid) {
    constexpr int MK = kLvdMK, WM = 4, WN = 2, KS = MK / 32;
    const int lane = threadIdx.x % 64;
    const int fr = lane % 32, hk = lane / 32;
    const int sw = lvd_swz(fr);   // the swizzle of rows wr + m 32 + fr and wc + n 32 + fr
    auto frag = [&](int ks, v4i_t (&fa)[WM], v4i_t (&fb)[WN]) {
        const int co = ((ks * 2 + hk) ^ sw) * 16;
#pragma unroll
        for (int m = 0; m < WM; ++m) fa[m] = *(const v4i_t*)(A + (wr + m * 32 + fr) * MK + co);
#pragma unroll
        for (int n = 0; n < WN; ++n) fb[n] = *(const v4i_t*)(B + (wc + n * 32 + fr) * MK + co);
        if constexpr (MODE == kLvSub) {   // the subtraction form wants bit 7 set
            const int h = (int)0x80808080u;
#pragma unroll
            for (int m = 0; m < WM; ++m) fa[m] |= h;
#pragma unroll
            for (int n = 0; n < WN; ++n) fb[n] |= h;
        }
    };
    auto level = [&](const v4i_t (&fa)[WM], const v4i_t (&fb)[WN], int t) {
        v4i_t xa[WM], xb[WN];
        if constexpr (MODE == kLvPerm) {
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
                acc[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa[m], xb[n], acc[m][n], 0, 0, 0);
    };
    v4i_t fa[2][WM], fb[2][WN];
    frag(0, fa[0], fb[0]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        if (ks + 1 < KS) frag(ks + 1, fa[(ks + 1) & 1], fb[(ks + 1) & 1]);
#pragma unroll(LC > 0 ? LC : 1)
        for (int t = 1; t <= L; ++t) level(fa[ks & 1], fb[ks & 1], t);
        if (ks == 0) {
            asm volatile("" ::: "memory");
            mid();
            asm volatile("" ::: "memory");
        }
    }
}

template <int LC, int MODE>
__global__ __launch_bounds__(256, 2) void ps_mfma2_lvd_kernel(LvArgs a) {
    constexpr int MK = kLvdMK;
    constexpr int kRowsA = kMB;                      // j rows; the i rows follow
    constexpr int kRows = kMB + kMB / 2;
    constexpr int kStageBytes = kRows * MK;
    constexpr int NU = kStageBytes / 1024 / 4;       // wave instructions per stage
    constexpr int WM = 4, WN = 2;
    static_assert(NU * 4 * 1024 == kStageBytes, "stage split");
    __shared__ __attribute__((aligned(1024))) int8_t lds[kLvdStages * kStageBytes];
    const int64_t t2 = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                       blockIdx.x / kXcds;
    if (t2 >= 2 * a.ntiles) return;
    int64_t bi, bj;
    grouped_tri_decode_rt(t2 / 2, a.nb, a.group, bi, bj);
    const int64_t i0 = bi * kMB + (t2 % 2) * (kMB / 2), j0 = bj * kMB;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wr = (wave % 2) * 128;        // j offset of the wave's block (A rows)
    const int wc = (wave / 2) * 32 * WN;    // i offset (B rows)
    const bool active = (i0 + wc < a.n_v) && (j0 + wr < a.n_v) && (i0 + wc + 1 < j0 + wr + 128);
    const uint8_t* src[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int row = (wave + 4 * u) * 16 + lane / 4;
        const int c = (lane % 4) ^ lvd_swz(row);
        int64_t g = row < kRowsA ? j0 + row : i0 + (row - kRowsA);
        if (g >= a.n_v) g = a.n_v - 1;
        src[u] = a.V + g * a.ld + c * 16;
    }
    auto issue = [&](int64_t s, int slot) {
#pragma unroll
        for (int u = 0; u < NU; ++u)
            __builtin_amdgcn_global_load_lds(
                (const void*)(src[u] + s * MK),
                (void*)(lds + slot * kStageBytes + (wave + 4 * u) * 1024), 16, 0, 0);
    };
    v16i_t acc[WM][WN];
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) acc[m][n] = (v16i_t){};
    const int L = LC > 0 ? LC : a.levels;
    auto compute = [&](int slot, auto mid) {
        const int8_t* A = lds + slot * kStageBytes;
        lvd_stage<LC, MODE>(A, A + kRowsA * MK, wr, wc, L, acc, mid);
    };
    const int64_t ns = a.n_f / MK;
    issue(0, 0);
    if (ns > 1) issue(1, 1);
    int slot = 0;
    for (int64_t s = 0; s < ns; ++s) {
        // stage s landed everywhere; slot (s + 2) % 3 (stage s - 1) no longer read
        if (s + 1 < ns)
            lvd_sync<NU>();
        else
            lvd_sync<0>();
        const int sn = slot == 0 ? 2 : slot - 1;
        auto mid = [&]() {
            if (s + 2 < ns) issue(s + 2, sn);
        };
        if (active)
            compute(slot, mid);
        else
            mid();
        slot = slot == 2 ? 0 : slot + 1;
    }
    if constexpr (MODE == kLvSub) {
#pragma unroll
        for (int m = 0; m < WM; ++m)
#pragma unroll
            for (int n = 0; n < WN; ++n)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[m][n][r] = -acc[m][n][r] >> 7;
    }
    if (!active) return;
    MfmaArgs e{};
    e.n_v = a.n_v;
    e.s = a.s;
    e.c2 = a.c2;
    e.n2 = a.n2;
    if (a.f32div)
        mfma_epilogue<WN, true>(acc, e, i0, j0, wr, wc, lane);
    else
        mfma_epilogue<WN>(acc, e, i0, j0, wr, wc, lane);
}

// Half h of tile t of part PART of the split tiling with LDS-direct stages
// (rows 16-byte aligned, n_f a multiple of kLvdMK): the tiles, waves and
// epilogues of lvs_tile, with the half's 256 plain rows (part 0: the k rows,
// part 1: the i rows) loaded straight into a ring of kLvdStages LDS slots
// and its 128 pair rows formed in registers (bytewise mins) and written into
// the same slots, both two stages ahead of the multiply-adds.  A slot holds
// the plain rows, then the pair rows, 64 bytes each in the lvd_swz layout.
// Plain rows past n_v load row n_v - 1 (their outputs are never stored).
// Per stage: the pair loads, then the plain-row loads of stage s + 2 are
// issued, stage s runs, the pair rows go to LDS once their loads (all but
// the newest plain-row loads) have landed, and a barrier.
template <int PART, int LC, int MODE>
__device__ __forceinline__ void lvsd_tile(const LvArgs& a, int64_t t, int h, int8_t* lds) {
    constexpr int TB = kMB, WN = 2, HB = TB / 2, MK = kLvdMK;
    constexpr int kStageBytes = (TB + HB) * MK;
    constexpr int NU = TB * MK / 1024 / 4;   // plain-row wave instructions per stage
    constexpr int NP = HB * MK / 16 / 256;   // pair-row chunks per thread per stage
    static_assert(NU * 4 * 1024 == TB * MK && NP * 256 * 16 == HB * MK, "stage split");
    const int64_t* pre = a.pre[PART];
    int64_t lo = 0, hi = a.nrt[PART];
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    const int64_t ct = t - pre[lo];
    const int64_t n = a.n_v;
    const int64_t r0 = a.r_begin[PART] + lo * TB, re = a.r_end[PART];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    int64_t g0;        // first plain row
    int64_t k0 = 0, i0 = 0, qa = 0;
    int wr, wl, wc;    // the wave's A rows, B rows (LDS) and output columns in the tile
    bool active;
    int ox[NP], oy[NP];
    auto pair_offsets = [&](auto pair) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            const int q = (int)threadIdx.x + 256 * c;
            int64_t x, y;
            pair(q / 4, x, y);
            ox[c] = (int)(x * a.ld) + (q % 4) * 16;
            oy[c] = (int)(y * a.ld) + (q % 4) * 16;
        }
    };
    if constexpr (PART == 0) {
        k0 = pair_j(r0) + 1 + ct * TB;
        g0 = k0;
        wr = (wave % 2) * (TB / 2);
        wl = (wave / 2) * 32 * WN;
        wc = h * HB + wl;
        const int64_t pq = r0 + wc;
        const int64_t kq = k0 + wr + TB / 2 - 1 < n - 1 ? k0 + wr + TB / 2 - 1 : n - 1;
        active = k0 + wr < n && pq < re && pair_j(pq) < kq;
        pair_offsets([&](int r, int64_t& x, int64_t& y) {
            const int64_t p = r0 + h * HB + r < re ? r0 + h * HB + r : re - 1;
            y = pair_j(p);
            x = p - y * (y - 1) / 2;
        });
    } else {
        i0 = ct * TB;
        g0 = i0;
        qa = r0 + h * HB;
        const int64_t qz = qa + HB - 1 < re ? qa + HB - 1 : re - 1;
        wr = 0;
        wl = wave * 32 * WN;
        wc = wl;
        int64_t jz, kz;
        lex_pair(n, qz, jz, kz);
        active = qa < re && i0 + wl < jz;
        pair_offsets([&](int r, int64_t& x, int64_t& y) {
            lex_pair(n, qa + r < re ? qa + r : re - 1, x, y);
        });
    }
    const uint8_t* src[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int row = (wave + 4 * u) * 16 + lane / 4;
        const int c = (lane % 4) ^ lvd_swz(row);
        const int64_t g = g0 + row < n ? g0 + row : n - 1;
        src[u] = a.V + g * a.ld + c * 16;
    }
    int pd[NP];   // LDS byte offsets of this thread's pair chunks within a slot
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const int q = (int)threadIdx.x + 256 * c, r = q / 4;
        pd[c] = (TB + r) * MK + ((q % 4) ^ lvd_swz(r)) * 16;
    }
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.V, (short)0, (int)(n * a.ld), kRsrcWord3);
    uint4 px[NP], py[NP];
    auto pload = [&](int64_t s) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            px[c] = lv_load16<true>(rs, ox[c] + (int)s * MK);
            py[c] = lv_load16<true>(rs, oy[c] + (int)s * MK);
        }
    };
    auto dma = [&](int64_t s, int slot) {
#pragma unroll
        for (int u = 0; u < NU; ++u)
            __builtin_amdgcn_global_load_lds(
                (const void*)(src[u] + s * MK),
                (void*)(lds + slot * kStageBytes + (wave + 4 * u) * 1024), 16, 0, 0);
    };
    auto issue = [&](int64_t s, int slot) {
        pload(s);
        asm volatile("" ::: "memory");   // pair loads first: their wait leaves the DMA in flight
        dma(s, slot);
    };
    auto pstore = [&](int slot) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            const uint4 x = lv_prep<MODE>(px[c], 16), y = lv_prep<MODE>(py[c], 16);
            *(uint4*)(lds + slot * kStageBytes + pd[c]) =
                make_uint4(lv_min<MODE>(x.x, y.x), lv_min<MODE>(x.y, y.y),
                           lv_min<MODE>(x.z, y.z), lv_min<MODE>(x.w, y.w));
        }
    };
    v16i_t acc[4][WN];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int nn = 0; nn < WN; ++nn) acc[m][nn] = (v16i_t){};
    const int L = LC > 0 ? LC : a.levels;
    const int64_t ns = a.n_f / MK;
    issue(0, 0);
    pstore(0);
    if (ns > 1) {
        issue(1, 1);
        pstore(1);
    }
    // stage s: stage s complete everywhere and slot (s + 2) % 3 (stage
    // s - 1) no longer read, then stage s + 2 in flight while s runs (one loop
    // for waves with work, one for the rest: a branch inside the loop makes
    // the accumulators spill)
    auto run = [&](auto compute) {
        int slot = 0;
        for (int64_t s = 0; s < ns; ++s) {
            if (s + 1 < ns)
                lvd_sync<NU>();
            else
                lvd_sync<0>();
            const int sn = slot == 0 ? 2 : slot - 1;
            compute(slot, [&]() {
                if (s + 2 < ns) issue(s + 2, sn);
            });
            if (s + 2 < ns) pstore(sn);
            slot = slot == 2 ? 0 : slot + 1;
        }
    };
    if (active)
        run([&](int slot, auto mid) {
            const int8_t* P = lds + slot * kStageBytes;   // plain rows
            const int8_t* Q = P + TB * MK;                 // pair rows
            if constexpr (PART == 0)
                lvd_stage<LC, MODE>(P, Q, wr, wl, L, acc, mid);
            else
                lvd_stage<LC, MODE>(Q, P, wr, wl, L, acc, mid);
        });
    else
        run([](int, auto mid) { mid(); });
    if constexpr (MODE == kLvSub) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nn = 0; nn < WN; ++nn)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[m][nn][r] = -acc[m][nn][r] >> 7;
    }
    // the epilogue's row data goes to slot (ns + 1) % 3, last read by stage
    // ns - 2 before the barrier of stage ns - 1
    int8_t* ep = lds + (int)((ns + 1) % 3) * kStageBytes;
    if constexpr (PART == 0) {
        if (a.f32div)
            lvs_epilogue0<true>(a, acc, r0, k0, wr, wc, active, ep);
        else
            lvs_epilogue0<false>(a, acc, r0, k0, wr, wc, active, ep);
    } else {
        if (a.f32div)
            lvs_epilogue1<true, HB>(a, acc, qa, i0, 0, wl, active, ep);
        else
            lvs_epilogue1<false, HB>(a, acc, qa, i0, 0, wl, active, ep);
    }
}

template <int LC, int MODE>
__global__ __launch_bounds__(256, 2) void ps_mfma3_lvsd_kernel(LvArgs a) {
    __shared__ __attribute__((aligned(1024))) int8_t lds[kLvdStages * (kMB + kMB / 2) * kLvdMK];
    const int64_t t2 = a.item0 + (int64_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) +
                       blockIdx.x / kXcds;
    if (t2 >= 2 * a.ntiles) return;
    const int64_t t = t2 / 2;
    const int h = (int)(t2 % 2);
    if (t < a.nt[0])
        lvsd_tile<0, LC, MODE>(a, t, h, lds);
    else
        lvsd_tile<1, LC, MODE>(a, t - a.nt[0], h, lds);
}

template <bool ALIGNED, int LC, int MODE>
static hipError_t go_mfma2_lv(const MfmaLaunch& m, hipStream_t st) {
    LvArgs a = lv_args(m);
    a.f32div = 2 * (int64_t)m.levels * m.n_f < ((int64_t)1 << 24);   // 2 n2 and s_i + s_j
    a.nb = (m.n_v + kMB - 1) / kMB;
    a.ntiles = a.nb * (a.nb + 1) / 2;
    if (ALIGNED && m.n_f >= kLvdMK && m.n_f % kLvdMK == 0) {
        auto go = [&](auto lc) {
            return launch_items(2 * a.ntiles, 256, kXcds, [&](unsigned grid, int64_t item0) {
                LvArgs b = a;
                b.item0 = item0;
                hipLaunchKernelGGL((ps_mfma2_lvd_kernel<decltype(lc)::value, MODE>), dim3(grid),
                                   dim3(256), 0, st, b);
            });
        };
        // one instantiation per level count up to 7 (a compile-time level
        // loop: 2 levels 6.81 -> 6.19 ms, 5 levels 12.40 -> 10.89 ms on
        // levels_8192x32768 capped at that many levels)
        if constexpr (MODE == kLvPerm) {
            switch (m.levels) {
            case 1: return go(std::integral_constant<int, 1>{});
            case 2: return go(std::integral_constant<int, 2>{});
            case 3: return go(std::integral_constant<int, 3>{});
            case 4: return go(std::integral_constant<int, 4>{});
            case 5: return go(std::integral_constant<int, 5>{});
            case 6: return go(std::integral_constant<int, 6>{});
            default: return go(std::integral_constant<int, 7>{});
            }
        } else {
            return go(std::integral_constant<int, LC>{});
        }
    }
    return launch_items(2 * a.ntiles, 256, kXcds, [&](unsigned grid, int64_t item0) {
        LvArgs b = a;
        b.item0 = item0;
        hipLaunchKernelGGL((ps_mfma2_lv_kernel<2, ALIGNED, LC, MODE>), dim3(grid), dim3(256), 0,
                           st, b);
    });
}


// The split tiling (split3): part 0 over the colex pairs of slabs
// [j_begin, js), part 1 over the lex pairs of slabs [js, j_end), in one
// launch, each part with the prefix of its row tiles' column-tile counts
// (part 1's after part 0's in the prefix workspace).
template <bool ALIGNED, int LC, int MODE>
static hipError_t go_mfma3_lvs(const MfmaLaunch& m, hipStream_t st) {
    const int64_t n = m.n_v, jb = m.j_begin, je = m.j_end, js = split3(n, jb, je);
    LvArgs a = lv_args(m);   // a.n2: the pair numerators of Eq. 1
    a.j_begin = jb;
    a.j_end = je;
    a.f32div = 6 * (int64_t)m.levels * m.n_f < ((int64_t)1 << 24);
    a.c3 = (uint32_t*)m.c3;
    a.nrt[0] = flat_row_tiles(jb, js, kMB);
    a.nrt[1] = lex_row_tiles(n, js, je, kMB);
    a.pre[0] = m.prefix;
    a.pre[1] = m.prefix + a.nrt[0] + 1;
    a.r_begin[0] = jb * (jb - 1) / 2;
    a.r_end[0] = js * (js - 1) / 2;
    a.r_begin[1] = lex_first(n, js);
    a.r_end[1] = lex_first(n, je);
    a.nt[0] = a.nrt[0] > 0 ? flat_tiles(n, jb, js, kMB) : 0;
    a.nt[1] = a.nrt[1] > 0 ? lex_tiles(n, js, je, kMB) : 0;
    hipError_t e = launch_prefix3_split(n, jb, js, je, kMB, m.prefix, m.prefix + a.nrt[0] + 1, st);
    if (e != hipSuccess) return e;
    a.ntiles = a.nt[0] + a.nt[1];
    // LDS-direct stages for 1..7 levels, one instantiation per level count
    // (with the count known only at run time the level loop spills the
    // accumulators in that kernel; more levels keep the register-staged one)
    if constexpr (ALIGNED && MODE == kLvPerm) {
        if (m.n_f >= kLvdMK && m.n_f % kLvdMK == 0 && m.levels >= 1 && m.levels <= 7) {
            auto go = [&](auto lc) {
                return launch_items(2 * a.ntiles, 256, kXcds, [&](unsigned grid, int64_t item0) {
                    LvArgs b = a;
                    b.item0 = item0;
                    hipLaunchKernelGGL((ps_mfma3_lvsd_kernel<decltype(lc)::value, kLvPerm>),
                                       dim3(grid), dim3(256), 0, st, b);
                });
            };
            switch (m.levels) {
            case 1: return go(std::integral_constant<int, 1>{});
            case 2: return go(std::integral_constant<int, 2>{});
            case 3: return go(std::integral_constant<int, 3>{});
            case 4: return go(std::integral_constant<int, 4>{});
            case 5: return go(std::integral_constant<int, 5>{});
            case 6: return go(std::integral_constant<int, 6>{});
            default: return go(std::integral_constant<int, 7>{});
            }
        }
    }
    return launch_items(2 * a.ntiles, 256, kXcds, [&](unsigned grid, int64_t item0) {
        LvArgs b = a;
        b.item0 = item0;
        hipLaunchKernelGGL((ps_mfma3_lvs_kernel<ALIGNED, LC, MODE>), dim3(grid), dim3(256), 0,
                           st, b);
    });
}

template <bool ALIGNED, int LC, int MODE>
static hipError_t go_mfma3_lv(const MfmaLaunch& m, hipStream_t st) {
    if (!m.slab3 && mfma3_split_ok(m.n_v, m.ld)) return go_mfma3_lvs<ALIGNED, LC, MODE>(m, st);
    constexpr int kEdge = kMB / 2;
    hipError_t e = launch_prefix3(m.n_v, m.j_begin, m.j_end, kMB, kSlabFull, kMB, m.prefix, st);
    if (e == hipSuccess)
        e = launch_prefix3(m.n_v, m.j_begin, m.j_end, kEdge, kSlabEdge, kMB, m.edge_prefix, st);
    if (e != hipSuccess) return e;
    LvArgs a = lv_args(m);   // a.n2: the pair numerators of Eq. 1
    a.j_begin = m.j_begin;
    a.j_end = m.j_end;
    a.f32div = 6 * (int64_t)m.levels * m.n_f < ((int64_t)1 << 24);
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
// table lookups for levels <= 7, the subtraction form above.  Three levels
// are a compile-time count throughout; the LDS-direct kernels (aligned rows,
// n_f a multiple of 64) take a compile-time count for every level count up
// to 7, the register-staged kernels a run-time one.
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
// (it is kept for int8 planes); on fp4 this one is.  (The fused int8 level
// tiles have an LDS-direct form of their own, ps_mfma2_lvd_kernel.)
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

// ps_internal.h -- declarations shared by the libps translation units.
// Not installed; the public interface is include/ps.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ps.h"

namespace ps {

constexpr int kThreads = 256;        // threads per workgroup of the tile kernels
constexpr int kXcds = 8;             // MI355X: 8 accelerator complex dies

// Record an error message for ps_last_error() and return `st`.
ps_status fail(ps_status st, const char* fmt, ...);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Element size in bytes of a storage type (0 if unknown).
inline int elem_size(int32_t dt) {
    return dt == PS_F32 ? 4 : dt == PS_F16 ? 2 : dt == PS_U8 ? 1 : dt == PS_F64 ? 8 : 0;
}

// Blocks of one launch: the dispatch size in work-items is a 32-bit number,
// so a launch holds at most (2^32 - 1) / threads blocks; the result is also
// a multiple of `multiple` (the block-to-work remaps need whole rounds of
// XCDs).  The environment variable PS_MAX_GRID_BLOCKS, read once, lowers the
// cap (a testing aid: it makes small problems take the multi-launch path).
int64_t max_grid_blocks(int threads, int64_t multiple);

// Launches `total` work items, one block each, in as few launches as the
// dispatch size allows; launch(grid, item0) enqueues one of them.  Every grid
// is a multiple of `multiple`.
template <class Launch>
hipError_t launch_items(int64_t total, int threads, int64_t multiple, Launch launch) {
    const int64_t cap = max_grid_blocks(threads, multiple);
    for (int64_t item0 = 0; item0 < total; item0 += cap) {
        const int64_t left = total - item0;
        const int64_t grid = left < cap ? ceil_div(left, multiple) * multiple : cap;
        launch((unsigned)grid, item0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


// Internal operand type of the BITS path (never a public ps_dtype): binary
// data packed 32 fields to a 32-bit word, bit e of word w = field 32 w + e.
constexpr int32_t PS_B1 = 4;
constexpr int kBitsPerWord = 32;
// Bytes of the words the VALU tile kernels stage and compute on: 8 for
// FP64 (one element), 4 otherwise (1, 2 or 4 elements, or 32 packed bits).
inline int word_bytes(int32_t dt) { return dt == PS_F64 ? 8 : 4; }
// Packed row length in words: whole 16-byte chunks.
inline int64_t bits_row_words(int64_t n_f) { return ceil_div(ceil_div(n_f, kBitsPerWord), 4) * 4; }

// Offset of the first triple of slab j in the j-slab layout:
// sum_{t<j} t (n-1-t) = (n-1) j(j-1)/2 - (j-1) j (2j-1)/6.
__host__ __device__ inline int64_t slab_offset(int64_t n, int64_t j) {
    if (j <= 0) return 0;
    return (n - 1) * (j * (j - 1) / 2) - ((j - 1) * j * (2 * j - 1)) / 6;
}

// Tile sets of a 3-way slab j (the rectangle i in [0, j), k in (j, n_v)):
//   kSlabAll   every bm x bm tile of the rectangle (edge tiles partly outside);
//   kSlabFull  only the ob x ob tiles wholly inside it (bm == ob);
//   kSlabEdge  the rest, in bm x bm tiles: rows [I1, j) against every k, and
//              rows [0, I1) against k in [K1, n_v), where I1 = ob floor(j / ob)
//              and K1 = j + 1 + ob floor((n_v - 1 - j) / ob).
// kSlabFull with ob tiles plus kSlabEdge with smaller bm tiles cover the
// rectangle exactly once, with edge waste at the bm granularity only.
// kSlabRange counts ranges of bm consecutive outputs of the slab instead
// (the elementwise 3-way finish).
// kSlabFlat does not tile slab by slab: its rows are the colex pairs of the
// stage (flat_* below).  kSlabSplit (the VALU slices): kSlabFlat over the
// slabs below the split point split3, then the lex-ordered tiling (lex_*
// below) over the rest, in one launch.  The per-slab sets serve the
// matrix-core slices' per-slab tiling and the finish.
enum { kSlabAll = 0, kSlabFull = 1, kSlabEdge = 2, kSlabRange = 3, kSlabFlat = 4, kSlabSplit = 5 };

// Pair (i, j), i < j, has colex index p = j (j - 1) / 2 + i.  pair_j(p) is
// its j: the largest j with j (j - 1) / 2 <= p.
__host__ __device__ inline int64_t pair_j(int64_t p) {
    int64_t j = (int64_t)((1.0 + __builtin_sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    while (j > 1 && j * (j - 1) / 2 > p) --j;
    while ((j + 1) * j / 2 <= p) ++j;
    return j;
}

// Flattened 3-way tiling (kSlabFlat).  The rows of the slices of a stage
// [jb, je) are the pairs (i, j), i < j, jb <= j < je, in colex order: slab
// after slab, so a row tile of bm consecutive pairs spans one slab or a few.
// Row tile rt (pairs P(jb) + rt bm .. + bm, P(j) = j (j - 1) / 2) is paired
// with the column tiles k in [jmin + 1 + c bm, + bm), jmin = j of its first
// pair, up to n_v.  Entries with k <= j are not stored; every triple of the
// stage lies in exactly one tile.
__host__ __device__ inline int64_t flat_row_tiles(int64_t jb, int64_t je, int bm) {
    const int64_t rows = je * (je - 1) / 2 - jb * (jb - 1) / 2;
    return rows > 0 ? (rows + bm - 1) / bm : 0;
}
__host__ __device__ inline int64_t flat_col_tiles(int64_t n_v, int64_t jb, int bm, int64_t rt) {
    const int64_t jmin = pair_j(jb * (jb - 1) / 2 + rt * bm);
    const int64_t w = n_v - 1 - jmin;
    return w > 0 ? (w + bm - 1) / bm : 0;
}

// Lex order of the pairs (j, k), j < k < n: first index ascending, then k.
// lex_first(n, j) pairs precede those with first index j; lex_pair inverts
// the order through the colex index of the mirrored pair (n-1-k, n-1-j).
__host__ __device__ inline int64_t lex_first(int64_t n, int64_t j) {
    return j * (n - 1) - j * (j - 1) / 2;
}
__host__ __device__ inline void lex_pair(int64_t n, int64_t q, int64_t& j, int64_t& k) {
    const int64_t p = n * (n - 1) / 2 - 1 - q;
    const int64_t kk = pair_j(p);
    j = n - 1 - kk;
    k = n - 1 - (p - kk * (kk - 1) / 2);
}
// Lex-ordered 3-way tiling (the second part of the split tiling of the
// fused int8 slices): the rows are the pairs (j, k), jb <= j < je, in lex
// order; row tile rt (bm consecutive pairs) is paired with the column tiles
// i in [c bm, (c + 1) bm) below the j of its last pair.  Entries with i >= j
// are not stored; every triple of the rows' slabs lies in exactly one tile.
__host__ __device__ inline int64_t lex_row_tiles(int64_t n, int64_t jb, int64_t je, int bm) {
    const int64_t rows = lex_first(n, je) - lex_first(n, jb);
    return rows > 0 ? (rows + bm - 1) / bm : 0;
}
__host__ __device__ inline int64_t lex_col_tiles(int64_t n, int64_t jb, int64_t je, int bm,
                                                 int64_t rt) {
    int64_t q = lex_first(n, jb) + (rt + 1) * bm - 1;
    const int64_t qe = lex_first(n, je) - 1;
    if (q > qe) q = qe;
    int64_t j, k;
    lex_pair(n, q, j, k);
    return (j + bm - 1) / bm;
}

__host__ __device__ inline int64_t slab_tile_count(int64_t n_v, int64_t j, int bm, int mode,
                                                   int ob) {
    const int64_t wk = n_v - 1 - j;
    if (mode == kSlabRange) return (j * wk + bm - 1) / bm;
    if (mode == kSlabAll) return ((j + bm - 1) / bm) * ((wk + bm - 1) / bm);
    if (mode == kSlabFull) return (j / ob) * (wk / ob);
    const int64_t i1 = j / ob * ob, rk = wk % ob;
    return ((j - i1 + bm - 1) / bm) * ((wk + bm - 1) / bm) + (i1 / bm) * ((rk + bm - 1) / bm);
}

// Origin (first i, first k) of tile `local` of slab j in the order the tile
// counts above enumerate them (row-major within each part).
__host__ __device__ inline void slab_tile_origin(int64_t n_v, int64_t j, int64_t local, int bm,
                                                 int mode, int ob, int64_t& row0,
                                                 int64_t& col0) {
    const int64_t wk = n_v - 1 - j;
    if (mode != kSlabEdge) {
        const int64_t nk = mode == kSlabAll ? (wk + bm - 1) / bm : wk / bm;
        row0 = local / nk * bm;
        col0 = j + 1 + local % nk * bm;
        return;
    }
    const int64_t i1 = j / ob * ob, k1 = j + 1 + wk / ob * ob;
    const int64_t nk = (wk + bm - 1) / bm, part1 = ((j - i1 + bm - 1) / bm) * nk;
    if (local < part1) {
        row0 = i1 + local / nk * bm;
        col0 = j + 1 + local % nk * bm;
    } else {
        const int64_t l = local - part1, nk2 = (n_v - k1 + bm - 1) / bm;
        row0 = l / nk2 * bm;
        col0 = k1 + l % nk2 * bm;
    }
}

// Upper-triangle block (bi <= bj) number t of an nb x nb block triangle in
// grouped order: block columns are taken G at a time and, inside a group,
// row by row, so the tiles that run side by side on one XCD share their row
// and column blocks in L2.  The group is found from the column-major
// position of t; the search inside a group is bounded by G rows.
template <int G>
__device__ __forceinline__ void grouped_tri_decode(int64_t t, int64_t nb, int64_t& bi,
                                                   int64_t& bj);
// The same with the group width G chosen at run time (1 <= G <= 64).
__device__ __forceinline__ void grouped_tri_decode_rt(int64_t t, int64_t nb, int G, int64_t& bi,
                                                      int64_t& bj) {
    int64_t j = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    const int64_t g0 = j / G * G;
    const int64_t g1 = g0 + G < nb ? g0 + G : nb;
    const int64_t w = g1 - g0;
    int64_t u = t - g0 * (g0 + 1) / 2;
    if (u < g0 * w) {
        bi = u / w;
        bj = g0 + u % w;
        return;
    }
    u -= g0 * w;
    for (int64_t r = g0; r < g1; ++r) {
        if (u < g1 - r) {
            bi = r;
            bj = r + u;
            return;
        }
        u -= g1 - r;
    }
    bi = bj = 0;
}
template <int G>
__device__ __forceinline__ void grouped_tri_decode(int64_t t, int64_t nb, int64_t& bi,
                                                   int64_t& bj) {
    int64_t j = (int64_t)((__builtin_sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    const int64_t g0 = j / G * G;                    // group of columns [g0, g1)
    const int64_t g1 = g0 + G < nb ? g0 + G : nb;
    const int64_t w = g1 - g0;
    int64_t u = t - g0 * (g0 + 1) / 2;
    if (u < g0 * w) {                                // rows above the group's diagonal
        bi = u / w;
        bj = g0 + u % w;
        return;
    }
    u -= g0 * w;
    for (int64_t r = g0; r < g1; ++r) {              // row r: columns r .. g1-1
        if (u < g1 - r) {
            bi = r;
            bj = r + u;
            return;
        }
        u -= g1 - r;
    }
    bi = bj = 0;   // not reached for 0 <= t < nb (nb + 1) / 2
}

// ---------------------------------------------------------------------------
// Tile configurations of the VALU min-product kernels.
// A workgroup is 2x2 waves; lane (lx, ly) of a wave owns a TM x TN micro-tile
// of rows {g*32 + lx*4 + e} and columns {g*32 + ly*4 + e}.  The workgroup
// output tile is BM x BN = 16*TM x 16*TN; each field tile is BKW 32-bit words
// (BKW * fields-per-word fields).
// ---------------------------------------------------------------------------
struct TileCfg {
    int tm, tn, bkw;
    int bm() const { return 16 * tm; }
    int bn() const { return 16 * tn; }
};

// Fields per chunk of the field-chunk split (PS_ACC_BLOCKED).
constexpr int64_t kChunkFields = 4096;

// Compiled configurations, indexed by ps_opts.tile - 1.
constexpr int kNumValuCfgs = 3;
extern const TileCfg kValuCfgs[kNumValuCfgs];

// Launch policy (policy.hip).
// Field-chunk plan of a 2-way launch.  Blocked accumulation splits at
// kChunkFields; with opts.acc = AUTO a small triangle (fewer work items than
// kMinItems) is split further, down to kMinChunkTiles field tiles per chunk,
// so that enough workgroups run.
struct Split {
    int32_t nchunks;
    int64_t chunk_tiles;
};
constexpr int64_t kMinItems = 2048;      // ~8 workgroups per CU
constexpr int64_t kMinChunkTiles = 4;
int choose_cfg(int32_t dt, int32_t way, int32_t path, int64_t n_f, int64_t n_v,
               const ps_opts* o);
int choose_acc(int64_t n_f, const ps_opts* o);
int32_t split_chunks(int32_t dt, int64_t n_f, int acc);
int64_t chunk_tiles(int32_t dt, int cfg);
Split plan_split(int32_t dt, int64_t n_f, int64_t n_v, int cfg, const ps_opts* o);
bool is_mfma(int path);
// AUTO for PS_U8 data with 1 <= levels <= 15: the path a tuned entry
// (dtype, way, PS_PATH_AUTO) registers for the shape, when that path can
// take it; else the int8 MFMA path when its rows fit the 32-bit tile offsets
// (mfma_ld_fits on the fused path, mfma_row_fits on planes); else VALU.  ld
// is the row stride (n_f in size queries).
int choose_path(int32_t dt, const ps_opts* o, int way, int64_t n_f, int64_t n_v, int64_t ld);
// Tile order of the fused 2-way int8 MFMA kernel: block columns are walked in
// groups of mfma_group(...) columns (a tuned entry for path MFMA registers
// idx, the group being 2^idx; default 4).
constexpr int kNumMfmaCfgs = 5;
int mfma_group(int64_t n_f, int64_t n_v);
int batch_cfg(const ps_problem* p, int32_t n, int32_t dt, const ps_opts* o);

// Arguments of one 2-way launch over the upper-triangle tile list.
struct Mg2Launch {
    const void* V;
    int64_t n_f, n_v, ld;        // ld in elements
    const double* s;
    float* c2;                   // may be null
    void* n2;                    // may be null
    int cfg;                     // index into kValuCfgs
    // field-chunk split: nchunks > 1 sums chunks of chunk_tiles field tiles
    // in separate workgroups into partial[chunk * npairs + pair] (FP32), then
    // a finish kernel adds the chunks in FP64
    int32_t nchunks;
    int64_t chunk_tiles;
    float* partial;
    // tile shard: only the tiles t = shard0 + u * nshards of the upper
    // triangle (nshards <= 1: all tiles)
    int64_t shard0, nshards;
};

// Tiles of the upper triangle in shard shard0 of nshards (tri_tiles when
// nshards <= 1).
inline int64_t shard_tiles(int64_t T, int64_t shard0, int64_t nshards) {
    if (nshards <= 1) return T;
    return T > shard0 ? (T - shard0 + nshards - 1) / nshards : 0;
}

// Arguments of one 3-way launch over the tiles of middle indices
// [j_begin, j_end).
struct Mg3Launch {
    const void* V;
    int64_t n_f, n_v, ld;
    const double* s;
    const void* n2;              // colex pair numerators
    int64_t j_begin, j_end;
    float* c3;
    int64_t* prefix;             // workspace: j_end - j_begin + 1 int64
    int64_t ntiles;
    int cfg;
    int32_t nchunks;             // field-chunk split as for Mg2Launch; partial
    int64_t chunk_tiles;         // holds nchunks * stage-size FP32 values (for
    float* partial;              // PS_F64: stage-size doubles of raw n3', no split)
    int32_t mode;                // tile set of the slice launch: kSlabFlat (prefix over the
                                 // colex row tiles) or kSlabSplit; kSlabAll for the finish
    // kSlabSplit: slabs [j_begin, js) as kSlabFlat (tiles [0, ntiles0), prefix),
    // slabs [js, j_end) lex-ordered (the other tiles, prefix1)
    int64_t js, ntiles0;
    int64_t* prefix1;
};

// Device problem record of a batched launch.
struct DevProblem {
    const void* V;
    int64_t n_f, n_v, ld;
    const double* s;
    float* c2;
    void* n2;
    float* partial;              // raw tile sums: nchunks * pairs 32-bit values
    int32_t nchunks;             // field chunks (1: no split)
    int32_t need_s;              // 1: the sums are computed into s (the caller gave none)
};

// One work item of a batched launch: a tile of a problem and a field chunk.
struct BatchTile {
    int32_t prob, bi, bj, chunk;
};

// A run of the batched work list: every upper-triangle tile (column-major)
// of one field chunk of one problem, starting at list position `start`.
struct BatchGroup {
    int32_t prob, chunk;
    int64_t start;
};

struct MgBatchLaunch {
    const DevProblem* probs;
    const BatchTile* tiles;      // work items: one list per XCD, back to back
    int64_t ntiles;
    int cfg;
    int64_t chunk_tiles;         // field tiles per chunk (same for all problems)
    // the list of XCD x: tiles[xcd_start[x] .. xcd_start[x] + xcd_len[x]),
    // run by the blocks b with b % kXcds == x (hardware deals blocks to the
    // XCDs round-robin), longest first
    int64_t xcd_start[kXcds], xcd_len[kXcds];
};

// Tiles of the 2-way upper triangle for n_v vectors and output tile `bm`.
inline int64_t tri_tiles(int64_t n_v, int bm) {
    int64_t nb = ceil_div(n_v, bm);
    return nb * (nb + 1) / 2;
}

// Tiles of the 3-way slices j in [jb, je).
// Tiles of slabs [jb, je) in a tile set (slab_tile_count).
int64_t slab_tiles(int64_t n_v, int64_t jb, int64_t je, int bm, int mode, int ob);

// Launchers (one per storage type; defined in the per-type units).
hipError_t launch_sums(const void* V, int32_t dt, int64_t n_f, int64_t n_v,
                       int64_t ld, double* s, int32_t* bad, hipStream_t st);
hipError_t launch_mg2_f32(const Mg2Launch& a, hipStream_t st);
hipError_t launch_mg2_f16(const Mg2Launch& a, hipStream_t st);
hipError_t launch_mg2_u8(const Mg2Launch& a, hipStream_t st);
hipError_t launch_mg3_f32(const Mg3Launch& a, hipStream_t st);
hipError_t launch_mg3_f16(const Mg3Launch& a, hipStream_t st);
hipError_t launch_mg3_u8(const Mg3Launch& a, hipStream_t st);
hipError_t launch_mg2_b1(const Mg2Launch& a, hipStream_t st);
hipError_t launch_mg2_f64(const Mg2Launch& a, hipStream_t st);
hipError_t launch_mg3_f64(const Mg3Launch& a, hipStream_t st);
hipError_t launch_mg3_b1(const Mg3Launch& a, hipStream_t st);
// V (uint8 0/1, n_v rows of ld bytes, n_f fields) -> P (n_v rows of
// bits_row_words(n_f) words), pad bits zero.
hipError_t launch_pack_bits(const uint8_t* V, int64_t n_f, int64_t n_v, int64_t ld,
                            uint32_t* P, hipStream_t st);
hipError_t launch_mg3_prefix(const Mg3Launch& a, hipStream_t st);
hipError_t launch_finish2(int32_t dt, const Mg2Launch& a, hipStream_t st);
hipError_t launch_finish2_batched(int32_t dt, const DevProblem* probs, int32_t n,
                                  int64_t max_pairs, hipStream_t st);
hipError_t launch_mgb_f32(const MgBatchLaunch& a, hipStream_t st);
hipError_t launch_mgb_f16(const MgBatchLaunch& a, hipStream_t st);
hipError_t launch_mgb_u8(const MgBatchLaunch& a, hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
hipError_t launch_batched_sums(const DevProblem* probs, int32_t n, int32_t dt, int64_t max_nv,
                               hipStream_t st);
// Host bytes -> device memory through kernel arguments (no host wait, no
// staging buffer; capturable): `bytes` (a multiple of 4) from src to dst.
hipError_t launch_put(void* dst, const void* src, size_t bytes, hipStream_t st);
// The batched work list from its groups: tiles[t] for t < ntiles.
hipError_t launch_batch_expand(const BatchGroup* groups, int32_t ngroups, BatchTile* tiles,
                               int64_t ntiles, hipStream_t st);

// Thermometer int8 MFMA path (PS_U8).
struct MfmaLaunch {
    const void* V;
    int64_t n_f, n_v, ld;
    int levels;
    const double* s;
    float* c2;
    void* n2;
    int8_t* planes;              // workspace: mfma_workspace_bytes()
    int fmt;                     // 0: int8 planes, 1: fp4 (e2m1) planes
    int wide;                    // 0: 4x2 MFMA blocks per wave, 1: 4x4
    int group;                   // fused 2-way: block columns per tile-order group
    int expand;                  // 1: write the planes first; 0: planes already hold V's
    // 3-way slices (launch_mfma3): n2 holds the pair numerators; the fused
    // path (mfma_fused) writes the metric c3 of the stage, the plane path raw
    // n3' (int32 bits) for launch_c3_finish_int
    int64_t j_begin, j_end;
    int64_t* prefix;             // workspace: j_end - j_begin + 1 int64
    float* c3;
    int64_t* edge_prefix;        // 3-way: the edge tiles' slab prefix, as prefix
    int slab3;                   // fused 3-way: 1 = slab tiles (whole + edge), 0 = the
                                 // split tiling when mfma3_split_ok
};
// The int8 thermometer kernels with the 4x2 wave layout threshold V's bytes
// in registers (no plane pass and no plane workspace) when the sums fit
// int32: as counts for levels <= 7 (levels * n_f < 2^31), as -128 counts
// for more levels (levels * n_f < 2^24).  The others read planes.
inline bool mfma_fused(int64_t n_f, int levels, int fmt, int wide) {
    return fmt == 0 && !wide &&
           (int64_t)levels * n_f < ((int64_t)1 << (levels <= 7 ? 31 : 24));
}
// The fused kernels address a 256-row tile of V with 32-bit buffer offsets
// (the last row's field offsets reach at most ld + 127 past its start).
inline bool mfma_ld_fits(int64_t ld) { return 256 * ld + 256 < ((int64_t)1 << 31); }
// The fused 3-way epilogue addresses a tile's rows of the pair table and of
// the slab with 32-bit byte offsets: about 1028 n_v bytes at most.
inline bool mfma3_nv_fits(int64_t n_v) { return n_v < ((int64_t)1 << 21); }
// Split tiling of the 3-way slices of a stage [jb, je): slabs j < js as
// colex pairs (i, j) x columns k, slabs j >= js as lex pairs (j, k) x
// columns i, so that the column range of a row tile is at least about
// min(n_v - js, js) long and the ragged last column tile wastes little
// (js = 2 n_v / 5, about the best in tile-area models for 128- and 256-wide
// tiles).  The int8 matrix-core slices address all of V and the whole pair
// table with 32-bit byte offsets (mfma3_split_ok); the VALU slices take it
// at any size.
inline bool mfma3_split_ok(int64_t n_v, int64_t ld) {
    return n_v * ld + 256 < ((int64_t)1 << 31) &&
           n_v * (n_v - 1) / 2 * 4 < ((int64_t)1 << 31);
}
inline int64_t split3(int64_t n_v, int64_t jb, int64_t je) {
    const int64_t js = 2 * n_v / 5;
    return js < jb ? jb : js > je ? je : js;
}
// Plane workspace of a thermometer launch (0 on the fused path).
size_t mfma_workspace_bytes(int64_t n_f, int64_t n_v, int levels, int fmt, int wide);
// Bytes of one thermometer plane row (all levels) of an n_f-field vector.
int64_t mfma_row_bytes(int64_t n_f, int levels, int fmt);
hipError_t launch_mfma2(const MfmaLaunch& a, hipStream_t st);
// Output tile edge of the MFMA kernels (the 3-way prefix is over these tiles).
constexpr int kMfmaTile = 256;
// The MFMA kernels address a 256-row tile of plane rows with 32-bit buffer
// offsets: 256 plane rows must span less than 2^31 bytes.
inline bool mfma_row_fits(int64_t n_f, int levels, int fmt) {
    return (int64_t)kMfmaTile * mfma_row_bytes(n_f, levels, fmt) < ((int64_t)1 << 31);
}
hipError_t launch_mfma3(const MfmaLaunch& a, hipStream_t st);
// prefix[t] = tiles of slabs jb .. jb+t-1 in a tile set, t = 0 .. je - jb.
hipError_t launch_prefix3(int64_t n_v, int64_t jb, int64_t je, int bm, int mode, int ob,
                          int64_t* prefix, hipStream_t st);
// prefix[rt] = column tiles of the flattened row tiles 0 .. rt-1,
// rt = 0 .. flat_row_tiles(jb, je, bm) (with lex: of the lex-ordered row
// tiles, rt = 0 .. lex_row_tiles(n_v, jb, je, bm)).
hipError_t launch_prefix3_flat(int64_t n_v, int64_t jb, int64_t je, int bm, int64_t* prefix,
                               hipStream_t st, bool lex = false);
// Both parts of the split tiling of a stage (colex slabs [jb, js) into
// prefix0, lex slabs [js, je) into prefix1) in one launch.
hipError_t launch_prefix3_split(int64_t n_v, int64_t jb, int64_t js, int64_t je, int bm,
                                int64_t* prefix0, int64_t* prefix1, hipStream_t st);
// Tiles of the flattened tiling (host loop over the row tiles).
int64_t flat_tiles(int64_t n_v, int64_t jb, int64_t je, int bm);
// Total tiles of the lex-ordered tiling (lex_row_tiles, lex_col_tiles), and
// the prefix of its column-tile counts (launch_prefix3_flat with lex).
int64_t lex_tiles(int64_t n_v, int64_t jb, int64_t je, int bm);
// Output reduction (reduce.hip).
hipError_t launch_quantize_u8(const float* c, int64_t n, uint8_t* q, hipStream_t st);
int64_t select_tiles(int64_t n);
hipError_t launch_select(const float* c, int64_t n, float thr, int64_t base, int64_t* idx,
                         float* val, int64_t cap, int64_t* count, int32_t* counts,
                         int64_t* offsets, hipStream_t st);
// Eq. 1 from exact integer raw n3' (int32 bits in c3) and int32 pair numerators.
hipError_t launch_c3_finish_int(const Mg3Launch& a, hipStream_t st);

}  // namespace ps

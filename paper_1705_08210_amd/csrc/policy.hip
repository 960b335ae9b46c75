// policy.hip -- launch policy of the tile kernels: the tile configurations,
// the tuning table that overrides the defaults, the accumulation mode and
// field-chunk split, and the path choice.  The kernels' work and traffic
// follow from these choices and from the kernel sources alone.
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ps_internal.h"

namespace ps {

const TileCfg kValuCfgs[kNumValuCfgs] = {
    {8, 8, 32},   // 128 x 128 output tile, 32-word field tile
    {4, 4, 32},   // 64 x 64
    {8, 8, 16},   // 128 x 128, 16-word field tile
};

// ---------------------------------------------------------------------------
// Tuning table.
// ---------------------------------------------------------------------------
struct TuneEntry {
    int32_t dt, way, path;
    int64_t nf_lo, nf_hi, nv_lo, nv_hi;
    int32_t idx;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

static int default_cfg(int32_t way, int64_t n_v) {
    // 128x128 output tiles with 16-word field tiles (measured fastest on the
    // large problems: 126 registers, 4 waves per SIMD) once the tiles fill
    // the chip a few times over; 64x64 tiles below that
    if (way == 2) return tri_tiles(n_v, 128) >= 1024 ? 2 : 1;
    return n_v >= 256 ? 2 : 1;
}

int choose_cfg(int32_t dt, int32_t way, int32_t path, int64_t n_f, int64_t n_v,
                      const ps_opts* o) {
    if (o && o->tile > 0) return o->tile - 1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
            if (it->dt == dt && it->way == way && it->path == path && n_f >= it->nf_lo &&
                n_f < it->nf_hi && n_v >= it->nv_lo && n_v < it->nv_hi)
                return it->idx;
    }
    if (dt == PS_F64) return 1;   // 64x64 tiles: the 128x128 FP64 tiles need >= 256 registers
    return default_cfg(way, n_v);
}

int choose_acc(int64_t n_f, const ps_opts* o) {
    const int a = o ? o->acc : PS_ACC_AUTO;
    if (a == PS_ACC_PLAIN || a == PS_ACC_BLOCKED) return a;
    return n_f > kChunkFields ? PS_ACC_BLOCKED : PS_ACC_PLAIN;
}

// Number of field chunks of the blocked (split) accumulation; 1 = no split.
// kChunkFields is a multiple of every configuration's field-tile depth.
int32_t split_chunks(int32_t dt, int64_t n_f, int acc) {
    if (dt == PS_U8 || dt == PS_F64 || acc != PS_ACC_BLOCKED) return 1;   // exact or FP64
    const int64_t n = ceil_div(n_f, kChunkFields);
    return n > 1 ? (int32_t)n : 1;
}

// Field tiles per chunk: a field tile is bkw words of word_bytes(dt) bytes.
int64_t chunk_tiles(int32_t dt, int cfg) {
    return kChunkFields / ((int64_t)kValuCfgs[cfg].bkw * word_bytes(dt) / elem_size(dt));
}

// Field-chunk plan of a 2-way launch (see Split in ps_internal.h).
Split plan_split(int32_t dt, int64_t n_f, int64_t n_v, int cfg, const ps_opts* o) {
    Split sp{split_chunks(dt, n_f, choose_acc(n_f, o)), chunk_tiles(dt, cfg)};
    const int acc_req = o ? o->acc : PS_ACC_AUTO;
    if (dt == PS_U8 || dt == PS_F64 || acc_req != PS_ACC_AUTO || n_v < 2) return sp;
    const int64_t ftiles = ceil_div(n_f * elem_size(dt), (int64_t)kValuCfgs[cfg].bkw * 4);
    const int64_t tiles = tri_tiles(n_v, kValuCfgs[cfg].bm());
    if (tiles * sp.nchunks >= kMinItems) return sp;
    const int64_t want = std::min(ceil_div(kMinItems, tiles), ftiles / kMinChunkTiles);
    if (want > sp.nchunks) {
        sp.chunk_tiles = ceil_div(ftiles, want);
        sp.nchunks = (int32_t)ceil_div(ftiles, sp.chunk_tiles);
    }
    return sp;
}

// Tile configuration of a batched launch: a tuning entry registered for
// way 0 and the field count of the largest problem, else 128x128 tiles with
// 16-word field tiles.
int batch_cfg(const ps_problem* p, int32_t n, int32_t dt, const ps_opts* o) {
    if (o && o->tile > 0) return o->tile - 1;
    // representative shape: the field count of the largest problem by work
    int64_t best = -1, nf = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t w = p[i].n_f * p[i].n_v * p[i].n_v;
        if (w > best) best = w, nf = p[i].n_f;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
        if (it->dt == dt && it->way == 0 && nf >= it->nf_lo && nf < it->nf_hi)
            return it->idx;
    return 2;
}

int64_t max_grid_blocks(int threads, int64_t multiple) {
    static const int64_t env_cap = [] {
        const char* e = getenv("PS_MAX_GRID_BLOCKS");
        const long long v = e ? atoll(e) : 0;
        return v > 0 ? (int64_t)v : (int64_t)0;
    }();
    int64_t cap = (int64_t)0xffffffffu / threads;
    if (env_cap > 0 && env_cap < cap) cap = env_cap;
    cap = cap / multiple * multiple;
    return cap > 0 ? cap : multiple;
}

bool is_mfma(int path) { return path == PS_PATH_MFMA || path == PS_PATH_MFMA_FP4; }

// Whether a matrix-core path can take the shape (exact sums, 32-bit offsets).
static bool mfma_can(int path, int way, int64_t n_f, int64_t n_v, int levels, int wide,
                     int64_t ld) {
    if (path == PS_PATH_MFMA_FP4)
        return (int64_t)levels * n_f < ((int64_t)1 << 24) && mfma_row_fits(n_f, levels, 1);
    if (mfma_fused(n_f, levels, 0, wide))
        return mfma_ld_fits(ld) && (way != 3 || mfma3_nv_fits(n_v));
    return (int64_t)levels * n_f < ((int64_t)1 << 31) && mfma_row_fits(n_f, levels, 0);
}

// A tuned entry for (dt, way, path) covering the shape, or -1.
static int tuned(int32_t dt, int way, int32_t path, int64_t n_f, int64_t n_v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
        if (it->dt == dt && it->way == way && it->path == path && n_f >= it->nf_lo &&
            n_f < it->nf_hi && n_v >= it->nv_lo && n_v < it->nv_hi)
            return it->idx;
    return -1;
}

int choose_path(int32_t dt, const ps_opts* o, int way, int64_t n_f, int64_t n_v, int64_t ld) {
    const int p = o ? o->path : PS_PATH_AUTO;
    if (p == PS_PATH_VALU || p == PS_PATH_MFMA || p == PS_PATH_MFMA_FP4 || p == PS_PATH_BITS)
        return p;
    if (dt != PS_U8 || !o || o->levels < 1 || o->levels > 15) return PS_PATH_VALU;
    const int wide = way == 2 && o->tile == 2;   // 3-way: tile 2 picks the slab tiles
    const int t = tuned(dt, way, PS_PATH_AUTO, n_f, n_v);
    if (t == PS_PATH_VALU) return PS_PATH_VALU;
    if ((t == PS_PATH_MFMA || t == PS_PATH_MFMA_FP4) &&
        mfma_can(t, way, n_f, n_v, o->levels, wide, ld))
        return t;
    return mfma_can(PS_PATH_MFMA, way, n_f, n_v, o->levels, wide, ld) ? PS_PATH_MFMA
                                                                      : PS_PATH_VALU;
}

int mfma_group(int64_t n_f, int64_t n_v) {
    const int t = tuned(PS_U8, 2, PS_PATH_MFMA, n_f, n_v);
    return 1 << (t >= 0 ? t : 2);
}

}  // namespace ps

using namespace ps;

extern "C" {

int32_t ps_tile_config(int32_t dtype, int32_t way, int32_t path, int32_t idx, int32_t* bm,
                       int32_t* bn, int32_t* bk) {
    if (elem_size(dtype) == 0 || (way != 2 && way != 3)) return 0;
    if (path == PS_PATH_MFMA && way == 3) {   // tilings of the fused 3-way int8 slices
        if (dtype != PS_U8) return 0;
        if (idx >= 0 && idx < 2) {
            if (bm) *bm = kMfmaTile;
            if (bn) *bn = kMfmaTile;
            if (bk) *bk = 128;
        }
        return 2;
    }
    if (path == PS_PATH_MFMA) {   // tile orders of the 2-way int8 kernel, 256 x 256 x 128
        if (dtype != PS_U8 || way != 2) return 0;
        if (idx >= 0 && idx < kNumMfmaCfgs) {
            if (bm) *bm = kMfmaTile;
            if (bn) *bn = kMfmaTile;
            if (bk) *bk = 128;
        }
        return kNumMfmaCfgs;
    }
    if (is_mfma(path)) return 0;
    if (idx >= 0 && idx < kNumValuCfgs) {
        if (bm) *bm = kValuCfgs[idx].bm();
        if (bn) *bn = kValuCfgs[idx].bn();
        if (bk) *bk = kValuCfgs[idx].bkw * word_bytes(dtype) / elem_size(dtype);  // fields
    }
    return kNumValuCfgs;
}

ps_status ps_tune_register(int32_t dtype, int32_t way, int32_t path, int64_t nf_lo,
                           int64_t nf_hi, int64_t nv_lo, int64_t nv_hi, int32_t idx) {
    if (elem_size(dtype) == 0) return fail(PS_ERR_DTYPE, "unknown dtype %d", dtype);
    if (way != 0 && way != 2 && way != 3)
        return fail(PS_ERR_ARG, "way must be 2, 3 (or 0 for batched)");
    if (path == PS_PATH_AUTO) {   // the path AUTO takes for integer data
        if (dtype != PS_U8 || way == 0)
            return fail(PS_ERR_ARG, "path choices are tuned for PS_U8, way 2 or 3");
        if (idx != PS_PATH_VALU && idx != PS_PATH_MFMA && idx != PS_PATH_MFMA_FP4)
            return fail(PS_ERR_ARG, "path choice %d is not VALU, MFMA or MFMA_FP4", idx);
    } else if (path == PS_PATH_MFMA) {
        if (idx < 0 || idx >= kNumMfmaCfgs)
            return fail(PS_ERR_ARG, "MFMA tile order %d out of range", idx);
    } else if (idx < 0 || idx >= kNumValuCfgs) {
        return fail(PS_ERR_ARG, "tile index %d out of range", idx);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.push_back(TuneEntry{dtype, way, path, nf_lo, nf_hi, nv_lo, nv_hi, idx});
    return PS_OK;
}

int32_t ps_path_choice(int32_t dtype, int32_t way, int64_t n_f, int64_t n_v, int64_t ld,
                       const ps_opts* opts) {
    if (elem_size(dtype) == 0 || (way != 2 && way != 3) || n_f < 0 || n_v < 0) return -1;
    return choose_path(dtype, opts, way, n_f, n_v, ld < n_f ? n_f : ld);
}

void ps_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

}  // extern "C"

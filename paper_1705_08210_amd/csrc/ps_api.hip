// ps_api.hip -- the C ABI of include/ps.h: argument checks, workspace
// carving, plan selection and launch sequencing.  No arithmetic of the
// metric happens here; every step runs in the kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ps_internal.h"

namespace ps {


static thread_local char g_err[512] = "";

ps_status fail(ps_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

static ps_status hip_fail(hipError_t e, const char* what) {
    return fail(PS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t slab_tiles(int64_t n_v, int64_t jb, int64_t je, int bm, int mode, int ob) {
    int64_t t = 0;
    for (int64_t j = jb; j < je; ++j) t += slab_tile_count(n_v, j, bm, mode, ob);
    return t;
}

// ---------------------------------------------------------------------------
// Argument checks.
// ---------------------------------------------------------------------------
static ps_status check_opts(const ps_opts* o) {
    if (!o) return PS_OK;
    if (o->acc < PS_ACC_PLAIN || o->acc > PS_ACC_AUTO)
        return fail(PS_ERR_ARG, "opts.acc = %d is not a ps_acc value", o->acc);
    if (o->path < PS_PATH_AUTO || o->path > PS_PATH_BITS)
        return fail(PS_ERR_ARG, "opts.path = %d is not a ps_path value", o->path);
    if (o->tile < 0 || o->tile > kNumValuCfgs)
        return fail(PS_ERR_ARG, "opts.tile = %d out of range [0, %d]", o->tile, kNumValuCfgs);
    if (o->levels < 0 || o->levels > 127)
        return fail(PS_ERR_ARG, "opts.levels = %d out of range [0, 127]", o->levels);
    return PS_OK;
}

static ps_status check_matrix(const void* V, int32_t dt, int64_t n_f, int64_t n_v, int64_t ld) {
    const int esz = elem_size(dt);
    if (esz == 0) return fail(PS_ERR_DTYPE, "unknown dtype %d", dt);
    if (n_f < 0 || n_v < 0) return fail(PS_ERR_ARG, "n_f = %lld, n_v = %lld must be >= 0",
                                        (long long)n_f, (long long)n_v);
    if (ld < (n_f > 1 ? n_f : 1))
        return fail(PS_ERR_ARG, "ld = %lld must be >= max(n_f, 1) = %lld", (long long)ld,
                    (long long)(n_f > 1 ? n_f : 1));
    if (n_v > (int64_t)1 << 31)
        return fail(PS_ERR_ARG, "n_v = %lld exceeds 2^31", (long long)n_v);
    if (n_v > 0 && n_f > 0 && !V) return fail(PS_ERR_ARG, "V is NULL");
    if ((uintptr_t)V % esz) return fail(PS_ERR_ARG, "V is not aligned to its element size");
    return PS_OK;
}

static bool aligned(const void* p, size_t a) { return (uintptr_t)p % a == 0; }

// Workspace carving: consecutive 256-byte aligned regions.
struct Carver {
    char* base;
    size_t used = 0;
    explicit Carver(void* b) : base((char*)b) {}
    void* take(size_t bytes) {
        void* p = base ? base + used : nullptr;
        used = align_up(used + bytes, 256);
        return p;
    }
};

static hipError_t launch_mg2(int32_t dt, const Mg2Launch& a, hipStream_t st) {
    switch (dt) {
    case PS_F32: return launch_mg2_f32(a, st);
    case PS_F16: return launch_mg2_f16(a, st);
    case PS_B1: return launch_mg2_b1(a, st);
    case PS_F64: return launch_mg2_f64(a, st);
    default: return launch_mg2_u8(a, st);
    }
}

static hipError_t launch_mg3(int32_t dt, const Mg3Launch& a, hipStream_t st) {
    switch (dt) {
    case PS_F32: return launch_mg3_f32(a, st);
    case PS_F16: return launch_mg3_f16(a, st);
    case PS_B1: return launch_mg3_b1(a, st);
    case PS_F64: return launch_mg3_f64(a, st);
    default: return launch_mg3_u8(a, st);
    }
}

// The BITS path takes binary uint8 data and says so with opts.levels = 1.
static ps_status check_bits(int32_t dtype, const ps_opts* o) {
    if (!o || o->path != PS_PATH_BITS) return PS_OK;
    if (dtype != PS_U8) return fail(PS_ERR_UNSUPPORTED, "the BITS path needs PS_U8 data");
    if (o->levels != 1)
        return fail(PS_ERR_ARG, "the BITS path needs binary data: opts.levels = 1, got %d",
                    o->levels);
    return PS_OK;
}

static bool is_bits(const ps_opts* o) { return o && o->path == PS_PATH_BITS; }

// The thermometer paths take uint8 data with a bound on its values, and every
// numerator (at most levels * n_f) must be exact in the accumulator.
static ps_status check_mfma(int path, int32_t dtype, int levels, int64_t n_f, int64_t ld,
                            int wide) {
    if (!is_mfma(path)) return PS_OK;
    if (dtype != PS_U8) return fail(PS_ERR_UNSUPPORTED, "the MFMA path needs PS_U8 data");
    if (levels < 1) return fail(PS_ERR_ARG, "the MFMA path needs opts.levels >= max(V) >= 1");
    if (path == PS_PATH_MFMA_FP4 && (int64_t)levels * n_f >= ((int64_t)1 << 24))
        return fail(PS_ERR_ARG, "fp4 path: levels * n_f = %lld exceeds the exact FP32 range",
                    (long long)levels * n_f);
    if (path == PS_PATH_MFMA && (int64_t)levels * n_f >= ((int64_t)1 << 31))
        return fail(PS_ERR_ARG, "int8 path: levels * n_f = %lld exceeds int32",
                    (long long)levels * n_f);
    const int fmt = path == PS_PATH_MFMA_FP4 ? 1 : 0;
    if (mfma_fused(n_f, levels, fmt, wide)) {
        if (!mfma_ld_fits(ld))
            return fail(PS_ERR_UNSUPPORTED,
                        "int8 MFMA path: rows of %lld bytes are too long for 32-bit tile offsets "
                        "(256 rows must span < 2^31 bytes); use the VALU path", (long long)ld);
        return PS_OK;
    }
    if (!mfma_row_fits(n_f, levels, fmt))
        return fail(PS_ERR_UNSUPPORTED,
                    "MFMA path: plane rows of %lld bytes (levels * n_f = %lld) are too long for "
                    "32-bit tile offsets (256 rows must span < 2^31 bytes); use the VALU path",
                    (long long)mfma_row_bytes(n_f, levels, path == PS_PATH_MFMA_FP4 ? 1 : 0),
                    (long long)levels * n_f);
    return PS_OK;
}

// The uint8 VALU kernels sum |a - b| four bytes at a time into uint32 and
// store pair numerators as int32; both hold only while 255 n_f < 2^31.  The
// BITS path stores population counts (at most n_f) as int32.
static ps_status check_int_range(int path, int32_t dtype, int64_t n_f) {
    if (dtype != PS_U8 || is_mfma(path)) return PS_OK;
    if (path == PS_PATH_BITS) {
        if (n_f >= ((int64_t)1 << 31))
            return fail(PS_ERR_UNSUPPORTED, "BITS path: n_f = %lld exceeds the int32 counts",
                        (long long)n_f);
        return PS_OK;
    }
    if (255 * n_f >= ((int64_t)1 << 31))
        return fail(PS_ERR_UNSUPPORTED,
                    "uint8 VALU path: 255 * n_f = %lld exceeds the 32-bit integer sums "
                    "(n_f must be below 8421505)", (long long)(255 * n_f));
    return PS_OK;
}

static size_t bits_bytes(int64_t n_f, int64_t n_v) {
    return (size_t)n_v * (size_t)bits_row_words(n_f) * sizeof(uint32_t);
}

static hipError_t launch_mgb(int32_t dt, const MgBatchLaunch& a, hipStream_t st) {
    switch (dt) {
    case PS_F32: return launch_mgb_f32(a, st);
    case PS_F16: return launch_mgb_f16(a, st);
    default: return launch_mgb_u8(a, st);
    }
}

// Sizes of the 2-way workspace regions.  Returns total bytes.
static size_t ws2_layout(int32_t dt, int64_t n_f, int64_t n_v, int32_t s_given, int path,
                         int levels, int wide, int32_t nchunks, void* ws, double** s_ws,
                         int8_t** planes, float** partial) {
    Carver c(ws);
    double* s = nullptr;
    if (!s_given) s = (double*)c.take((size_t)n_v * sizeof(double));
    int8_t* pl = nullptr;
    float* part = nullptr;
    if (is_mfma(path) && dt == PS_U8)
        pl = (int8_t*)c.take(
            mfma_workspace_bytes(n_f, n_v, levels, path == PS_PATH_MFMA_FP4 ? 1 : 0, wide));
    else if (path == PS_PATH_BITS && dt == PS_U8)   // the packed bits
        pl = (int8_t*)c.take(bits_bytes(n_f, n_v));
    else if (nchunks > 1)
        part = (float*)c.take((size_t)nchunks * (size_t)(n_v * (n_v - 1) / 2) * sizeof(float));
    if (s_ws) *s_ws = s;
    if (planes) *planes = pl;
    if (partial) *partial = part;
    return c.used;
}

}  // namespace ps

using namespace ps;

extern "C" {

const char* ps_status_string(ps_status st) {
    switch (st) {
    case PS_OK: return "PS_OK";
    case PS_ERR_ARG: return "PS_ERR_ARG";
    case PS_ERR_DTYPE: return "PS_ERR_DTYPE";
    case PS_ERR_WORKSPACE: return "PS_ERR_WORKSPACE";
    case PS_ERR_HIP: return "PS_ERR_HIP";
    case PS_ERR_UNSUPPORTED: return "PS_ERR_UNSUPPORTED";
    }
    return "PS_STATUS_UNKNOWN";
}

const char* ps_last_error(void) { return g_err; }

int32_t ps_version(void) { return 10000; }

ps_status ps_vector_sums(const void* V, int32_t dtype, int64_t n_f, int64_t n_v, int64_t ld,
                         double* s, int32_t* bad_count, hipStream_t stream) {
    ps_status st = check_matrix(V, dtype, n_f, n_v, ld);
    if (st != PS_OK) return st;
    if (n_v > 0 && !s) return fail(PS_ERR_ARG, "s is NULL");
    if (!aligned(s, 8)) return fail(PS_ERR_ARG, "s is not 8-byte aligned");
    if (!aligned(bad_count, 4)) return fail(PS_ERR_ARG, "bad_count is not 4-byte aligned");
    hipError_t e = launch_sums(V, dtype, n_f, n_v, ld, s, bad_count, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "ps_vector_sums launch");
}

size_t ps2_workspace_size(int32_t dtype, int64_t n_f, int64_t n_v, int32_t s_given,
                          const ps_opts* opts) {
    if (elem_size(dtype) == 0 || n_f < 0 || n_v < 0) return 0;
    const int path = choose_path(dtype, opts, 2, n_f, n_v, n_f);
    const Split sp = path == PS_PATH_BITS
                         ? Split{1, 0}
                         : plan_split(dtype, n_f, n_v,
                                      choose_cfg(dtype, 2, PS_PATH_VALU, n_f, n_v, opts), opts);
    return ws2_layout(dtype, n_f, n_v, s_given, path, opts ? opts->levels : 0,
                      opts && opts->tile == 2, sp.nchunks, nullptr, nullptr, nullptr, nullptr);
}

// ps2_compute over the tiles of one shard (nshards > 1, see
// ps2_compute_shard) or over all tiles (nshards == 1).
static ps_status ps2_run(const void* V, int32_t dtype, int64_t n_f, int64_t n_v, int64_t ld,
                         const double* s, float* c2, void* n2, int64_t shard, int64_t nshards,
                         void* workspace, size_t ws_bytes, const ps_opts* opts,
                         hipStream_t stream) {
    ps_status st = check_matrix(V, dtype, n_f, n_v, ld);
    if (st != PS_OK) return st;
    if ((st = check_opts(opts)) != PS_OK) return st;
    if (nshards < 1 || shard < 0 || shard >= nshards)
        return fail(PS_ERR_ARG, "need 0 <= shard < nshards, got shard %lld of %lld",
                    (long long)shard, (long long)nshards);
    if (n_v < 2) return PS_OK;
    if (!c2 && !n2) return fail(PS_ERR_ARG, "both c2 and n2 are NULL");
    if (!aligned(c2, 4) || !aligned(n2, 4) || !aligned(s, 8))
        return fail(PS_ERR_ARG, "misaligned output or sums pointer");
    if ((st = check_bits(dtype, opts)) != PS_OK) return st;
    const int path = choose_path(dtype, opts, 2, n_f, n_v, ld);
    const int levels = opts ? opts->levels : 0;
    const int wide = opts && opts->tile == 2;
    if ((st = check_mfma(path, dtype, levels, n_f, ld, wide)) != PS_OK) return st;
    if ((st = check_int_range(path, dtype, n_f)) != PS_OK) return st;
    if (nshards > 1 && is_mfma(path))
        return fail(PS_ERR_UNSUPPORTED, "sharded calls run on the VALU and BITS paths only");
    double* s_ws = nullptr;
    int8_t* planes = nullptr;
    float* partial = nullptr;
    const bool bits = path == PS_PATH_BITS;
    const int cfg = bits ? choose_cfg(PS_B1, 2, PS_PATH_BITS, n_f, n_v, opts)
                         : choose_cfg(dtype, 2, PS_PATH_VALU, n_f, n_v, opts);
    // a shard takes the whole call's field-chunk plan: its workspace and sums are the same
    const Split sp = bits ? Split{1, 0} : plan_split(dtype, n_f, n_v, cfg, opts);
    const size_t need = ws2_layout(dtype, n_f, n_v, s != nullptr, path, levels, wide,
                                   sp.nchunks, workspace, &s_ws, &planes, &partial);
    if (ws_bytes < need || (need && !workspace))
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(PS_ERR_ARG, "workspace is not 256-byte aligned");
    hipError_t e;
    if (!s) {
        e = launch_sums(V, dtype, n_f, n_v, ld, s_ws, nullptr, stream);
        if (e != hipSuccess) return hip_fail(e, "sums launch");
        s = s_ws;
    }
    if (is_mfma(path)) {
        // opts.tile: 0 or 1 -> 4x2 blocks per wave, 2 -> 4x4 blocks per wave
        MfmaLaunch m{V,    n_f,  n_v, ld, levels, s, c2, n2, planes, path == PS_PATH_MFMA_FP4 ? 1 : 0,
                     wide, mfma_group(n_f, n_v), 1, 0, 0, nullptr, nullptr};
        e = launch_mfma2(m, stream);
        if (e == hipErrorNotSupported)
            return fail(PS_ERR_UNSUPPORTED, "MFMA path not available in this library");
        return e == hipSuccess ? PS_OK : hip_fail(e, "mfma launch");
    }
    if (bits) {   // pack, then the min-product on words (zero pad words add nothing)
        const int64_t W = bits_row_words(n_f);
        e = launch_pack_bits((const uint8_t*)V, n_f, n_v, ld, (uint32_t*)planes, stream);
        if (e != hipSuccess) return hip_fail(e, "bit packing launch");
        Mg2Launch a{planes, W, n_v, W, s, c2, n2, cfg, 1, 0, nullptr, shard, nshards};
        e = launch_mg2(PS_B1, a, stream);
        return e == hipSuccess ? PS_OK : hip_fail(e, "2-way bits launch");
    }
    Mg2Launch a{V,         n_f,           n_v,     ld,    s,      c2, n2, cfg,
                sp.nchunks, sp.chunk_tiles, partial, shard, nshards};
    e = launch_mg2(dtype, a, stream);
    if (e == hipSuccess && sp.nchunks > 1) e = launch_finish2(dtype, a, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "2-way launch");
}

// The field-split partials of the pair prepass and of the slices run one
// after the other on the stream and share one region.
// Prefix entries of a 3-way stage [jb, je): two slab prefixes of n_v + 1
// (whole and edge tiles of the per-slab matrix-core slices, the finish's
// ranges), or the row tiles of the split tiling's two parts, whichever is more.
static int64_t prefix3_entries(int64_t n_v, int64_t jb, int64_t je) {
    // the split tiling's two parts (colex slabs [jb, js), lex slabs [js, je)) at
    // the smallest tile edge of any path (64; the matrix-core tiles are 256)
    const int64_t js = split3(n_v, jb, je);
    const int64_t split = flat_row_tiles(jb, js, 64) + lex_row_tiles(n_v, js, je, 64) + 2;
    return 2 * (n_v + 1) > split ? 2 * (n_v + 1) : split;
}

static size_t ws3_layout(int64_t n_v, int64_t npre, int32_t s_given, int32_t n2_given,
                         int n2_bytes, int32_t nchunks2, int32_t nchunks3, int64_t stage,
                         size_t packed_bytes, void* ws,
                         double** s_ws, void** n2_ws, int64_t** prefix, float** partial,
                         uint32_t** packed) {
    Carver c(ws);
    double* s = nullptr;
    void* n2 = nullptr;
    float* part = nullptr;
    if (packed) *packed = packed_bytes ? (uint32_t*)c.take(packed_bytes) : nullptr;
    else if (packed_bytes) c.take(packed_bytes);
    if (!s_given) s = (double*)c.take((size_t)n_v * sizeof(double));
    if (!n2_given) n2 = c.take((size_t)(n_v * (n_v - 1) / 2) * (size_t)n2_bytes);
    int64_t* pre = (int64_t*)c.take((size_t)npre * sizeof(int64_t));
    const int64_t need2 = (!n2_given && nchunks2 > 1) ? nchunks2 * (n_v * (n_v - 1) / 2) : 0;
    // floats of the slice sums: FP32 chunk partials, or (nchunks3 < 0) FP64 raw sums
    const int64_t need3 = nchunks3 < 0 ? 2 * stage : nchunks3 > 1 ? nchunks3 * stage : 0;
    if (need2 > 0 || need3 > 0)
        part = (float*)c.take((size_t)(need2 > need3 ? need2 : need3) * sizeof(float));
    if (s_ws) *s_ws = s;
    if (n2_ws) *n2_ws = n2;
    if (prefix) *prefix = pre;
    if (partial) *partial = part;
    return c.used;
}

// 3-way on the matrix cores (uint8 levels): planes once, the pair
// numerators by the 2-way MFMA kernel (unless given), the masked slices, then
// Eq. 1 from exact integers.
static ps_status ps3_mfma(const void* V, int64_t n_f, int64_t n_v, int64_t ld, const double* s,
                          const void* n2, int64_t j_begin, int64_t j_end, float* c3,
                          void* workspace, size_t ws_bytes, int path, int levels, int tile,
                          hipStream_t stream) {
    const int fmt = path == PS_PATH_MFMA_FP4 ? 1 : 0;
    const int64_t stage = ps3_stage_size(n_v, j_begin, j_end);
    double* s_ws = nullptr;
    void* n2_ws = nullptr;
    int64_t* prefix = nullptr;
    float* partial = nullptr;
    uint32_t* planes = nullptr;
    const size_t need = ws3_layout(n_v, prefix3_entries(n_v, j_begin, j_end), s != nullptr,
                                   n2 != nullptr, 4, 1, 1, stage,
                                   mfma_workspace_bytes(n_f, n_v, levels, fmt, 0), workspace,
                                   &s_ws, &n2_ws, &prefix, &partial, &planes);
    if (ws_bytes < need || !workspace)
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(PS_ERR_ARG, "workspace is not 256-byte aligned");
    hipError_t e;
    if (!s) {
        e = launch_sums(V, PS_U8, n_f, n_v, ld, s_ws, nullptr, stream);
        if (e != hipSuccess) return hip_fail(e, "sums launch");
        s = s_ws;
    }
    MfmaLaunch m{V,   n_f, n_v, ld, levels, s, nullptr, nullptr, (int8_t*)planes, fmt, 0,
                 mfma_group(n_f, n_v), 1, j_begin, j_end, prefix, c3, prefix + (n_v + 1)};
    if (!n2) {   // pair numerators; this launch also writes the planes
        MfmaLaunch m2 = m;
        m2.n2 = n2_ws;
        e = launch_mfma2(m2, stream);
        if (e != hipSuccess) return hip_fail(e, "3-way numerator prepass launch");
        n2 = n2_ws;
        m.expand = 0;
    }
    m.n2 = (void*)n2;   // the pair numerators of Eq. 1
    m.slab3 = tile == 2;
    e = launch_mfma3(m, stream);
    if (e != hipSuccess) return hip_fail(e, "3-way mfma launch");
    if (mfma_fused(n_f, levels, fmt, 0)) return PS_OK;   // Eq. 1 applied in the slices
    Mg3Launch f{V, n_f, n_v, ld, s, n2, j_begin, j_end, c3, prefix, 0, 0, 1, 0, nullptr, kSlabAll};
    e = launch_c3_finish_int(f, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "3-way finish launch");
}

size_t ps3_workspace_size(int32_t dtype, int64_t n_f, int64_t n_v, int32_t s_given,
                          int32_t n2_given, int64_t j_begin, int64_t j_end,
                          const ps_opts* opts) {
    if (elem_size(dtype) == 0 || n_f < 0 || n_v < 0) return 0;
    if (j_begin < 1) j_begin = 1;
    if (j_end > n_v - 1) j_end = n_v - 1;
    const int64_t stage = ps3_stage_size(n_v, j_begin, j_end);
    const int64_t npre = prefix3_entries(n_v, j_begin, j_end);
    if (is_bits(opts))
        return ws3_layout(n_v, npre, s_given, n2_given, 4, 1, 1, stage, bits_bytes(n_f, n_v),
                          nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    const int path = choose_path(dtype, opts, 3, n_f, n_v, n_f);
    if (is_mfma(path) && dtype == PS_U8)
        return ws3_layout(n_v, npre, s_given, n2_given, 4, 1, 1, stage,
                          mfma_workspace_bytes(n_f, n_v, opts ? opts->levels : 0,
                                               path == PS_PATH_MFMA_FP4 ? 1 : 0, 0),
                          nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    const Split sp2 =
        plan_split(dtype, n_f, n_v, choose_cfg(dtype, 2, PS_PATH_VALU, n_f, n_v, opts), opts);
    return ws3_layout(n_v, npre, s_given, n2_given, dtype == PS_F64 ? 8 : 4, sp2.nchunks,
                      dtype == PS_F64 ? -1 : split_chunks(dtype, n_f, choose_acc(n_f, opts)),
                      stage, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

ps_status ps_quantize_u8(const float* c, int64_t n, uint8_t* q, hipStream_t stream) {
    if (n < 0) return fail(PS_ERR_ARG, "n = %lld < 0", (long long)n);
    if (n > 0 && (!c || !q)) return fail(PS_ERR_ARG, "c or q is NULL");
    if (!aligned(c, 4)) return fail(PS_ERR_ARG, "c is not 4-byte aligned");
    hipError_t e = launch_quantize_u8(c, n, q, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "quantize launch");
}

// counts (int32 per tile) then offsets (int64 per tile)
size_t ps_threshold_workspace_size(int64_t n) {
    if (n < 0) return 0;
    Carver c(nullptr);
    c.take((size_t)select_tiles(n) * sizeof(int32_t));
    c.take((size_t)select_tiles(n) * sizeof(int64_t));
    return c.used;
}

ps_status ps_threshold(const float* c, int64_t n, float threshold, int64_t base,
                       int64_t* idx, float* val, int64_t cap, int64_t* count,
                       void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || cap < 0) return fail(PS_ERR_ARG, "n = %lld, cap = %lld: need >= 0",
                                      (long long)n, (long long)cap);
    if (!count) return fail(PS_ERR_ARG, "count is NULL");
    if (n > 0 && !c) return fail(PS_ERR_ARG, "c is NULL");
    if (cap > 0 && (!idx || !val)) return fail(PS_ERR_ARG, "idx or val is NULL");
    if (!aligned(c, 4) || !aligned(val, 4) || !aligned(idx, 8) || !aligned(count, 8))
        return fail(PS_ERR_ARG, "misaligned pointer");
    const size_t need = ps_threshold_workspace_size(n);
    if (ws_bytes < need || (need && !workspace))
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(PS_ERR_ARG, "workspace is not 256-byte aligned");
    Carver w(workspace);
    int32_t* counts = (int32_t*)w.take((size_t)select_tiles(n) * sizeof(int32_t));
    int64_t* offsets = (int64_t*)w.take((size_t)select_tiles(n) * sizeof(int64_t));
    hipError_t e = launch_select(c, n, threshold, base, idx, val, cap, count, counts, offsets,
                                 stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "threshold launch");
}

int64_t ps3_stage_size(int64_t n_v, int64_t j_begin, int64_t j_end) {
    if (n_v < 3 || j_end <= j_begin) return 0;
    return slab_offset(n_v, j_end) - slab_offset(n_v, j_begin);
}

}  // extern "C"

namespace ps {

// Static scratch of ps3_compute_noalloc.  Each GPU holds its own copy of this
// array (allocated when the library's code is loaded on it, kept until the
// process ends).  Host code never uses the array's name as an address: the
// per-device address comes from hipGetSymbolAddress, taken once per device
// with that device current.
static __device__ __align__(256) unsigned char scratch[PS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static ps_status scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(PS_ERR_UNSUPPORTED, "device %d: the static scratch serves devices 0..%d",
                    dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || !aligned(p, 256))
            return fail(PS_ERR_HIP, "static scratch of device %d has no usable address", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PS_OK;
}

// The body of ps3_compute and ps3_compute_noalloc: `workspace` is the
// caller's buffer or, with from_scratch, looked up after the argument checks:
// the static scratch of the current device (ws_bytes is then its size).
static ps_status ps3_run(const void* V, int32_t dtype, int64_t n_f, int64_t n_v, int64_t ld,
                         const double* s, const void* n2, int64_t j_begin, int64_t j_end,
                         float* c3, void* workspace, size_t ws_bytes, bool from_scratch,
                         const ps_opts* opts, hipStream_t stream) {
    ps_status st = check_matrix(V, dtype, n_f, n_v, ld);
    if (st != PS_OK) return st;
    if ((st = check_opts(opts)) != PS_OK) return st;
    if ((st = check_bits(dtype, opts)) != PS_OK) return st;
    const int path = choose_path(dtype, opts, 3, n_f, n_v, ld);
    const int levels = opts ? opts->levels : 0;
    if ((st = check_mfma(path, dtype, levels, n_f, ld, 0)) != PS_OK) return st;
    if (path == PS_PATH_MFMA && mfma_fused(n_f, levels, 0, 0) && !mfma3_nv_fits(n_v))
        return fail(PS_ERR_UNSUPPORTED,
                    "3-way int8 MFMA path: n_v = %lld is too large for the 32-bit offsets of "
                    "its epilogue (n_v < 2^21); use the VALU path", (long long)n_v);
    if ((st = check_int_range(path, dtype, n_f)) != PS_OK) return st;
    if (n_v < 3) return PS_OK;
    if (j_begin < 1 || j_end > n_v - 1 || j_begin > j_end)
        return fail(PS_ERR_ARG, "need 1 <= j_begin <= j_end <= n_v-1, got [%lld, %lld)",
                    (long long)j_begin, (long long)j_end);
    if (j_begin == j_end) return PS_OK;
    if (!c3) return fail(PS_ERR_ARG, "c3 is NULL");
    if (!aligned(c3, 4) || !aligned(n2, 4) || !aligned(s, 8))
        return fail(PS_ERR_ARG, "misaligned output, n2 or sums pointer");
    if (from_scratch) {
        const size_t need = ps3_workspace_size(dtype, n_f, n_v, s != nullptr, n2 != nullptr,
                                               j_begin, j_end, opts);
        if (need > ws_bytes)
            return fail(PS_ERR_WORKSPACE,
                        "ps3_compute_noalloc: this call needs %zu bytes of scratch, the static "
                        "scratch holds %zu (pass s and n2, use a shorter j range, or call "
                        "ps3_compute with a workspace)", need, ws_bytes);
        if ((st = scratch_of_current_device(&workspace)) != PS_OK) return st;
    }
    double* s_ws = nullptr;
    void* n2_ws = nullptr;
    int64_t* prefix = nullptr;
    float* partial = nullptr;
    if (is_mfma(path)) return ps3_mfma(V, n_f, n_v, ld, s, n2, j_begin, j_end, c3, workspace,
                                       ws_bytes, path, levels, opts ? opts->tile : 0, stream);
    const bool bits = is_bits(opts);
    const int32_t kdt = bits ? PS_B1 : dtype;   // operand type of the kernels
    const int cfg2 = choose_cfg(kdt, 2, bits ? PS_PATH_BITS : PS_PATH_VALU, n_f, n_v, opts);
    const Split sp2 = bits ? Split{1, 0} : plan_split(dtype, n_f, n_v, cfg2, opts);
    const int32_t nchunks = bits ? 1 : split_chunks(dtype, n_f, choose_acc(n_f, opts));
    const int64_t stage = ps3_stage_size(n_v, j_begin, j_end);
    uint32_t* packed = nullptr;
    const size_t need = ws3_layout(n_v, prefix3_entries(n_v, j_begin, j_end), s != nullptr,
                                   n2 != nullptr, dtype == PS_F64 ? 8 : 4,
                                   sp2.nchunks, dtype == PS_F64 ? -1 : nchunks, stage,
                                   bits ? bits_bytes(n_f, n_v) : 0, workspace, &s_ws, &n2_ws,
                                   &prefix, &partial, &packed);
    if (ws_bytes < need || !workspace)
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (!aligned(workspace, 256)) return fail(PS_ERR_ARG, "workspace is not 256-byte aligned");
    hipError_t e;
    if (!s) {
        e = launch_sums(V, dtype, n_f, n_v, ld, s_ws, nullptr, stream);
        if (e != hipSuccess) return hip_fail(e, "sums launch");
        s = s_ws;
    }
    // the kernels' operand: V itself, or its packed bits (words as elements)
    const void* KV = V;
    int64_t kn_f = n_f, kld = ld;
    if (bits) {
        e = launch_pack_bits((const uint8_t*)V, n_f, n_v, ld, packed, stream);
        if (e != hipSuccess) return hip_fail(e, "bit packing launch");
        KV = packed;
        kn_f = kld = bits_row_words(n_f);
    }
    if (!n2) {  // the pair numerators of Eq. 1 (the 2-way mGEMM prepass)
        Mg2Launch a{KV, kn_f, n_v, kld, s, nullptr, n2_ws, cfg2, sp2.nchunks, sp2.chunk_tiles,
                    partial};
        e = launch_mg2(kdt, a, stream);
        if (e == hipSuccess && sp2.nchunks > 1) e = launch_finish2(dtype, a, stream);
        if (e != hipSuccess) return hip_fail(e, "3-way numerator prepass launch");
        n2 = n2_ws;
    }
    const int cfg = choose_cfg(kdt, 3, bits ? PS_PATH_BITS : PS_PATH_VALU, n_f, n_v, opts);
    const int bm = kValuCfgs[cfg].bm();
    // one launch over the split tiling of the stage: colex (pair, k) tiles of
    // the slabs below js, lex (pair, i) tiles of the others
    const int64_t js = split3(n_v, j_begin, j_end);
    const int64_t nt0 = flat_tiles(n_v, j_begin, js, bm);
    Mg3Launch a{KV, kn_f, n_v, kld, s, n2, j_begin, j_end, c3, prefix,
                nt0 + lex_tiles(n_v, js, j_end, bm), cfg, nchunks,
                bits ? 0 : chunk_tiles(dtype, cfg), partial, kSlabSplit,
                js, nt0, prefix + flat_row_tiles(j_begin, js, bm) + 1};
    e = launch_mg3_prefix(a, stream);
    if (e == hipSuccess) e = launch_mg3(kdt, a, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "3-way launch");
}

}  // namespace ps

extern "C" {

ps_status ps2_compute(const void* V, int32_t dtype, int64_t n_f, int64_t n_v, int64_t ld,
                      const double* s, float* c2, void* n2, void* workspace, size_t ws_bytes,
                      const ps_opts* opts, hipStream_t stream) {
    return ps2_run(V, dtype, n_f, n_v, ld, s, c2, n2, 0, 1, workspace, ws_bytes, opts, stream);
}

ps_status ps2_compute_shard(const void* V, int32_t dtype, int64_t n_f, int64_t n_v, int64_t ld,
                            const double* s, float* c2, void* n2, int64_t shard,
                            int64_t nshards, void* workspace, size_t ws_bytes,
                            const ps_opts* opts, hipStream_t stream) {
    return ps2_run(V, dtype, n_f, n_v, ld, s, c2, n2, shard, nshards, workspace, ws_bytes, opts,
                   stream);
}

ps_status ps3_compute(const void* V, int32_t dtype, int64_t n_f, int64_t n_v, int64_t ld,
                      const double* s, const void* n2, int64_t j_begin, int64_t j_end,
                      float* c3, void* workspace, size_t ws_bytes, const ps_opts* opts,
                      hipStream_t stream) {
    return ps3_run(V, dtype, n_f, n_v, ld, s, n2, j_begin, j_end, c3, workspace, ws_bytes,
                   false, opts, stream);
}

ps_status ps3_compute_noalloc(const void* V, int32_t dtype, int64_t n_f, int64_t n_v,
                              int64_t ld, const double* s, const void* n2, int64_t j_begin,
                              int64_t j_end, float* c3, const ps_opts* opts,
                              hipStream_t stream) {
    return ps3_run(V, dtype, n_f, n_v, ld, s, n2, j_begin, j_end, c3, nullptr,
                   (size_t)PS_NOALLOC_SCRATCH_BYTES, true, opts, stream);
}

}  // extern "C"

namespace ps {

// ---------------------------------------------------------------------------
// Batched 2-way.
// ---------------------------------------------------------------------------
struct BatchLayout {
    DevProblem* probs = nullptr;
    BatchGroup* groups = nullptr;
    BatchTile* tiles = nullptr;
    double* s = nullptr;
    float* partial = nullptr;    // all split problems' chunk partials, back to back
    size_t bytes = 0;
};

static int64_t batch_sums_len(const ps_problem* p, int32_t n) {
    int64_t t = 0;
    for (int32_t i = 0; i < n; ++i)
        if (!p[i].s) t += p[i].n_v;
    return t;
}

static int64_t pairs_of(int64_t n_v) { return n_v * (n_v - 1) / 2; }

// Field chunks of problem p of a batch (each problem takes its own
// accumulation choice from its n_f).
static int32_t batch_chunks(const ps_problem& p, int32_t dt, const ps_opts* o) {
    return split_chunks(dt, p.n_f, choose_acc(p.n_f, o));
}

static int64_t batch_items(const ps_problem* p, int32_t n, int32_t dt, const ps_opts* o,
                           int bm) {
    int64_t t = 0;
    for (int32_t i = 0; i < n; ++i)
        if (p[i].n_v >= 2) t += tri_tiles(p[i].n_v, bm) * batch_chunks(p[i], dt, o);
    return t;
}

// Raw tile sums of every problem (all problems, split or not, go through the
// batched finish kernel).
static int64_t batch_partial_len(const ps_problem* p, int32_t n, int32_t dt, const ps_opts* o) {
    int64_t t = 0;
    for (int32_t i = 0; i < n; ++i)
        if (p[i].n_v >= 2) t += (int64_t)batch_chunks(p[i], dt, o) * pairs_of(p[i].n_v);
    return t;
}

// Field-chunk groups of a batch: one per (problem with pairs, chunk).
static int64_t batch_groups(const ps_problem* p, int32_t n, int32_t dt, const ps_opts* o) {
    int64_t t = 0;
    for (int32_t i = 0; i < n; ++i)
        if (p[i].n_v >= 2) t += batch_chunks(p[i], dt, o);
    return t;
}

static BatchLayout batch_layout(const ps_problem* p, int32_t n, int32_t dt, const ps_opts* o,
                                int bm, void* ws) {
    Carver c(ws);
    BatchLayout L;
    L.probs = (DevProblem*)c.take(sizeof(DevProblem) * (size_t)(n > 0 ? n : 1));
    L.groups = (BatchGroup*)c.take(sizeof(BatchGroup) * (size_t)batch_groups(p, n, dt, o));
    L.tiles = (BatchTile*)c.take(sizeof(BatchTile) * (size_t)batch_items(p, n, dt, o, bm));
    L.s = (double*)c.take(sizeof(double) * (size_t)batch_sums_len(p, n));
    L.partial = (float*)c.take(sizeof(float) * (size_t)batch_partial_len(p, n, dt, o));
    L.bytes = c.used;
    return L;
}

// Prefix the recorded message with the number of the problem it concerns
// (copied first: the message buffer is also the destination).
static ps_status prefix_error(ps_status st, int32_t i) {
    char msg[sizeof g_err];
    memcpy(msg, g_err, sizeof msg);
    msg[sizeof msg - 1] = 0;
    return fail(st, "problem %d: %s", i, msg);
}

static ps_status check_batch(const ps_problem* probs, int32_t n, int32_t dt, const ps_opts* o) {
    if (n < 0) return fail(PS_ERR_ARG, "n = %d < 0", n);
    if (n > 0 && !probs) return fail(PS_ERR_ARG, "probs is NULL");
    ps_status st = check_opts(o);
    if (st != PS_OK) return st;
    if (o && (is_mfma(o->path) || o->path == PS_PATH_BITS))
        return fail(PS_ERR_UNSUPPORTED, "batched runs on the VALU path only");
    if (dt == PS_F64) return fail(PS_ERR_UNSUPPORTED, "batched calls take F32, F16 or U8 data");
    for (int32_t i = 0; i < n; ++i) {
        const ps_problem& p = probs[i];
        st = check_matrix(p.V, dt, p.n_f, p.n_v, p.ld);
        if (st != PS_OK) return prefix_error(st, i);
        if (p.n_v >= 2 && !p.c2 && !p.n2)
            return fail(PS_ERR_ARG, "problem %d: both c2 and n2 are NULL", i);
        if (!aligned(p.c2, 4) || !aligned(p.n2, 4) || !aligned(p.s, 8))
            return fail(PS_ERR_ARG, "problem %d: misaligned pointer", i);
        if (p.n_v > ((int64_t)1 << 31) / 2) return fail(PS_ERR_ARG, "problem %d too large", i);
        st = check_int_range(PS_PATH_VALU, dt, p.n_f);
        if (st != PS_OK) return prefix_error(st, i);
    }
    return PS_OK;
}

// Host-side tables of a batch: device problem records (with workspace sums
// and chunk partials where needed) and the groups of the work list.  A group
// is one field chunk of one problem; it lists the problem's tiles in
// column-major order, each item costing the fields its chunk covers.  The
// groups are packed onto the XCDs by total cost (largest first, to the least
// loaded), and each XCD's list holds its groups longest item first.
struct BatchTables {
    std::vector<DevProblem> dp;
    std::vector<BatchGroup> groups;
    int64_t ntiles = 0, max_nv = 0, max_pairs = 0;
    int64_t xcd_start[kXcds] = {}, xcd_len[kXcds] = {};
};

static BatchTables batch_tables(const ps_problem* probs, int32_t n, int32_t dt, const ps_opts* o,
                                int bm, const BatchLayout& L) {
    BatchTables T;
    T.dp.resize(n);
    int64_t soff = 0, poff = 0;
    for (int32_t i = 0; i < n; ++i) {
        const ps_problem& p = probs[i];
        const int32_t nch = p.n_v >= 2 ? batch_chunks(p, dt, o) : 1;
        T.dp[i] = DevProblem{p.V, p.n_f, p.n_v, p.ld, p.s, p.c2, p.n2, nullptr, nch, p.s ? 0 : 1};
        if (!p.s) {
            T.dp[i].s = L.s + soff;
            soff += p.n_v;
        }
        if (p.n_v >= 2) {
            T.dp[i].partial = L.partial + poff;
            poff += (int64_t)nch * pairs_of(p.n_v);
            T.max_pairs = std::max(T.max_pairs, pairs_of(p.n_v));
        }
        T.max_nv = std::max(T.max_nv, p.n_v);
    }
    struct G { int64_t cost, tiles; BatchGroup g; int x; };
    std::vector<G> gs;
    for (int32_t pi = 0; pi < n; ++pi) {
        if (probs[pi].n_v < 2) continue;
        const int32_t nch = T.dp[pi].nchunks;
        for (int32_t c = 0; c < nch; ++c) {
            const int64_t f0 = nch > 1 ? c * kChunkFields : 0;
            const int64_t f1 = nch > 1 ? std::min(probs[pi].n_f, f0 + kChunkFields) : probs[pi].n_f;
            gs.push_back(G{f1 - f0, tri_tiles(probs[pi].n_v, bm), BatchGroup{pi, c, 0}, 0});
        }
    }
    // groups onto XCDs: largest total cost first, each to the least loaded
    // XCD (ties: the lower index, so the packing is deterministic)
    std::vector<size_t> by_total(gs.size());
    for (size_t k = 0; k < gs.size(); ++k) by_total[k] = k;
    std::stable_sort(by_total.begin(), by_total.end(), [&](size_t a, size_t b) {
        return gs[a].cost * gs[a].tiles > gs[b].cost * gs[b].tiles;
    });
    int64_t load[kXcds] = {};
    for (size_t k : by_total) {
        int x = 0;
        for (int y = 1; y < kXcds; ++y)
            if (load[y] < load[x]) x = y;
        gs[k].x = x;
        load[x] += gs[k].cost * gs[k].tiles;
    }
    // each XCD's list: its groups by the fields of their items, longest
    // first (stable: problem and chunk order otherwise)
    std::stable_sort(gs.begin(), gs.end(), [](const G& a, const G& b) {
        return a.x != b.x ? a.x < b.x : a.cost > b.cost;
    });
    T.groups.resize(gs.size());
    for (size_t k = 0; k < gs.size(); ++k) {
        T.groups[k] = gs[k].g;
        T.groups[k].start = T.ntiles;
        T.xcd_len[gs[k].x] += gs[k].tiles;
        T.ntiles += gs[k].tiles;
    }
    for (int x = 1; x < kXcds; ++x) T.xcd_start[x] = T.xcd_start[x - 1] + T.xcd_len[x - 1];
    return T;
}

// The whole batched sequence on one stream: table upload (through kernel
// arguments), work-list expansion, sums, tile sums, finish.  Nothing waits on
// the host, so the same sequence serves eager calls and graph capture.
static ps_status batch_enqueue(const BatchLayout& L, const BatchTables& T, int32_t n, int32_t dt,
                               int cfg, hipStream_t st) {
    hipError_t e = launch_put(L.probs, T.dp.data(), sizeof(DevProblem) * (size_t)n, st);
    if (e == hipSuccess && !T.groups.empty())
        e = launch_put(L.groups, T.groups.data(), sizeof(BatchGroup) * T.groups.size(), st);
    if (e == hipSuccess)
        e = launch_batch_expand(L.groups, (int32_t)T.groups.size(), L.tiles, T.ntiles, st);
    if (e == hipSuccess) e = launch_batched_sums(L.probs, n, dt, T.max_nv, st);
    if (e == hipSuccess) {
        MgBatchLaunch a{L.probs, L.tiles, T.ntiles, cfg, chunk_tiles(dt, cfg), {}, {}};
        for (int x = 0; x < kXcds; ++x) {
            a.xcd_start[x] = T.xcd_start[x];
            a.xcd_len[x] = T.xcd_len[x];
        }
        e = launch_mgb(dt, a, st);
    }
    if (e == hipSuccess) e = launch_finish2_batched(dt, L.probs, n, T.max_pairs, st);
    return e == hipSuccess ? PS_OK : hip_fail(e, "batched launch");
}

}  // namespace ps

extern "C" {

size_t ps2_batched_workspace_size(const ps_problem* probs, int32_t n, int32_t dtype,
                                  const ps_opts* opts) {
    if (n < 0 || (n > 0 && !probs) || elem_size(dtype) == 0) return 0;
    const int cfg = batch_cfg(probs, n, dtype, opts);
    if (cfg < 0 || cfg >= kNumValuCfgs) return 0;
    return batch_layout(probs, n, dtype, opts, kValuCfgs[cfg].bm(), nullptr).bytes;
}

ps_status ps2_compute_batched(const ps_problem* probs, int32_t n, int32_t dtype, void* ws,
                              size_t ws_bytes, const ps_opts* opts, hipStream_t stream) {
    ps_status st = check_batch(probs, n, dtype, opts);
    if (st != PS_OK) return st;
    if (n == 0) return PS_OK;
    const int cfg = batch_cfg(probs, n, dtype, opts);
    const int bm = kValuCfgs[cfg].bm();
    const BatchLayout L = batch_layout(probs, n, dtype, opts, bm, ws);
    if (ws_bytes < L.bytes || !ws)
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.bytes);
    if (!aligned(ws, 256)) return fail(PS_ERR_ARG, "workspace is not 256-byte aligned");
    const BatchTables T = batch_tables(probs, n, dtype, opts, bm, L);
    return batch_enqueue(L, T, n, dtype, cfg, stream);
}

}  // extern "C"

struct ps_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Captures enqueue(cs) on a private stream into a graph and instantiates it.
template <class Enqueue>
static ps_status capture_plan(ps_plan** plan, Enqueue enqueue) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "plan capture stream");
    ps_plan* p = new ps_plan();
    ps_status st;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue(cs);
        hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
        if (st == PS_OK && e2 != hipSuccess) st = hip_fail(e2, "plan capture");
    } else {
        st = hip_fail(e, "plan capture begin");
    }
    if (st == PS_OK) {
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_fail(e, "plan instantiate");
    }
    (void)hipStreamDestroy(cs);
    if (st != PS_OK) {
        ps_plan_destroy(p);
        return st;
    }
    *plan = p;
    return PS_OK;
}

extern "C" {

ps_status ps_plan_create_batched(ps_plan** plan, const ps_problem* probs, int32_t n,
                                 int32_t dtype, const ps_opts* opts, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
    (void)stream;   // creation launches nothing: the tables travel inside the graph
    if (!plan) return fail(PS_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    ps_status st = check_batch(probs, n, dtype, opts);
    if (st != PS_OK) return st;
    const int cfg = batch_cfg(probs, n, dtype, opts);
    const int bm = kValuCfgs[cfg].bm();
    const BatchLayout L = batch_layout(probs, n, dtype, opts, bm, ws);
    if (ws_bytes < L.bytes || !ws)
        return fail(PS_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.bytes);
    if (!aligned(ws, 256)) return fail(PS_ERR_ARG, "workspace is not 256-byte aligned");
    const BatchTables T = batch_tables(probs, n, dtype, opts, bm, L);
    return capture_plan(plan, [&](hipStream_t cs) {
        return n > 0 ? batch_enqueue(L, T, n, dtype, cfg, cs) : PS_OK;
    });
}

ps_status ps_plan_create_3way(ps_plan** plan, const void* V, int32_t dtype, int64_t n_f,
                              int64_t n_v, int64_t ld, const double* s, const void* n2,
                              int64_t j_begin, int64_t j_end, float* c3, void* ws,
                              size_t ws_bytes, const ps_opts* opts) {
    if (!plan) return fail(PS_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    // the options are read now: the captured launches keep their values
    ps_opts o{};
    if (opts) o = *opts;
    const ps_opts* op = opts ? &o : nullptr;
    return capture_plan(plan, [&](hipStream_t cs) {
        return ps3_run(V, dtype, n_f, n_v, ld, s, n2, j_begin, j_end, c3, ws, ws_bytes, false,
                       op, cs);
    });
}

ps_status ps_plan_execute(ps_plan* plan, hipStream_t stream) {
    if (!plan || !plan->exec) return fail(PS_ERR_ARG, "plan is NULL or empty");
    hipError_t e = hipGraphLaunch(plan->exec, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "plan launch");
}

void ps_plan_destroy(ps_plan* plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
}

}  // extern "C"

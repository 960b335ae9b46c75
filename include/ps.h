/*
 * ps.h -- C ABI of libps, the MI355X (gfx950) library for the 2-way and
 * 3-way Proportional Similarity (PS, Czekanowski) metric of Joubert et al.,
 * "Parallel Accelerated Vector Similarity Calculations for Genomics
 * Applications" (arXiv 1705.08210).
 *
 * Notation (0-based).  V holds n_v non-negative vectors of n_f fields.
 * Vector i is stored at V[i*ld + q], q < n_f, ld >= n_f elements: the
 * column-major n_f x n_v matrix of Section 3.1.
 *
 *   s_i        = sum_q v_{i,q}                              (Section 2.1)
 *   n2(i,j)    = sum_q min(v_{i,q}, v_{j,q})                (Section 2.1)
 *   c2(i,j)    = 2 n2(i,j) / (s_i + s_j)                    (Section 2.1)
 *   n3'(i,j,k) = sum_q min(v_{i,q}, v_{j,q}, v_{k,q})       (Section 2.2)
 *   n3(i,j,k)  = n2(i,j) + n2(i,k) + n2(j,k) - n3'(i,j,k)   (Section 2.2, Eq. 1)
 *   c3(i,j,k)  = (3/2) n3 / (s_i + s_j + s_k)               (Section 2.2)
 *
 * A metric whose denominator is 0 (all-zero vectors) is returned as 0.
 * Only distinct tuples are produced: pairs i<j and triples i<j<k (the
 * symmetry reductions of Sections 2.1 and 2.2).
 *
 * Packed output layouts
 *   2-way, colex:  index(i,j) = j(j-1)/2 + i,  i < j.   For a fixed j the
 *                  i are contiguous.
 *   3-way, j-slab: index(i,j,k) = off(j) + (k-j-1) j + i,  i < j < k,
 *                  off(j) = sum_{t<j} t (n_v-1-t).  Middle index j is the
 *                  slowest, so the triples of a range of j values (a stage,
 *                  Section 4.2) form one contiguous block.
 *
 * Conventions
 *  - Every pointer argument named V, s, c2, c3, n2, bad_count or workspace
 *    is a DEVICE pointer owned by the caller.  Problem and option structs
 *    are host memory, read during the call only.
 *  - Calls are asynchronous on `stream` (0 = the null stream) and never
 *    synchronise the device.  The library allocates no memory that the
 *    caller sees; scratch comes from the caller's workspace, sized by the
 *    matching *_workspace_size call.
 *  - Arguments are checked before anything is launched; on an error nothing
 *    is written and ps_last_error() describes it.  Faults in kernels show up
 *    at the caller's next synchronisation.
 *  - Inputs outside the domain (negative, NaN, Inf) are not checked on the
 *    compute path; ps_vector_sums counts them.  Results for such inputs are
 *    unspecified.
 *  - Thread safety: calls may be made from several host threads; calls that
 *    share a workspace buffer must be ordered by the caller.
 *  - Work lists longer than one dispatch allows (2^32 work-items) are split
 *    over several launches on the same stream.  The environment variable
 *    PS_MAX_GRID_BLOCKS (read once per process, a testing aid) lowers the
 *    blocks per launch so that small problems take that path too.
 */
#ifndef PS_H
#define PS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PS_OK = 0,
    PS_ERR_ARG = 1,          /* bad size, null pointer, misaligned pointer */
    PS_ERR_DTYPE = 2,        /* unknown or unsupported storage type */
    PS_ERR_WORKSPACE = 3,    /* workspace too small (see *_workspace_size) */
    PS_ERR_HIP = 4,          /* a HIP runtime call failed */
    PS_ERR_UNSUPPORTED = 5   /* valid request the library does not implement */
} ps_status;

/* Storage type of V. */
typedef enum {
    PS_F32 = 0,   /* float;   FP32 min, FP32 accumulation                     */
    PS_F16 = 1,   /* _Float16; packed FP16 min, FP32 accumulation             */
    PS_U8 = 2,    /* uint8 integer levels; exact integer arithmetic           */
    PS_F64 = 3    /* double;  FP64 min, FP64 accumulation (the paper's
                     double-precision build, Section 5); c2/c3 outputs are
                     still float, raw numerators (n2) are double.  Not for
                     the batched calls. */
} ps_dtype;

/* FP32 accumulation of the numerator sums (floating storage only).  A NULL
 * opts means PS_ACC_AUTO; a zero-filled ps_opts means PS_ACC_PLAIN. */
typedef enum {
    PS_ACC_PLAIN = 0,    /* one running FP32 sum per output over all fields */
    PS_ACC_BLOCKED = 1,  /* the fields are split into chunks of 4096, each
                            chunk is summed in FP32 and the chunk sums are
                            added in FP64 in a fixed order (deterministic;
                            needs workspace for the chunk partials; batched
                            calls split the same way per problem) */
    PS_ACC_AUTO = 2      /* BLOCKED when n_f > 4096, else PLAIN; a 2-way
                            triangle too small to fill the chip is also split
                            over field chunks so that enough workgroups run */
} ps_acc;

/* Compute path for the pair numerators. */
typedef enum {
    PS_PATH_AUTO = 0,    /* U8 with 1 <= levels <= 15 and rows within the MFMA
                            limits below: MFMA; otherwise VALU */
    PS_PATH_VALU = 1,    /* register-blocked min/add on the vector ALUs */
    PS_PATH_MFMA = 2,    /* alias PS_PATH_MFMA_THERMO.  U8 only:
                            min(a,b) = sum_{t=1..levels} [a>=t][b>=t], an
                            exact int8 matrix-core contraction with int32
                            accumulation; needs levels >= max(V).  With the
                            default wave layout (opts.tile != 2) the level
                            planes are formed in registers from V's bytes (no
                            plane workspace) when levels * n_f < 2^31 for
                            levels <= 7, < 2^24 for more levels; a tile of 256
                            rows of V is addressed with 32-bit offsets, so
                            256 * ld + 256 < 2^31 bytes (3-way also
                            n_v < 2^21).  Otherwise the
                            planes are written to the workspace first (levels
                            x n_f rounded up to 128 fields per row, one byte
                            per value for int8, half a byte for FP4) and 256
                            plane rows must span < 2^31 bytes.  Beyond these
                            limits: PS_ERR_UNSUPPORTED */
    PS_PATH_MFMA_FP4 = 3, /* U8 only: the same 0/1 planes as FP4 (e2m1) operands
                            of the scaled matrix-core instruction, FP32
                            accumulation (exact: sums are integers < 2^24,
                            needs levels * n_f < 2^24); needs levels >= max(V) */
    PS_PATH_BITS = 4     /* U8 binary data, values in {0, 1} (opts.levels = 1):
                            the Sorensen special case of Section 2.3, where min
                            is AND.  The fields are packed 32 to a word and a
                            word pair costs an AND and a population count;
                            exact integer sums.  2-way and 3-way.  Values above
                            1 are outside this path's domain (results
                            unspecified). */
} ps_path;
#define PS_PATH_MFMA_THERMO PS_PATH_MFMA

typedef struct {
    int32_t acc;      /* ps_acc */
    int32_t path;     /* ps_path */
    int32_t levels;   /* PS_U8 + MFMA: upper bound on the values of V, 1..127;
                         PS_U8 + BITS: must be 1 */
    int32_t tile;     /* 0 = library choice (tuning table); else 1 + index
                         into the tile configurations of ps_tile_config */
} ps_opts;

/* Human-readable name of a status code (static string). */
const char* ps_status_string(ps_status st);
/* Message of the last error on the calling host thread (static per thread). */
const char* ps_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int32_t ps_version(void);

/*
 * Per-vector sums s_i = sum_q v_{i,q} (the denominator terms of Sections 2.1
 * and 2.2), accumulated in FP64 (exact for PS_U8).
 *   V          device, n_v vectors, element type `dtype`, stride ld >= n_f
 *   s          device, n_v doubles (written)
 *   bad_count  device int32 or NULL; when given it is overwritten with the
 *              number of entries that are negative, NaN or infinite
 * n_v == 0 is a no-op.  Errors: PS_ERR_ARG, PS_ERR_DTYPE, PS_ERR_HIP.
 */
ps_status ps_vector_sums(const void* V, int32_t dtype, int64_t n_f, int64_t n_v,
                         int64_t ld, double* s, int32_t* bad_count,
                         hipStream_t stream);

/* Workspace bytes that ps2_compute needs for these arguments (0 if none).
 * s_given / n2 are as they will be passed to ps2_compute. */
size_t ps2_workspace_size(int32_t dtype, int64_t n_f, int64_t n_v,
                          int32_t s_given, const ps_opts* opts);

/*
 * 2-way metric over all pairs i<j (Section 2.1) via the min-product
 * "mGEMM" N2 = V^T o_min V of Section 3.1, restricted to the upper triangle.
 *   s       device FP64 sums from ps_vector_sums, or NULL to compute them
 *           into the workspace
 *   c2      device float, n_v(n_v-1)/2, colex layout; may be NULL if n2 given
 *   n2      device, optional raw numerators n2(i,j) in colex layout: float
 *           for PS_F32/PS_F16, double for PS_F64, int32 for PS_U8 (every
 *           path); may be NULL
 *   workspace / ws_bytes   device scratch, at least ps2_workspace_size()
 *   opts    may be NULL (all defaults)
 * Each c2 is formed in FP64 from the numerator and FP64 sums, then rounded
 * once to FP32.  n_v < 2 writes nothing.
 */
ps_status ps2_compute(const void* V, int32_t dtype, int64_t n_f, int64_t n_v,
                      int64_t ld, const double* s, float* c2, void* n2,
                      void* workspace, size_t ws_bytes, const ps_opts* opts,
                      hipStream_t stream);

/*
 * One GPU's share of ps2_compute when the pairs are spread over nshards GPUs
 * by tiles (the single-node analogue of the block-circulant distribution of
 * the pair blocks over processors, Section 4.1): the upper-triangle tiles of
 * the chosen tile configuration are numbered t = bj (bj + 1) / 2 + bi
 * (bi <= bj, block rows/columns of ps_tile_config's edge), and this call
 * computes the tiles t with t mod nshards == shard, writing c2 (and n2) at
 * those tiles' pairs only.  It takes the same tile configuration, field-chunk
 * plan and workspace (ps2_workspace_size) as ps2_compute with these
 * arguments, so the calls for shard = 0 .. nshards-1 together write every
 * pair once, bit for bit as one ps2_compute call.  Arguments as for
 * ps2_compute, with the full-size c2 / n2 arrays.  VALU and BITS paths only
 * (MFMA paths with nshards > 1: PS_ERR_UNSUPPORTED); nshards = 1 is
 * ps2_compute.  Errors: as ps2_compute; PS_ERR_ARG unless
 * 0 <= shard < nshards.
 */
ps_status ps2_compute_shard(const void* V, int32_t dtype, int64_t n_f, int64_t n_v,
                            int64_t ld, const double* s, float* c2, void* n2,
                            int64_t shard, int64_t nshards, void* workspace,
                            size_t ws_bytes, const ps_opts* opts, hipStream_t stream);

/* Workspace bytes that ps3_compute needs for the stage [j_begin, j_end)
 * (s_given / n2_given as they will be passed). */
size_t ps3_workspace_size(int32_t dtype, int64_t n_f, int64_t n_v,
                          int32_t s_given, int32_t n2_given, int64_t j_begin,
                          int64_t j_end, const ps_opts* opts);

/*
 * 3-way metric over the triples i<j<k whose middle index j lies in
 * [j_begin, j_end) (Section 2.2, Eq. 1; the per-j slices B_j = X_j^T o_min V
 * of Section 3.2, with X_j = min(V, v_j) formed while staging operands and
 * never stored).  A stage of the paper's staged runs (Section 4.2) is a j
 * range; calling with consecutive ranges and concatenating the outputs gives
 * the full j-slab layout.
 *   s      device FP64 sums, or NULL (computed into the workspace)
 *   n2     device pair numerators in colex layout (float for F32/F16, double
 *          for F64, int32 for U8, as written by ps2_compute for the same V),
 *          or NULL to compute them into the workspace
 *   opts   path VALU, BITS (binary U8 data, X_j = V AND v_j), or for U8
 *          data the MFMA paths, exact: a pair's row is staged as the
 *          bytewise min of its two vectors and thresholded per level,
 *          [min(a,b) >= t][c >= t] = [min(a,b,c) >= t]; the int8 path tiles
 *          the stage as pairs x vectors (ps_tile_config, way 3); AUTO picks
 *          as for ps2_compute
 *   c3     device float; receives the triples of [j_begin, j_end) packed in
 *          j-slab order starting at offset 0 (i.e. at global index
 *          off(j_begin))
 * Needs 1 <= j_begin <= j_end <= n_v-1 (empty range writes nothing).
 */
ps_status ps3_compute(const void* V, int32_t dtype, int64_t n_f, int64_t n_v,
                      int64_t ld, const double* s, const void* n2,
                      int64_t j_begin, int64_t j_end, float* c3,
                      void* workspace, size_t ws_bytes, const ps_opts* opts,
                      hipStream_t stream);

/*
 * ps3_compute without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Arguments, outputs and results are those of
 * ps3_compute; the call allocates nothing: its scratch is a static device
 * array of PS_NOALLOC_SCRATCH_BYTES bytes that each GPU the library runs on
 * holds from the library's first use there until the process ends.  The
 * array of the calling thread's current device is used, so `stream` must
 * belong to that device.
 *   Scratch need: the value of ps3_workspace_size() for the same arguments.
 *   With s and n2 given and n_f <= 4096 it is a few tens of KB; computing
 *   the pair numerators inside takes C(n_v, 2) values plus field-chunk
 *   partials.  A call that needs more than PS_NOALLOC_SCRATCH_BYTES returns
 *   PS_ERR_WORKSPACE before anything is launched.
 *   Every call on one GPU shares that GPU's array, which keeps the last
 *   call's contents: calls that overlap on one GPU (on different streams,
 *   or from several host threads without ordering) race and give wrong
 *   results.  Order them on one stream.
 */
#define PS_NOALLOC_SCRATCH_BYTES (32u << 20)
ps_status ps3_compute_noalloc(const void* V, int32_t dtype, int64_t n_f, int64_t n_v,
                              int64_t ld, const double* s, const void* n2,
                              int64_t j_begin, int64_t j_end, float* c3,
                              const ps_opts* opts, hipStream_t stream);

/* Number of c3 values of the stage [j_begin, j_end): off(j_end)-off(j_begin). */
int64_t ps3_stage_size(int64_t n_v, int64_t j_begin, int64_t j_end);

/* One independent 2-way problem of a batch (all pointers device). */
typedef struct {
    const void* V;       /* n_v vectors, stride ld */
    int64_t n_f, n_v, ld;
    const double* s;     /* NULL: computed into the workspace */
    float* c2;           /* colex, n_v(n_v-1)/2 floats (or NULL if n2 given) */
    void* n2;            /* optional raw numerators, colex */
} ps_problem;

/* Workspace bytes for a batch of problems. */
size_t ps2_batched_workspace_size(const ps_problem* probs, int32_t n,
                                  int32_t dtype, const ps_opts* opts);

/*
 * Many independent uneven 2-way problems in one launch over a combined list
 * of (problem, tile, field chunk) work items (the load-balancing idea of
 * Section 4.1 applied to the tiles of one GPU): the (problem, field chunk)
 * groups are packed onto the GPU's dies by cost and each die takes its list
 * longest item first as slots free up.  A finish pass forms every problem's
 * c2 (and n2).  The problem
 * table and the list's groups travel to the workspace as kernel arguments
 * and a kernel expands the list there, so the call returns without waiting
 * for anything and the host arrays may be freed at once.  All problems share
 * `dtype` (F32, F16 or U8; VALU path only, else PS_ERR_UNSUPPORTED).
 */
ps_status ps2_compute_batched(const ps_problem* probs, int32_t n, int32_t dtype,
                              void* workspace, size_t ws_bytes,
                              const ps_opts* opts, hipStream_t stream);

/* A captured batch: the whole launch sequence of ps2_compute_batched (table
 * writes, work-list expansion, sums, tile sums, finish) in a HIP graph. */
typedef struct ps_plan ps_plan;

/* Captures the sequence into a graph (on a private stream; nothing is
 * launched at creation, `stream` is not used).  The workspace must stay
 * valid and untouched by others until ps_plan_destroy. */
ps_status ps_plan_create_batched(ps_plan** plan, const ps_problem* probs,
                                 int32_t n, int32_t dtype, const ps_opts* opts,
                                 void* workspace, size_t ws_bytes,
                                 hipStream_t stream);
/* A captured 3-way stage: the whole launch sequence of ps3_compute for these
 * arguments (sums and pair numerators when not given, slab prefixes, the
 * slices over [j_begin, j_end), Eq. 1) in a HIP graph, for campaigns that
 * replay a stage shape many times (Section 4.2 staging; Section 3.2 slices).
 * Arguments as for ps3_compute; they are checked while capturing and every
 * pointer is baked into the graph, so V, s, n2, c3 and the workspace must
 * stay valid (their contents may change between replays) until
 * ps_plan_destroy.  Nothing is launched at creation.  Errors: those of
 * ps3_compute, or PS_ERR_HIP when capture fails. */
ps_status ps_plan_create_3way(ps_plan** plan, const void* V, int32_t dtype, int64_t n_f,
                              int64_t n_v, int64_t ld, const double* s, const void* n2,
                              int64_t j_begin, int64_t j_end, float* c3,
                              void* workspace, size_t ws_bytes, const ps_opts* opts);
/* Replays the captured graph on `stream`. */
ps_status ps_plan_execute(ps_plan* plan, hipStream_t stream);
void ps_plan_destroy(ps_plan* plan);

/*
 * Tile configurations (for tuning).  `way` is 2 or 3.  Returns the number of
 * compiled configurations for (dtype, way, path); when idx is in range
 * writes the output-tile rows/cols and field-tile depth of configuration idx.
 * VALU and BITS paths: the tile shapes that opts.tile = 1 + idx selects.
 * PS_PATH_MFMA (PS_U8, way 2): the tile orders of the int8 matrix-core
 * kernel, all 256 x 256 x 128: configuration idx walks the upper triangle in
 * groups of 2^idx block columns (tiles running side by side share rows in
 * L2); chosen through ps_tune_register only.
 * PS_PATH_MFMA (PS_U8, way 3, register-formed levels): two tilings of the
 * slices, both of 256 x 256 output tiles with 128-field tiles; opts.tile =
 * 1 + idx selects one.  idx 0 (also opts.tile = 0): the split tiling, whose
 * rows are the pairs (i, j) of slabs j < 2 n_v / 5 with columns k, and the
 * pairs (j, k) of the later slabs with columns i, so every tile is whole;
 * it needs n_v ld < 2^31 bytes and a pair table below 2^31 bytes, else
 * idx 1 runs.  idx 1: per-slab tiles, whole 256 x 256 tiles inside each
 * slab and 128 x 128 tiles over its ragged edges.
 */
int32_t ps_tile_config(int32_t dtype, int32_t way, int32_t path, int32_t idx,
                       int32_t* bm, int32_t* bn, int32_t* bk);

/* Register a tuned choice for problems with n_f in [nf_lo, nf_hi) and n_v in
 * [nv_lo, nv_hi); later registrations take precedence.  Host-side table only.
 *   path VALU / BITS, way 2, 3 (or 0: batched): idx = the tile configuration
 *     the library uses when opts.tile = 0;
 *   path MFMA, way 2, PS_U8: idx = the matrix-core tile order (above);
 *   path AUTO, way 2 or 3, PS_U8: idx = the ps_path (VALU, MFMA or
 *     MFMA_FP4) that opts.path = AUTO takes for integer levels (1..15), used
 *     when that path can take the shape.
 * Errors: PS_ERR_DTYPE, PS_ERR_ARG (way, path or idx out of range). */
ps_status ps_tune_register(int32_t dtype, int32_t way, int32_t path,
                           int64_t nf_lo, int64_t nf_hi, int64_t nv_lo,
                           int64_t nv_hi, int32_t idx);
/* The path (a ps_path value other than AUTO) that ps2_compute (way 2) or
 * ps3_compute (way 3) takes for these arguments: opts.path itself unless it
 * is AUTO, else the library's choice (policy and tuning table).  -1 for an
 * unknown dtype or way. */
int32_t ps_path_choice(int32_t dtype, int32_t way, int64_t n_f, int64_t n_v, int64_t ld,
                       const ps_opts* opts);

/* Forget all registered choices. */
void ps_tune_clear(void);

/*
 * Output reduction on the device (the output handling of Section 6.5, where
 * each metric is stored as one unsigned byte and thresholding is named as
 * the way to cut the volume of a campaign's output).
 */

/* q[i] = round-half-even(255 * clamp(c[i], 0, 1)) for i < n: one byte per
 * metric (about 2.5 significant figures).  c, q device pointers (any
 * alignment); n >= 0.  Errors: PS_ERR_ARG for n < 0 or a NULL pointer with
 * n > 0. */
ps_status ps_quantize_u8(const float* c, int64_t n, uint8_t* q, hipStream_t stream);

/* Workspace bytes of ps_threshold for n entries. */
size_t ps_threshold_workspace_size(int64_t n);

/*
 * Thresholding: the entries i < n with c[i] >= threshold, in increasing i.
 *   idx, val   device outputs with room for `cap` entries: idx = base + i
 *              (base turns stage-relative positions into global ones, e.g.
 *              the packed index of a stage's first triple), val = c[i]
 *   count      device int64: the number of entries selected; when it
 *              exceeds cap only the first cap are written
 *   workspace  device scratch of ps_threshold_workspace_size(n) bytes,
 *              256-byte aligned
 * Deterministic.  Errors: PS_ERR_ARG (n < 0, cap < 0, NULL or misaligned
 * pointers), PS_ERR_WORKSPACE.
 */
ps_status ps_threshold(const float* c, int64_t n, float threshold, int64_t base,
                       int64_t* idx, float* val, int64_t cap, int64_t* count,
                       void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Measurement aid (not part of the metric): the shader clock under a full
 * vector-ALU load.  Launches 2048 workgroups of 256 lanes, each running
 * `iters` rounds of FP32 min + add on 8 independent chains; the first lane of
 * each workgroup writes three uint64 values to the workspace: shader-clock
 * cycles elapsed, 100 MHz real-time ticks elapsed, and a zero.  The mean
 * clock in GHz is sum(cycles) / sum(ticks) / 10.  workspace: device, at
 * least ps_clock_probe_workspace_size() bytes, 8-byte aligned.
 */
size_t ps_clock_probe_workspace_size(void);
ps_status ps_clock_probe(int64_t iters, void* workspace, size_t ws_bytes,
                         hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PS_H */

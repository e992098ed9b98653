/*
 * selfjoin.h -- C ABI of the MI355X (gfx950) epsilon-distance self-join.
 *
 * Problem (Gallet & Gowanlock, "Leveraging GPU Tensor Cores for Double
 * Precision Euclidean Distance Calculations", Section II-A, Eq. (1)): given n
 * points V in d dimensions (FP64) and a search distance eps, report every
 * ordered pair (a, b) of V x V whose Euclidean distance is at most eps; each
 * point pairs with itself (Section IV-A counts it in |R|).
 *
 * Exact result. A pair (i, j) is in R iff d2(i, j) <= fl(eps * eps), where
 * d2 is accumulated over dimensions in ascending order starting at +0.0, each
 * step delta = fl(x_i[t] - x_j[t]) then acc = fma(delta, delta, acc)
 * (Section III-A, Eq. (2): the distance as a chain of multiply-accumulate
 * steps). Every path below returns exactly this set; the low-precision and
 * matrix-core paths reach it by re-evaluating, with this chain, every pair
 * whose fast value lies inside a proven error band around eps^2.
 *
 * Method (Sections II-D, III-A, III-B): points are bucketed into a uniform grid
 * with cells of side eps ("search"), and each group of queries from the same
 * run of cells is refined against the points of the neighbouring cells with
 * distance tiles in the expanded form |a|^2 + |b|^2 - 2 a.b (Eq. (3), Fig. 2),
 * computed as matrix multiply-accumulate tiles on MFMA.
 *
 * Conventions for every function:
 *  - Pointers marked "device" are device memory of the current HIP device
 *    (e.g. a torch tensor's data_ptr()); "host" pointers are host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; a function returns after the host-visible
 *    outputs it names (totals, cursors) are known, which synchronises that
 *    stream. Device outputs are complete when the stream reaches that point.
 *  - Calls never throw; they return a status. On error, outputs are left
 *    unchanged except where stated; selfjoin_last_error() gives detail.
 *  - Argument validation happens on the host before any device call, so an
 *    invalid call returns SJ_ERR_INVALID even on a machine without a GPU.
 */
#ifndef SELFJOIN_H
#define SELFJOIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sj_grid sj_grid; /* opaque grid index handle */

typedef enum {
    SJ_OK = 0,
    SJ_ERR_INVALID = 1,     /* bad argument or non-finite coordinate */
    SJ_ERR_OOM = 2,         /* device allocation failed */
    SJ_ERR_HIP = 3,         /* a HIP runtime call failed */
    SJ_ERR_CAPACITY = 4,    /* output buffer too small (see selfjoin_pairs) */
    SJ_ERR_UNSUPPORTED = 5  /* valid but not supported by this library */
} sj_status;

/* Distance-tile path. All return the same exact set R.
 *  SJ_FP64_VALU : direct form of Eq. (1)/(2) on the FP64 vector ALU -- the
 *                 comparison path (the paper's CUDA-core baseline role).
 *  SJ_FP64_MFMA : Gram-form tiles (Eq. (3), Fig. 2) on FP64 MFMA.
 *  SJ_FP32_MFMA : Gram-form tiles on FP32 MFMA with FP32 accumulation, inputs
 *                 centred per work group; FP64 recheck of the band.
 *  SJ_BF16_MFMA : as FP32 but BF16 inputs, FP32 accumulation.
 *  SJ_BF16X3_MFMA : split BF16 -- each centred coordinate as hi + lo BF16
 *                 parts (about 16 significant bits), three BF16 MFMAs per
 *                 tile (lo.hi, hi.lo, hi.hi), FP32 accumulation; its band is
 *                 about an order of magnitude narrower than SJ_BF16_MFMA's
 *                 (the dropped lo.lo products and the FP32 accumulation set
 *                 it), same FP64 recheck.
 *  SJ_FP8_MFMA  : FP8 (E4M3) tiles, FP32 accumulation, as a filter: its band
 *                 is wider than eps^2 (4 significant bits), so no pair is
 *                 accepted by the tiles alone; they reject the candidates
 *                 beyond eps^2 + Delta and every other pair takes the FP64
 *                 recheck.
 * (Other MFMA precisions are the paper's future work, Section V.)
 *
 * Range guards. Every path returns the exact set for every finite input; a
 * path whose arithmetic could overflow on the given data hands the call to
 * the next path down, which returns the same set (sj_stats.path_run says
 * which ran):
 *  - FP32 / BF16 / split BF16 / FP8: the tiles work on centred coordinates
 *    scaled by a power of two that puts eps in [1, 2); they run when eps is
 *    in [2^-500, 2^500] and every dimension's extent (max - min) is at most
 *    2^40 eps (FP8: 100 eps), otherwise FP64 MFMA runs;
 *  - FP64 MFMA: runs when the largest squared norm of the rows centred on
 *    the bounding-box midpoint is at most 2^1000, otherwise FP64 VALU runs
 *    (the exact chain itself, which has no range limit). */
typedef enum {
    SJ_FP64_VALU = 0,
    SJ_FP64_MFMA = 1,
    SJ_FP32_MFMA = 2,
    SJ_BF16_MFMA = 3,
    SJ_BF16X3_MFMA = 4,
    SJ_FP8_MFMA = 5
} sj_path;

/* Build options; pass NULL for defaults. */
typedef struct {
    int32_t index_dims;     /* number of leading dimensions indexed by the grid
                               (Section II-D: fewer than d); 0 = min(d, 4);
                               -1 = no index (selfjoin_build_grid only): one
                               cell holds every point, so every ordered pair
                               is a candidate -- the brute-force mode of
                               Section IV (Fig. 3), C_ref = n^2. The result
                               does not depend on it. */
    int32_t tune;           /* batched form only: nonzero = choose index_dims per
                               d by timing the FP64 MFMA count on the largest
                               problem of that d (result-neutral) */
    const char *tune_cache; /* batched form only: text file of tuned choices,
                               read before and written after tuning; NULL =
                               in-process cache only */
    /* Device allocator for every buffer the library creates for this handle
     * (the grid index, counts, in-masks, per-call temporaries), e.g. a
     * framework's caching allocator. alloc returns `bytes` of device memory
     * usable in stream order on `stream` (NULL = failure, reported as
     * SJ_ERR_OOM); free releases a pointer alloc returned, in stream order.
     * Both are called from the calling thread of the library call, with
     * `alloc_ctx`. alloc NULL = the library's own caching allocator. The
     * hook must stay callable until the handle is freed. */
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *alloc_ctx;
    int32_t short_circuit;  /* the partial-distance short-circuit of the FP64
                               tile paths (Section III-B; a filter, the result
                               does not depend on it), for d > 4: 0 = the
                               library's schedule, -1 = off, k > 0 = every k
                               K-steps of 4 dimensions. FP64 MFMA: one check
                               after half the K-steps for d <= 16, every k
                               (default 4) K-steps beyond; FP64 VALU: every
                               4k (default 4) dimensions for d > 8 (the d <= 8
                               forms keep the query rows in registers and run
                               without checks) */
    int32_t dim_order;      /* order of the dimensions in the FP64 MFMA tiles
                               (a filter choice, the result does not depend
                               on it; the exact FP64 chain always runs in
                               input order), for d > 4: 0 = the indexed
                               dimensions first (a tile's candidates lie close
                               together on them), then the others by
                               decreasing variance (Section II-D), so the
                               partial distance at each check grows fastest;
                               1 = input order */
    int32_t symmetric;      /* half-stencil count on the FP64 paths (0 = off,
                               1 = on; the result does not depend on it): the
                               count pass of SJ_FP64_MFMA / SJ_FP64_VALU meets
                               each pair within eps once, from its smaller
                               index in the grid's order (a work item keeps
                               only the candidates from its first query on,
                               and a value counts only for a candidate after
                               its query), and adds it to both points' counts
                               (to the candidate by a device atomic per tile
                               column), with 1 for the point itself: about
                               half the distance tiles. For count-only use
                               (selfjoin_count, selfjoin_core_points): the
                               count then records no in-masks, so a following
                               selfjoin_pairs / selfjoin_knn evaluates its
                               tiles again (full stencil). The batched form
                               (selfjoin_batch_build) takes it for every
                               problem: no in-mask buffer, and
                               selfjoin_batch_pairs re-runs the tiles. The
                               low-precision paths ignore it. */
    int32_t reserved32;
    int64_t reserved[2];
} sj_opts;

/* Statistics of one call (all optional, pass NULL). */
typedef struct {
    int64_t cand_ref;    /* C_ref: ordered candidate pairs of the full 3^k
                            stencil of the reference grid (work unit);
                            -1 until selfjoin_grid_info has computed it */
    int64_t cand_eval;   /* candidate pairs the path evaluated, tile padding
                            excluded (a half-stencil count: the pairs after
                            each work item's first query) */
    int64_t pairs;       /* |R| for count; pairs written for pairs */
    int64_t rechecked;   /* pairs of this call's tile kernels whose fast value
                            fell inside the error band and were re-evaluated
                            with the exact FP64 chain (0 on the FP64 VALU
                            path, and for pairs expanded from the in-masks a
                            count recorded) */
    int64_t rechecked_in; /* of those, the pairs found within eps */
    double band_rel;     /* largest band half-width used, divided by eps^2 */
    double ms;           /* device time of the whole call (ms) */
    double ms_build;     /* device time of the grid build of this handle (ms) */
    double ms_refine;    /* device time of the count pass (distance tiles)
                            run by this call; 0 when the counts were cached */
    double ms_emit;      /* pairs: device time of the emission kernel (the
                            recorded in-masks expanded, or the tiles re-run
                            in emission form); 0 for count */
    int64_t tiles_pruned; /* 16 x 16 tiles left before their last K-step
                            because every value's partial distance already
                            exceeded the threshold (the short-circuit of
                            Section III-B, see sj_opts.short_circuit): FP64
                            MFMA against eps^2 + Delta (prefix norms at the
                            K-step boundaries), FP64 VALU against eps^2 (its
                            chain never decreases); 0 on the FP32 / BF16
                            paths */
    int32_t path_run;    /* the path whose kernels ran (an sj_path): the
                            requested one unless its range guard routed the
                            call to the next exact path (see sj_path) */
    int32_t reserved;
} sj_stats;

/* Grid facts (for tests and reports). */
typedef struct {
    int64_t n;
    int32_t d, k;        /* dims, indexed dims */
    int64_t cells;       /* non-empty cells */
    int64_t items;       /* query groups (work items) */
    double eps, eps2, cell_side;
    int64_t cand_ref;    /* C_ref, as in sj_stats */
    int64_t cand_items;  /* candidates seen by the work items (>= C_ref) */
} sj_grid_info;

/* Builds the grid index (Sections II-D, III-B) over `points`.
 *  points : device, n x d row-major FP64, read during the call's stream work;
 *           the library copies what it needs (sorted), so the caller may
 *           release `points` once the stream has passed this call.
 *  n      : 0 <= n <= 2,000,000,000 (n = 0 gives an empty index; the bound
 *           keeps work-item and row indices below 2^31).
 *  d      : 1 <= d <= 256.
 *  eps    : finite, > 0.
 *  opts   : host, nullable.
 *  out    : host; receives the handle (owned by the caller, release with
 *           selfjoin_free_grid).
 * Errors: SJ_ERR_INVALID for bad arguments or any non-finite coordinate
 * (detected on the device), SJ_ERR_OOM, SJ_ERR_HIP. */
sj_status selfjoin_build_grid(const double *points, int64_t n, int32_t d, double eps,
                              const sj_opts *opts, void *stream, sj_grid **out);

/* Counts R (Section IV-A selectivity needs |R|).
 *  per_point : device int32[n] in the input order, or NULL; entry i receives
 *              |{j : (i, j) in R}| (>= 1: the self-pair).
 *  total     : host, receives |R|.
 *  stats     : host, nullable.
 * The count is cached on the handle and reused by selfjoin_pairs. */
sj_status selfjoin_count(sj_grid *g, sj_path path, int32_t *per_point, int64_t *total,
                         sj_stats *stats, void *stream);

/* Core points of density-based clustering (DBSCAN, named in Section I as a
 * consumer of these distance calculations): point i is core when its
 * eps-neighbourhood, itself included, holds at least min_pts points, i.e.
 * the per-point count of selfjoin_count is >= min_pts.
 *  min_pts : >= 1.
 *  is_core : device uint8[n] in the input order (1 = core, 0 = not), or NULL
 *            when n = 0.
 *  ncore   : host, receives the number of core points.
 * Uses the handle's cached counts (any path gives the same exact counts) or
 * runs the count with `path` first. Errors: SJ_ERR_INVALID for bad
 * arguments, SJ_ERR_OOM, SJ_ERR_HIP. */
sj_status selfjoin_core_points(sj_grid *g, sj_path path, int32_t min_pts, uint8_t *is_core, int64_t *ncore,
                               void *stream);

/* k nearest neighbours within eps (kNN, named in Section I as a consumer of
 * these distance calculations), from the pairs of R: for point i, the points
 * j != i with d2(i, j) <= eps^2 ordered by the exact squared distance of
 * Eq. (2) and then by the smaller index j; the first k of them.
 *  k           : in [1, 64].
 *  pair_budget : most pairs (with their distances) held in device memory at
 *                once, 16 bytes each, allocated and freed by the call; 0 =
 *                2^26. Fewer than the total runs several chunks.
 *  nbr         : device int32[n * k], row i (input order) = the indices of
 *                i's neighbours, -1 past nfound[i].
 *  nbr_d2      : device double[n * k] or NULL: their squared distances, +inf
 *                past nfound[i].
 *  nfound      : device int32[n]: min(k, neighbours of i within eps).
 * nbr / nfound may be NULL when n = 0. Uses the handle's cached counts or
 * counts with `path` first. Errors: SJ_ERR_INVALID for bad arguments,
 * SJ_ERR_UNSUPPORTED when one point has more pairs than pair_budget,
 * SJ_ERR_OOM, SJ_ERR_HIP. */
sj_status selfjoin_knn(sj_grid *g, sj_path path, int32_t k, int64_t pair_budget, int32_t *nbr, double *nbr_d2,
                       int32_t *nfound, void *stream);

/* Writes pairs of R, one chunk per call (result batching, Section III-B:
 * the result may exceed device memory).
 *  cursor      : first query to emit, in the grid's query order (0 = start;
 *                pass back *next_cursor to continue).
 *  pairs       : device int32[capacity][2], rows (i, j) in input indices.
 *  d2          : device double[capacity] or NULL; receives d2(i, j) of each
 *                written pair, computed with the exact chain above.
 *  capacity    : rows available in pairs (and d2).
 *  written     : host, pairs written.
 *  next_cursor : host, the cursor to pass next; n when done.
 * Every chunk holds all pairs of whole queries, in query order and, per
 * query, in candidate order; the order is deterministic. If the next query's
 * pairs do not fit, returns SJ_ERR_CAPACITY and sets *written to the capacity
 * that query needs (nothing else is written). */
sj_status selfjoin_pairs(sj_grid *g, sj_path path, int64_t cursor, int32_t *pairs, double *d2,
                         int64_t capacity, int64_t *written, int64_t *next_cursor,
                         sj_stats *stats, void *stream);

/* Debug measurement of a path's fast values against the exact chain: runs the
 * path over every evaluated candidate pair whose exact d2 is within the
 * range its band bound covers (d2 <= 4 eps^2 for FP64 MFMA, whose bound is
 * global; d2 <= eps^2 for FP32/BF16, whose bound is per query and covers the
 * candidates that can be within eps) and reports the largest
 * |fast - exact| (max_abs_err), the largest band half-width used (max_band),
 * and how many pairs had an error larger than their band (violations; must
 * be 0). Slow; not for timing. */
sj_status selfjoin_measure_error(sj_grid *g, sj_path path, double *max_abs_err, double *max_band,
                                 int64_t *violations, void *stream);

/* Grid facts of a built handle. The first call computes C_ref (one pass over
 * the cells on `stream`) and caches it on the handle. */
sj_status selfjoin_grid_info(sj_grid *g, sj_grid_info *info, void *stream);

/* Releases the handle; its device memory is freed in stream order on
 * `stream`. NULL is accepted. */
void selfjoin_free_grid(sj_grid *g, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): build + count in one call, with every
 * temporary taken from a static device scratch array of 256 MiB that the
 * library holds on each GPU it runs on until the process ends. Nothing is
 * allocated (no hipMalloc / hipFree, no allocator hook, no events).
 *  points, n, d, eps : as selfjoin_build_grid (device, n x d row-major FP64).
 *  path      : as selfjoin_count; the same exact set and counts.
 *  per_point : device int32[n] in the input order, or NULL (as
 *              selfjoin_count).
 *  total     : host, receives |R|.
 * The call returns after its stream work has finished, so the scratch is
 * free again on return. Calls on one GPU share its array: the library runs
 * them one at a time (a per-device lock), and work that overlaps with a call
 * on the same GPU from outside the library must not touch that array (it
 * cannot: its address is private to the library).
 * Limit: inputs whose worst-case need exceeds the array return
 * SJ_ERR_CAPACITY before any device work (about n <= 1.29M at d = 2, 647k
 * at d = 4, 175k at d = 64, 50k at d = 256; selfjoin_last_error states the
 * need).
 * Errors: SJ_ERR_INVALID (bad argument or non-finite coordinate),
 * SJ_ERR_UNSUPPORTED (low-precision path with d > 64), SJ_ERR_CAPACITY,
 * SJ_ERR_HIP. No pair list: use the handle-based calls for pairs. */
sj_status selfjoin_count_noalloc(const double *points, int64_t n, int32_t d, double eps, sj_path path,
                                 int32_t *per_point, int64_t *total, void *stream);

/* ---- Batched form: B independent self-joins of uneven n and d ----------
 * selfjoin_batch_build builds every problem's grid in one segmented pass
 * (one set of launches for all problems: one radix sort whose keys carry the
 * problem index above each problem's cell key; two host synchronisations),
 * falling back to one build per problem when the problem index does not fit
 * above the widest cell key. The work items of all problems sit in one queue, grouped by d (one tile
 * form each) and ordered by descending cost within a group. The count
 * pipeline (counter reset, one tile kernel per form, per-problem prefix sums)
 * and the pairs launch are each captured into a HIP graph on first use and
 * replayed. The count pass records every problem's in-masks (up to 64 GiB;
 * beyond, the pairs launch re-runs the tiles), so the pairs launch is one
 * kernel that expands them. With opts->tune, the tuner picks per d the
 * index_dims and the short-circuit setting (timing the FP64 MFMA count on the
 * largest problem of that d; cached in tune_cache), and on the first count
 * the schedule of the tile kernels: persistent grids of the resident waves
 * dealing the items round-robin, or one wave per item. Every choice is
 * result-neutral. FP64 paths only (SJ_FP64_MFMA, SJ_FP64_VALU); other paths
 * return SJ_ERR_UNSUPPORTED. */
typedef struct sj_batch sj_batch;

/* points : host array of B device pointers, problem i is n[i] x d[i]
 *          row-major FP64 (validated like selfjoin_build_grid).
 * n, d, eps : host arrays of B entries. opts: index_dims / short_circuit /
 *          dim_order (every problem) or tune / tune_cache; symmetric (the
 *          half-stencil count for every problem, with no in-mask buffer);
 *          the allocator hook is not used by the batched form.
 * out    : host; receives the handle (release with selfjoin_batch_free). */
sj_status selfjoin_batch_build(int32_t B, const double *const *points, const int64_t *n,
                               const int32_t *d, const double *eps, const sj_opts *opts,
                               void *stream, sj_batch **out);

/* totals : host int64[B], |R| of each problem. stats (nullable): ms =
 * ms_refine = device time of the count graph; ms_build = wall time of
 * selfjoin_batch_build (grid builds, queue, in-mask buffer); cand_eval,
 * rechecked, tiles_pruned over all problems (cand_eval of a half-stencil
 * batch: counted by one extra pass over the ranges on the first call that
 * asks for stats); cand_ref = -1. */
sj_status selfjoin_batch_count(sj_batch *b, sj_path path, int64_t *totals, sj_stats *stats,
                               void *stream);

/* Writes every problem's pairs into one device buffer, problem i's rows
 * (input indices of problem i) at [offsets[i], offsets[i + 1]), each in the
 * order selfjoin_pairs would give. offsets: host int64[B + 1]. If the sum
 * exceeds capacity, returns SJ_ERR_CAPACITY with offsets[B] = the sum. */
sj_status selfjoin_batch_pairs(sj_batch *b, sj_path path, int32_t *pairs, int64_t capacity,
                               int64_t *offsets, sj_stats *stats, void *stream);

/* Indexed dimensions and work items of problem i. */
sj_status selfjoin_batch_info(const sj_batch *b, int32_t i, int32_t *index_dims, int64_t *items);

void selfjoin_batch_free(sj_batch *b, void *stream);

/* ---- Achievable peaks (measurement utility, not on the join path) -------
 * Short microbenchmarks of this GPU, the measured denominators beside the
 * published peaks when the distance kernels are placed on their roofline
 * (the roofline of the work unit C_ref: 2 d flops per distance on the matrix
 * or vector unit, or the bytes the pairs pass must move):
 *  fp64_mfma_tflops : v_mfma_f64_16x16x4f64 (the FP64 MFMA tiles)
 *  fp32_mfma_tflops : v_mfma_f32_16x16x4f32 (the FP32 tiles)
 *  bf16_mfma_tflops : v_mfma_f32_16x16x32_bf16 (BF16 and split-BF16 tiles)
 *  fp8_mfma_tflops  : v_mfma_f32_16x16x32_fp8_fp8 (FP8 tiles)
 *  fp64_valu_tflops : v_fma_f64 (the FP64 vector path), 2 flops per FMA
 *  hbm_read_gbs     : streaming read of `bytes`
 *  hbm_copy_gbs     : streaming copy of `bytes` (read and written bytes)
 * Matrix forms: 1024 blocks of 4 waves, every wave running four independent
 * accumulator chains, so the unit never waits on a result; FMA: 16 waves
 * per SIMD, eight chains each; HBM: 16-byte non-temporal loads / stores.
 * Each figure is the best of three timed launches after one warmup.
 * bytes : size of each of the two bandwidth buffers (>= 16; 0 skips the
 *         bandwidth probes and leaves their fields 0). Take it well above
 *         the 256 MB last-level cache (1 GiB is typical); the two buffers
 *         are allocated from the runtime (not through the allocator hook)
 *         and freed before return.
 * Returns after the stream work has finished. Errors: SJ_ERR_INVALID
 * (out NULL, bytes < 0), SJ_ERR_OOM, SJ_ERR_HIP. */
typedef struct {
    double fp64_mfma_tflops, fp32_mfma_tflops, bf16_mfma_tflops, fp8_mfma_tflops;
    double fp64_valu_tflops;
    double hbm_read_gbs, hbm_copy_gbs;
} sj_peaks;

sj_status selfjoin_probe_peaks(int64_t bytes, sj_peaks *out, void *stream);

/* Static text for a status. */
const char *selfjoin_status_string(sj_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char *selfjoin_last_error(void);

/* Library version string. */
const char *selfjoin_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SELFJOIN_H */

// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/selfjoin.h"

namespace sj {

constexpr int kMaxIndexDims = 4;   // default k = min(d, kMaxIndexDims)
constexpr int kMaxDims = 256;
// Largest n of one grid: the work items (up to n + n / 16 + 1) and the rows
// with their padding stay below 2^31 (int32 indices on the device).
constexpr int64_t kMaxPoints = 2000000000;
constexpr int kTileQ = 16;         // queries per work item (one wave)
constexpr int kRowPad = 64;        // extra zeroed rows after every point array
constexpr int kBlockItems = 4;     // work items per block item (low-precision paths)
constexpr int kLpMaxD = 64;        // largest d of the low-precision paths
constexpr int64_t kMaskBudget = int64_t(16) << 30;  // largest in-mask buffer (bytes)
constexpr int64_t kLeanLineTable = int64_t(1) << 20;  // largest dense line table of a lean build

// Thread-local error text.
void set_error(const std::string &msg);
const char *last_error();

struct HipError {
    hipError_t code;
    std::string where;
};

// Throws HipError on failure; caught at the ABI boundary.
#define SJ_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) throw ::sj::HipError{e_, std::string(#call)};       \
    } while (0)

struct OomError {
    size_t bytes;
};

struct Unsupported {
    std::string what;
};

// Device allocation. Every device buffer of the library comes from
// dev_alloc / dev_free, which serve it from one of three sources, chosen per
// thread by the innermost live AllocScope:
//  - none (the default): the library's caching allocator (blocks kept per
//    device and stream and reused; hipMalloc only on a miss);
//  - a caller's hook (sj_opts.alloc / free / alloc_ctx): every allocation
//    and release goes to the hook, with the stream;
//  - an arena (a fixed device buffer): bump allocation, release is a no-op,
//    exhaustion throws ArenaFull; nothing is allocated from the runtime.
struct AllocHook {
    void *(*alloc)(size_t bytes, void *stream, void *ctx) = nullptr;
    void (*free)(void *p, void *stream, void *ctx) = nullptr;
    void *ctx = nullptr;
};

struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0, peak = 0;
};

struct ArenaFull {
    size_t need, size;
};

class AllocScope {
public:
    explicit AllocScope(const AllocHook &h);  // h.alloc null: the caching allocator
    explicit AllocScope(Arena *a);
    ~AllocScope();
    AllocScope(const AllocScope &) = delete;
    AllocScope &operator=(const AllocScope &) = delete;
    const AllocHook *hook = nullptr;
    Arena *arena = nullptr;
    AllocScope *prev = nullptr;
};

void *dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);

template <typename T>
T *dev_alloc_n(size_t n, hipStream_t s) {
    return static_cast<T *>(dev_alloc(n * sizeof(T) + 16, s));
}

// Device counters of one refine launch (zeroed before it). Non-negative
// doubles are kept as their bit patterns, whose integer order is theirs.
struct DevCounters {
    unsigned long long rechecked;     // band pairs re-evaluated with the exact chain
    unsigned long long rechecked_in;  // of those, within eps
    unsigned long long pruned;        // tiles left early by the partial-distance bound
    unsigned long long max_delta;     // largest band half-width used (bits)
    unsigned long long max_err;       // measure: largest |fast - exact| (bits)
    unsigned long long violations;    // measure: errors above their band
    unsigned long long spare[2];
};

// Candidate range of a work item: the union of the neighbouring cells of its
// first and last cell along one offset of the leading indexed dimensions.
struct Range {
    int32_t begin, end;
};

// A work item: up to kTileQ consecutive queries of one grid line (cells that
// differ only in the last indexed coordinate), and the cells they lie in.
struct Item {
    int32_t qbegin, qend;
    int32_t cell_first, cell_last;
};

// Device-side view of a grid (kernel argument).
struct DevGrid {
    const double *xs;
    const double *xa;
    const double *nrm;
    const double *pn;  // prefix norms of xa rows at the K-step boundaries: npc per row, else null
    const int32_t *perm;
    const Range *ranges;
    const Item *items;
    int64_t n;
    int32_t d, dp, da, nranges;
    int32_t nitems;
    const int32_t *blocks;  // first item of each block item (+ end), plus item_base, or null
    int32_t item_base;      // offset of the item indices in blocks (segmented builds: the problem's first item)
    int32_t nblocks;
    int32_t united;         // the items of each block item share one candidate list
    int32_t npc;   // prefix norms per row: da / 4 - 1 for d > 4, else 0
    int32_t sc;    // short-circuit (sj_opts.short_circuit): 0 = default schedule, -1 = off, k > 0 = every k K-steps
    double eps2;
    const int64_t *tile_off;
};

// One problem of a batch, as the batch kernels see it.
struct BProb {
    DevGrid G;
    double delta;      // FP64 MFMA band half-width
    int32_t *cnt;      // per-query counts (sorted order), n + 1
    int64_t *off;      // exclusive prefix of cnt, n + 1
    int64_t pout;      // first output row of this problem
    unsigned long long *masks;  // this problem's in-masks (recorded by the count pass), or null
};

// The items of the problems of one dimensionality d (one tile form): queue
// positions [lo, hi), longest first. sched: 0 = a persistent grid of the
// resident waves dealing them round-robin, 1 = one wave per item.
struct BatchForm {
    int32_t d;
    int32_t lo, hi;
    int32_t sched;
    int32_t blo, bhi;  // FP64 MFMA count, d = 5 .. 16: its block items' positions in the block queue
};

struct Grid {
    int64_t n = 0;
    int32_t d = 0, k = 0;
    int32_t dp = 0;        // row stride of xs (multiple of 4, >= d)
    int32_t da = 0;        // row stride of xa (multiple of 4; slot d holds the norm when d % 4 != 0)
    int32_t nranges = 1;   // 3^(k-1) ranges per cell
    double eps = 0, eps2 = 0, w = 0;
    double lo[kMaxDims];   // per-dimension minimum (grid origin on indexed dims)
    double hi[kMaxDims];
    double mid[kMaxDims];  // centring reference of xa
    int64_t m[kMaxIndexDims];
    int64_t stride[kMaxIndexDims];
    int32_t key_bits = 0;  // bits of the cell key
    int32_t sub_bits = 0;  // bits appended to the sort key: position inside the cell along the last
                           // indexed dimension, so a line's points are in coordinate order there
    int64_t cells = 0;
    int64_t items = 0;
    int64_t nblocks = 0;
    int64_t cand_ref = -1;   // C_ref (lazily computed; -1 = not yet)
    int64_t cand_items = 0;  // candidate pairs the work items evaluate
    double nmax = 0;       // max squared norm of the centred rows of xa
    // Dimension order of the distance tiles (xa, the low-precision tiles):
    // column t holds input dimension fo[t]. For d > 4 (unless dim_order = 1)
    // the non-indexed dimensions come first, then the indexed ones, each by
    // decreasing variance; identity otherwise. The exact chain on xs is
    // always in input order.
    uint8_t fo[kMaxDims];
    int32_t dim_order = 0;  // sj_opts.dim_order
    int32_t sc = 0;         // sj_opts.short_circuit: 0 = default schedule, -1 = off, k > 0 = every k K-steps
    int32_t sym = 0;        // sj_opts.symmetric: half-stencil count on the FP64 paths
    int32_t npc = 0;        // prefix norms per row in pn
    bool united = false;    // d > 4: every item's ranges are its block item's union
    int32_t item_base = 0;  // blocks[] holds item indices plus this (segmented builds)

    // device buffers
    double *xs = nullptr;        // sorted original coordinates, n x dp (+pad rows)
    double *xa = nullptr;        // sorted centred coordinates (+norm slot), n x da (+pad rows)
    double *nrm = nullptr;       // squared norms of xa rows (FP64 chain), n (+pad)
    double *pn = nullptr;        // d > 4: squared norms of xa rows over their first 4s columns,
                                 // s = 1 .. npc (FP64 chain), n (+pad) x npc; else null
    int32_t *perm = nullptr;     // sorted position -> input index
    int64_t *cell_key = nullptr; // per non-empty cell
    int32_t *cell_start = nullptr; // cells + 1 entries
    Range *ranges = nullptr;     // items x nranges: candidate ranges of each work item
    Item *item = nullptr;        // items
    int32_t *line_first = nullptr;  // first cell of each grid line (+ end marker)
    int32_t *line_table = nullptr;  // dense line key -> line id (or null when too large)
    int32_t *blocks = nullptr;      // first item of each block item (+ end sentinel)
    int64_t *tile_off = nullptr;    // first in-mask tile slot of each item, whole groups of 16 (+ total)
    int64_t tiles = 0;              // in-mask tile slots over all items (32 bytes each)
    // per-tile in-masks written by the FP64 count passes (4 x 64 bits per tile:
    // word r, bit 16g + j = query g + 4r of the item, candidate j of the tile)
    unsigned long long *masks = nullptr;
    bool masks_valid = false;
    // in-masks written by the low-precision count passes (after their FP64
    // recheck, so exact): per block item, its 64-candidate tiles in groups
    // of 4; per group 4 waves x 64 lanes x 64 bits (bit 4 (4 t + s) + r of
    // lane (g, j) = query 4g + r of the wave's item, candidate 16 s + j of
    // tile t of the group); lp_goff = first group of each block item (+ total)
    int64_t *lp_goff = nullptr;
    int64_t lp_groups = -1;      // -1 until the layout is computed
    unsigned long long *lp_masks = nullptr;
    bool lp_masks_valid = false;
    double *dev_nmax = nullptr;  // device copy of nmax

    // cached per-query counts (sorted order) and their exclusive prefix sums
    int32_t *cnt = nullptr;
    int64_t *off = nullptr;      // n + 1 entries
    DevCounters *ctr = nullptr;  // counters of the count pass, read with the total
    bool have_counts = false;
    int64_t total = 0;
    sj_path count_path = SJ_FP64_VALU;  // the path whose kernels made the cached counts

    bool borrowed = false;       // xs, xa, nrm, pn, perm, item, ranges, tile_off belong to a segmented
                                 // build (released with the batch, not by free_grid)
    AllocHook hook;              // the handle's device allocator (alloc null: the caching allocator)
    bool lean = false;           // build and count without events or in-masks, dense line table
                                 // only up to kLeanLineTable entries (static-scratch calls)
    double ms_build = 0;         // device time of the build (0 when lean)
    hipStream_t build_stream = nullptr;
};

// Build steps (sj_build.hip).
void build_grid(Grid &g, const double *points, int64_t n, int d, double eps, int index_dims,
                hipStream_t s);
void free_grid(Grid &g, hipStream_t s);

// Segmented build of many problems (sj_build.hip): the grids of every
// problem in one pass of launches; their index arrays are slices of shared
// buffers appended to `owned` (released by the caller), their tile_off
// values count the tile slots of all problems together. Returns false (and
// builds nothing) when the problem index does not fit above the widest cell
// key; throws like build_grid.
struct SegInput {
    const double *points;
    int64_t n;
    int32_t d;
    double eps;
    int32_t index_dims, sc, dim_order;
};
bool build_grids_segmented(const std::vector<SegInput> &in, std::vector<Grid *> &out, std::vector<void *> &owned,
                           hipStream_t s);
// C_ref of the reference grid, computed on first request and cached.
int64_t grid_cref(Grid &g, hipStream_t s);

// Zero fill by kernel (usable under stream capture, unlike a memset node).
void fill_zero(void *p, size_t bytes, hipStream_t s);

// Scans and sort (sj_build.hip).
void exclusive_scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s);
void radix_sort_pairs(unsigned long long **key_a, int32_t **val_a, unsigned long long *key_b, int32_t *val_b,
                      int64_t n, int bits, hipStream_t s);

// Refine (sj_refine.hip).
// Events bracketing one kernel launch on a stream.
struct KernelTimer {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    void start(bool enable, hipStream_t s) {
        on = enable;
        if (!on) return;
        SJ_HIP(hipEventCreate(&a));
        SJ_HIP(hipEventCreate(&b));
        SJ_HIP(hipEventRecord(a, s));
    }
    void stop(hipStream_t s) {
        if (on) SJ_HIP(hipEventRecord(b, s));
    }
    float ms() {  // waits for the end event
        if (!on) return 0.f;
        float v = 0.f;
        SJ_HIP(hipEventSynchronize(b));
        SJ_HIP(hipEventElapsedTime(&v, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        on = false;
        return v;
    }
    ~KernelTimer() {
        if (on) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    }
};

struct RefineOut {
    bool timed = false;      // record events around the tile kernel
    KernelTimer kt;          // those events
    DevCounters *ctr = nullptr;            // device counters (zeroed by the launcher)
    unsigned long long *masks = nullptr;   // per-tile in-masks to record (FP64 count), nullable
    bool record_lp = false;  // low-precision count: record its in-masks (layout and buffer on the grid)
    double band_rel = 0;     // largest band half-width / eps^2
    int64_t cand_eval = 0;
    bool sym = false;        // FP64 count: half stencil (counts zeroed by the caller); the
                             // candidate pairs it evaluates land in ctr->spare[0]
};

// Host copy of a launch's counters (one device-to-host copy with the
// caller's other readbacks).
struct HostCounters {
    int64_t rechecked = 0, rechecked_in = 0, pruned = 0, violations = 0;
    double max_delta = 0, max_err = 0;
};
HostCounters read_counters(const DevCounters &c);


struct ChunkPlan {
    bool too_small = false;  // the next query alone needs more than the capacity
    int64_t written = 0;     // pairs of the chunk (or the capacity needed)
    int64_t next = 0;        // cursor after the chunk
    int64_t item_lo = 0, item_hi = 0;  // work items covering the chunk
    int64_t block_lo = 0, block_hi = 0;  // block items covering the chunk
    int64_t base = 0;        // prefix count at the cursor
};
void refine_count(Grid &g, sj_path path, int32_t *cnt_sorted, RefineOut &ro, hipStream_t s);
ChunkPlan plan_chunk(Grid &g, int64_t cursor, int64_t capacity, hipStream_t s);
void refine_pairs(Grid &g, sj_path path, const ChunkPlan &p, int64_t qlo, int32_t *pairs, double *d2,
                  RefineOut &ro, hipStream_t s);
void refine_measure(Grid &g, sj_path path, double *max_err, double *max_band, int64_t *viol,
                    hipStream_t s);

// Batched form (sj_refine.hip).
void batch_reset(DevCounters *ctr, hipStream_t s);
// sym: the count with the half stencil (FP64 paths; counts added into
// per-point arrays zeroed by launch_batch_zero_counts, no in-masks).
void launch_batch_form(bool emit, bool sym, const BatchForm &f, sj_path path, const BProb *probs,
                       const int64_t *item_base, int B, const int32_t *queue, int32_t *pairs, DevCounters *ctr,
                       hipStream_t s, const int64_t *block_base = nullptr, const int32_t *bqueue = nullptr);
void launch_batch_zero_counts(const BProb *probs, int B, int64_t max_n, hipStream_t s);
// Adds to *acc the candidate pairs a half-stencil count of g evaluates.
void launch_sym_cand(const Grid &g, unsigned long long *acc, hipStream_t s);
void launch_batch_emit(const BProb *probs, const int64_t *item_base, int B, const int32_t *queue, int total,
                       int sched, int32_t *pairs, hipStream_t s);
void launch_seg_scan(const BProb *probs, int B, int64_t *totals, hipStream_t s);
DevGrid make_dev_grid(const Grid &g);
double fp64_mfma_delta(const Grid &g);

// Range guards. FP64 MFMA: the Gram form over centred rows stays finite
// when the largest centred squared norm is at most 2^1000. FP32 / BF16 tiles
// (scaled by lowp_scale, a power of two putting eps in [1, 2)): eps in
// [2^-500, 2^500] and every dimension's extent at most 2^40 eps. A request
// for a path whose guard fails runs the next path that passes (low
// precision -> FP64 MFMA -> FP64 VALU, which is the exact chain itself).
bool m64_in_range(const Grid &g);
bool lowp_in_range(const Grid &g, sj_path path);
// The low-precision tile paths (FP32, BF16, split BF16, FP8: d <= 64).
inline bool is_lowp(sj_path p) {
    return p == SJ_FP32_MFMA || p == SJ_BF16_MFMA || p == SJ_BF16X3_MFMA || p == SJ_FP8_MFMA;
}
double lowp_scale(const Grid &g);
sj_path effective_path(const Grid &g, sj_path requested);

// Low-precision paths (sj_lowp.hip).
void lowp_count(Grid &g, sj_path path, int32_t *cnt_sorted, RefineOut &ro, hipStream_t s);
void lowp_pairs(Grid &g, sj_path path, const ChunkPlan &p, int64_t qlo, int32_t *pairs, double *d2,
                RefineOut &ro, hipStream_t s);
void lowp_measure(Grid &g, sj_path path, double *max_err, double *max_band, int64_t *viol, hipStream_t s);

}  // namespace sj

struct sj_grid {
    sj::Grid g;
};

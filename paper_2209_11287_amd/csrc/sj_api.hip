// The C ABI (include/selfjoin.h): validation, error mapping, allocation,
// counts cache, chunked pair output.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "sj_internal.h"

namespace sj {

namespace {
thread_local std::string g_err;

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

// The count's total (the last entry of the offsets' exclusive scan) beside
// its counters, so that one copy brings both to the host.
__global__ void k_total_to_ctr(const int64_t *total, DevCounters *ctr) { ctr->spare[1] = (unsigned long long)*total; }

// Core flags in the input order and their number (one counter atomic per
// block).
__global__ void k_core_flags(const int32_t *__restrict__ cnt, const int32_t *__restrict__ perm, int64_t n,
                             int32_t min_pts, uint8_t *__restrict__ is_core, unsigned long long *__restrict__ ncore) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool core = false;
    if (i < n) {
        core = cnt[i] >= min_pts;
        is_core[perm[i]] = core ? 1 : 0;
    }
    __shared__ unsigned part[256 / 64];
    const unsigned c = (unsigned)__popcll(__ballot(core));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0;
        for (int w = 0; w < 256 / 64; ++w) t += part[w];
        if (t) atomicAdd(ncore, (unsigned long long)t);
    }
}

constexpr int32_t kKnnMax = 64;                  // largest k of selfjoin_knn
constexpr int64_t kKnnBudget = int64_t(1) << 26;  // default pairs held at once (1 GiB with d2)

// k nearest within eps for sorted queries [qlo, qhi) of one pair chunk, one
// wave per query: k rounds, each taking the smallest (d2, index) key above
// the previous round's over the query's pairs (the point itself skipped).
// Rows are written in the input order; unused slots get -1 / +inf.
__global__ void k_knn_select(const int2 *__restrict__ pairs, const double *__restrict__ d2,
                             const int64_t *__restrict__ off, int64_t base, const int32_t *__restrict__ perm,
                             int64_t qlo, int64_t qhi, int32_t k, int32_t *__restrict__ nbr,
                             double *__restrict__ nbr_d2, int32_t *__restrict__ nfound) {
    const int lane = threadIdx.x & 63;
    const int64_t q = qlo + (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (q >= qhi) return;  // whole wave
    const int64_t b = off[q] - base, e = off[q + 1] - base;
    const int32_t self = perm[q];
    int64_t row = (int64_t)self * k;
    double pd = -1.0;  // previous key (d2 >= 0)
    int32_t pj = -1;
    int found = 0;
    for (; found < k; ++found) {
        double bd = INFINITY;
        int32_t bj = INT_MAX;
        for (int64_t p = b + lane; p < e; p += 64) {
            const int32_t j = pairs[p].y;
            if (j == self) continue;
            const double x = d2[p];
            const bool above = x > pd || (x == pd && j > pj);
            if (above && (x < bd || (x == bd && j < bj))) {
                bd = x;
                bj = j;
            }
        }
        for (int sh = 32; sh > 0; sh >>= 1) {
            const double od = __shfl_xor(bd, sh);
            const int32_t oj = __shfl_xor(bj, sh);
            if (od < bd || (od == bd && oj < bj)) {
                bd = od;
                bj = oj;
            }
        }
        if (bj == INT_MAX) break;  // wave-uniform after the reduction
        if (lane == 0) {
            nbr[row + found] = bj;
            if (nbr_d2) nbr_d2[row + found] = bd;
        }
        pd = bd;
        pj = bj;
    }
    for (int r = found + lane; r < k; r += 64) {
        nbr[row + r] = -1;
        if (nbr_d2) nbr_d2[row + r] = INFINITY;
    }
    if (lane == 0) nfound[self] = found;
}

__global__ void k_scatter_counts(const int32_t *__restrict__ cnt, const int32_t *__restrict__ perm, int64_t n,
                                 int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[perm[i]] = cnt[i];
}

}  // namespace

// ------------------------------------------------------------------------
// Device memory: a caching allocator. hipMalloc is slow and synchronising,
// and a build makes a few dozen temporary allocations, so freed blocks are
// kept per device (tagged with the stream they were released on) and reused
// on that stream only (work on several streams never waits on each other
// here). The cache is returned to the runtime when an allocation fails.
// ------------------------------------------------------------------------
namespace {

struct FreeBlock {
    void *p;
    size_t size;
    hipStream_t s;
};

struct DevCache {
    std::multimap<size_t, FreeBlock> free;   // by size
    std::unordered_map<void *, size_t> live; // allocation sizes
};

std::mutex g_mu;
std::unordered_map<int, DevCache> g_cache;

size_t round_size(size_t b) {
    if (b <= 4096) return 4096;
    if (b <= (size_t(1) << 20)) return (b + 4095) & ~size_t(4095);
    // 1/8-octave classes above 1 MiB: at most 12.5% slack
    int e = 63 - __builtin_clzll(b);
    size_t step = size_t(1) << (e - 3);
    return (b + step - 1) / step * step;
}

void release_cache(DevCache &c) {
    (void)hipDeviceSynchronize();
    for (auto &kv : c.free) (void)hipFree(kv.second.p);
    c.free.clear();
}

}  // namespace

thread_local AllocScope *tl_scope = nullptr;

AllocScope::AllocScope(const AllocHook &h) : hook(h.alloc ? &h : nullptr), prev(tl_scope) { tl_scope = this; }
AllocScope::AllocScope(Arena *a) : arena(a), prev(tl_scope) { tl_scope = this; }
AllocScope::~AllocScope() { tl_scope = prev; }

static void *cache_alloc(size_t bytes, hipStream_t s);
static void cache_free(void *p, hipStream_t s);

void *dev_alloc(size_t bytes, hipStream_t s) {
    AllocScope *sc = tl_scope;
    if (sc && sc->arena) {
        Arena &a = *sc->arena;
        const size_t off = (a.used + 255) & ~size_t(255);
        if (off > a.size || bytes > a.size - off) throw ArenaFull{off + bytes, a.size};
        a.used = off + bytes;
        a.peak = std::max(a.peak, a.used);
        return a.base + off;
    }
    if (sc && sc->hook) {
        void *p = sc->hook->alloc(bytes, static_cast<void *>(s), sc->hook->ctx);
        if (!p) throw OomError{bytes};
        return p;
    }
    return cache_alloc(bytes, s);
}

void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    AllocScope *sc = tl_scope;
    if (sc && sc->arena) return;  // released with the arena
    if (sc && sc->hook) {
        if (sc->hook->free) sc->hook->free(p, static_cast<void *>(s), sc->hook->ctx);
        return;
    }
    cache_free(p, s);
}

static void *cache_alloc(size_t bytes, hipStream_t s) {
    int dev = 0;
    SJ_HIP(hipGetDevice(&dev));
    const size_t sz = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &c = g_cache[dev];
    // smallest cached block of this stream that fits without wasting more than 2x
    auto it = c.free.lower_bound(sz);
    for (auto j = it; j != c.free.end() && j->first <= 2 * sz; ++j) {
        if (j->second.s == s) {
            const FreeBlock fb = j->second;
            c.free.erase(j);
            c.live[fb.p] = fb.size;
            return fb.p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e == hipErrorOutOfMemory) {
        // blocks cached for other streams: drain the device and return them
        (void)hipGetLastError();
        release_cache(c);
        e = hipMalloc(&p, sz);
    }
    if (e == hipErrorOutOfMemory || (e == hipSuccess && !p)) {
        (void)hipGetLastError();
        throw OomError{bytes};
    }
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    c.live[p] = sz;
    return p;
}

static void cache_free(void *p, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &c = g_cache[dev];
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free.insert({it->second, FreeBlock{p, it->second, s}});
    c.live.erase(it);
}

void set_error(const std::string &msg) { g_err = msg; }
const char *last_error() { return g_err.c_str(); }

// A device buffer released (in stream order) when it goes out of scope.
template <typename T>
struct DevBuf {
    T *p = nullptr;
    hipStream_t s = nullptr;
    DevBuf(size_t n, hipStream_t st) : p(dev_alloc_n<T>(n, st)), s(st) {}
    ~DevBuf() {
        if (p) dev_free(p, s);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

// Device time between two events recorded on one stream.
struct CallTimer {
    hipEvent_t a = nullptr, b = nullptr;
    explicit CallTimer(bool on, hipStream_t s) {
        if (!on) return;
        SJ_HIP(hipEventCreate(&a));
        SJ_HIP(hipEventCreate(&b));
        SJ_HIP(hipEventRecord(a, s));
    }
    float stop(hipStream_t s) {
        if (!a) return 0.f;
        SJ_HIP(hipEventRecord(b, s));
        SJ_HIP(hipEventSynchronize(b));
        float ms = 0;
        SJ_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~CallTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Counts of one count pass, as the calls report them.
struct CountRun {
    bool ran = false;  // false: the counts were cached
    HostCounters hc;
    double band_rel = 0;
    float ms_refine = 0;
    int64_t cand_eval = -1;  // half-stencil count: the candidate pairs it evaluated
};

// Computes per-query counts with `path` (range-checked) into the handle's
// cache (sorted order), their exclusive prefix sums and the total.
static void compute_counts(Grid &g, sj_path path, bool timed, CountRun &cr, hipStream_t s) {
    if (!g.cnt) {
        g.cnt = dev_alloc_n<int32_t>((size_t)g.n + 1, s);
        g.off = dev_alloc_n<int64_t>((size_t)g.n + 1, s);
        g.ctr = dev_alloc_n<DevCounters>(1, s);
    }
    RefineOut ro;
    ro.timed = timed;
    ro.ctr = g.ctr;
    // FP64 count passes record per-tile in-masks; emission then reuses them
    const bool fp64 = path == SJ_FP64_VALU || path == SJ_FP64_MFMA;
    // half stencil (FP64 paths): counts accumulate from zero, no in-masks
    const bool sym = fp64 && g.sym != 0;
    g.masks_valid = false;
    g.lp_masks_valid = false;
    ro.record_lp = is_lowp(path) && !g.lean;
    if (fp64 && !sym && !g.lean && !g.masks && g.tiles > 0 && g.tiles * 32 <= kMaskBudget)
        g.masks = dev_alloc_n<unsigned long long>((size_t)g.tiles * 4, s);
    ro.masks = fp64 && !sym ? g.masks : nullptr;
    ro.sym = sym;
    if (sym && g.n > 0) fill_zero(g.cnt, (size_t)g.n * sizeof(int32_t), s);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, g.cnt + g.n, 0);
    SJ_HIP(hipGetLastError());
    if (g.n > 0) refine_count(g, path, g.cnt, ro, s);
    else fill_zero(g.ctr, sizeof(DevCounters), s);
    exclusive_scan_i32_to_i64(g.cnt, g.off, g.n + 1, s);
    // the total and the counters: one copy, one sync
    hipLaunchKernelGGL(k_total_to_ctr, dim3(1), dim3(1), 0, s, g.off + g.n, g.ctr);
    SJ_HIP(hipGetLastError());
    DevCounters hctr{};
    SJ_HIP(hipMemcpyAsync(&hctr, g.ctr, sizeof hctr, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const int64_t total = (int64_t)hctr.spare[1];
    g.total = total;
    g.masks_valid = ro.masks != nullptr;
    g.lp_masks_valid = ro.record_lp && g.lp_masks != nullptr;
    g.count_path = path;
    cr.ran = true;
    cr.hc = read_counters(hctr);
    cr.band_rel = ro.band_rel;
    if (is_lowp(path)) {
        const double sc = lowp_scale(g);  // the band is in the tiles' scaled units
        cr.band_rel = g.eps2 > 0 ? cr.hc.max_delta / (g.eps2 * sc * sc) : 0.0;
    }
    cr.ms_refine = ro.kt.ms();
    cr.cand_eval = sym ? (int64_t)hctr.spare[0] : -1;
    g.have_counts = true;
}

// The path that runs a request: unsupported d for the low-precision tiles is
// an error; otherwise the range guards pick the first exact path that fits.
static sj_path path_for(const Grid &g, sj_path path) {
    if (is_lowp(path) && g.d > kLpMaxD)
        throw Unsupported{"FP32/BF16 MFMA paths support d <= 64"};
    return effective_path(g, path);
}

static void fill_stats(sj_stats *st, const Grid &g, int64_t pairs, const CountRun &cr, sj_path run, float ms,
                       float ms_emit, const HostCounters *emit_ctr, double emit_band_rel) {
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    st->cand_ref = g.cand_ref;  // -1 until selfjoin_grid_info computed it
    st->cand_eval = cr.ran && cr.cand_eval >= 0 ? cr.cand_eval : g.cand_items;
    st->pairs = pairs;
    st->rechecked = (cr.ran ? cr.hc.rechecked : 0) + (emit_ctr ? emit_ctr->rechecked : 0);
    st->rechecked_in = (cr.ran ? cr.hc.rechecked_in : 0) + (emit_ctr ? emit_ctr->rechecked_in : 0);
    st->band_rel = std::max(cr.ran ? cr.band_rel : 0.0, emit_band_rel);
    st->ms = ms;
    st->ms_build = g.ms_build;
    st->ms_refine = cr.ran ? cr.ms_refine : 0.0;
    st->ms_emit = ms_emit;
    st->tiles_pruned = cr.ran ? cr.hc.pruned : 0;
    st->path_run = (int32_t)run;
}

// The whole result in one chunk (no device search needed).
static ChunkPlan whole_plan(const Grid &g) {
    ChunkPlan p;
    p.written = g.total;
    p.next = g.n;
    p.item_lo = 0;
    p.item_hi = g.items;
    p.block_lo = 0;
    p.block_hi = g.nblocks;
    p.base = 0;
    return p;
}

// ------------------------------------------------------------------------
// Static scratch for selfjoin_count_noalloc: every temporary of a lean build
// and count is bump-allocated from one file-scope device array (each GPU the
// library runs on holds its own copy until the process ends). Host code never
// passes the array's name to a kernel: its device address, taken per device
// with hipGetSymbolAddress on the first call there, is the arena's base.
// ------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(256) << 20;

}  // namespace sj

static __device__ __align__(256) unsigned char scratch[sj::kScratchBytes];

namespace sj {
namespace {

struct ScratchDev {
    void *ptr = nullptr;
    std::mutex mu;  // one call at a time per device (the array is shared)
};
std::mutex g_scratch_mu;
std::unordered_map<int, ScratchDev> g_scratch;

// The current device's scratch entry, its address looked up once.
ScratchDev &scratch_for_current_device() {
    int dev = 0;
    SJ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchDev &e = g_scratch[dev];
    if (!e.ptr) {
        void *p = nullptr;
        SJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
        e.ptr = p;
    }
    return e;
}

// Upper bound of the scratch bytes a lean build + count of n points in d
// dimensions takes: the sum of every allocation the two make (the arena
// releases nothing), each with its 16-byte tail and 256-byte alignment.
// Table sizes use the build's own upper bounds (items <= n + n/16 + 1,
// 3^(k-1) ranges per item with k <= min(d, 4)); each exclusive scan of L
// entries is charged L/256 + 4096 bytes of tile sums.
size_t lean_need(int64_t n, int32_t d) {
    const size_t N = (size_t)n;
    const size_t dp = (size_t)((d + 3) & ~3);
    const size_t da = (d & 3) ? (size_t)((d + 1 + 3) & ~3) : (size_t)d;
    const size_t rows = N + kRowPad;
    const size_t items_ub = N + N / kTileQ + 1;
    size_t nr = 1;
    for (int j = 0; j < std::min(d, kMaxIndexDims) - 1; ++j) nr *= 3;
    auto A = [](size_t b) { return (b + 16 + 255) & ~size_t(255); };
    auto scan = [](size_t L) { return L / 256 + 4096; };
    const size_t sort_tiles = (N + 4095) / 4096 + 1;
    size_t need = 0;
    need += A(4 * 2048 * (size_t)d * 8) + A((4 * (size_t)d + 1) * 8);              // bounding box, moments
    need += 2 * A(8 * N) + 2 * A(4 * N);                                             // keys, indices
    need += A((8 * 256 + 9) * 4) + A(8 * sort_tiles * 256 * 8);                     // radix sort
    const size_t npc = d > 4 ? da / 4 - 1 : 0;
    need += A(rows * dp * 8) + A(rows * da * 8) + A(rows * 8) + A(rows * npc * 8) + 3 * A(16);  // rows, norms
    need += A(std::max<size_t>(4096, N / 256 + 1) * 8);                              // norm maxima
    need += 2 * A((N + N / kTileQ + 2) * 4);                                         // flags, ids
    need += A(8 * (N + 1)) + 4 * A(4 * (N + 2)) + 3 * scan(N + 1);                   // cells, lines
    need += A(8 * (items_ub + 1)) + 2 * A(4 * (items_ub + 1)) + A(16 * items_ub);    // items
    need += A(8 * items_ub * nr) * (d > 4 ? 2 : 1) + A(4 * (size_t)kLeanLineTable) + 2 * scan(items_ub + 1);
    need += A(4 * (N + 1)) + A(8 * (N + 1)) + A(sizeof(DevCounters)) + scan(N + 1);  // counts
    return need;
}

}  // namespace

}  // namespace sj

using namespace sj;

#define SJ_API_BEGIN try {
#define SJ_API_END                                                                         \
    }                                                                                      \
    catch (const HipError &e) {                                                            \
        set_error(e.where + ": " + hipGetErrorString(e.code));                             \
        return SJ_ERR_HIP;                                                                 \
    }                                                                                      \
    catch (const OomError &e) {                                                            \
        set_error("device allocation of " + std::to_string(e.bytes) + " bytes failed");    \
        return SJ_ERR_OOM;                                                                 \
    }                                                                                      \
    catch (const ArenaFull &e) {                                                           \
        set_error("the work needs " + std::to_string(e.need) + " bytes of the " +          \
                  std::to_string(e.size) + "-byte static scratch");                        \
        return SJ_ERR_CAPACITY;                                                            \
    }                                                                                      \
    catch (const std::bad_alloc &) {                                                       \
        set_error("host allocation failed");                                               \
        return SJ_ERR_OOM;                                                                 \
    }                                                                                      \
    catch (const Unsupported &u) {                                                         \
        set_error(u.what);                                                                 \
        return SJ_ERR_UNSUPPORTED;                                                         \
    }                                                                                      \
    catch (const std::string &msg) {                                                       \
        set_error(msg);                                                                    \
        return SJ_ERR_INVALID;                                                             \
    }                                                                                      \
    catch (...) {                                                                          \
        set_error("unexpected exception");                                                 \
        return SJ_ERR_HIP;                                                                 \
    }

static sj_status invalid(const char *msg) {
    set_error(msg);
    return SJ_ERR_INVALID;
}

static bool valid_path(sj_path p) {
    return p == SJ_FP64_VALU || p == SJ_FP64_MFMA || is_lowp(p);
}

namespace sj {
// Achievable peaks of the GPU (microbenchmarks, sj_probe.hip).
void probe_peaks(int64_t bytes, sj_peaks &out, hipStream_t s);
}  // namespace sj

extern "C" {

sj_status selfjoin_build_grid(const double *points, int64_t n, int32_t d, double eps, const sj_opts *opts,
                              void *stream, sj_grid **out) {
    set_error("");
    if (!out) return invalid("out is NULL");
    if (n < 0 || n > kMaxPoints) return invalid("n must be in [0, 2,000,000,000]");
    if (d < 1 || d > kMaxDims) return invalid("d must be in [1, 256]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return invalid("eps must be finite and > 0");
    if (n > 0 && !points) return invalid("points is NULL");
    if (opts && (opts->index_dims < -1 || opts->index_dims > kMaxIndexDims))
        return invalid("index_dims must be in [-1, 4]");
    if (opts && !opts->alloc != !opts->free) return invalid("alloc and free must be given together");
    if (opts && (opts->short_circuit < -1 || opts->short_circuit > 64))
        return invalid("short_circuit must be in [-1, 64]");
    if (opts && (opts->dim_order < 0 || opts->dim_order > 1)) return invalid("dim_order must be 0 or 1");
    if (opts && (opts->symmetric < 0 || opts->symmetric > 1)) return invalid("symmetric must be 0 or 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    sj_grid *h = nullptr;
    SJ_API_BEGIN
    h = new sj_grid();
    if (opts) {
        h->g.sc = opts->short_circuit;
        h->g.dim_order = opts->dim_order;
        h->g.sym = opts->symmetric;
    }
    if (opts && opts->alloc) {
        h->g.hook.alloc = opts->alloc;
        h->g.hook.free = opts->free;
        h->g.hook.ctx = opts->alloc_ctx;
    }
    AllocScope scope(h->g.hook);
    try {
        build_grid(h->g, points, n, d, eps, opts ? opts->index_dims : 0, s);
    } catch (...) {
        free_grid(h->g, s);
        delete h;
        h = nullptr;
        throw;
    }
    *out = h;
    return SJ_OK;
    SJ_API_END
}

sj_status selfjoin_count(sj_grid *gh, sj_path path, int32_t *per_point, int64_t *total, sj_stats *stats,
                         void *stream) {
    set_error("");
    if (!gh) return invalid("grid is NULL");
    if (!valid_path(path)) return invalid("unknown path");
    if (!total) return invalid("total is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    Grid &g = gh->g;
    AllocScope scope(g.hook);
    const sj_path run = path_for(g, path);
    CallTimer tm(stats != nullptr, s);
    CountRun cr;
    compute_counts(g, run, stats != nullptr, cr, s);
    if (per_point && g.n > 0) {
        hipLaunchKernelGGL(k_scatter_counts, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g.cnt, g.perm,
                           g.n, per_point);
        SJ_HIP(hipGetLastError());
    }
    *total = g.total;
    if (stats) fill_stats(stats, g, g.total, cr, run, tm.stop(s), 0.f, nullptr, 0.0);
    return SJ_OK;
    SJ_API_END
}

sj_status selfjoin_knn(sj_grid *gh, sj_path path, int32_t k, int64_t pair_budget, int32_t *nbr, double *nbr_d2,
                       int32_t *nfound, void *stream) {
    set_error("");
    if (!gh) return invalid("grid is NULL");
    if (!valid_path(path)) return invalid("unknown path");
    if (k < 1 || k > kKnnMax) return invalid("k must be in [1, 64]");
    if (pair_budget < 0) return invalid("pair_budget < 0");
    if (gh->g.n > 0 && (!nbr || !nfound)) return invalid("nbr / nfound is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    Grid &g = gh->g;
    if (g.n == 0) return SJ_OK;
    AllocScope scope(g.hook);
    const sj_path run = path_for(g, path);  // checked before anything is allocated
    CountRun cr;
    if (!g.have_counts) compute_counts(g, run, false, cr, s);
    const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(g.total, pair_budget ? pair_budget : kKnnBudget));
    DevBuf<int32_t> pairs(2 * (size_t)cap, s);
    DevBuf<double> pd2((size_t)cap, s);
    DevBuf<DevCounters> ctr(1, s);
    int64_t cursor = 0;
    while (cursor < g.n) {
        const ChunkPlan p = (cursor == 0 && cap >= g.total) ? whole_plan(g) : plan_chunk(g, cursor, cap, s);
        if (p.too_small) throw Unsupported{"a point has more pairs than pair_budget"};
        RefineOut re;
        re.ctr = ctr.p;
        refine_pairs(g, run, p, cursor, pairs.p, pd2.p, re, s);
        const int64_t nq = p.next - cursor;
        hipLaunchKernelGGL(k_knn_select, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s,
                           reinterpret_cast<const int2 *>(pairs.p), pd2.p, g.off, p.base, g.perm, cursor, p.next, k,
                           nbr, nbr_d2, nfound);
        SJ_HIP(hipGetLastError());
        cursor = p.next;
    }
    return SJ_OK;
    SJ_API_END
}

sj_status selfjoin_core_points(sj_grid *gh, sj_path path, int32_t min_pts, uint8_t *is_core, int64_t *ncore,
                               void *stream) {
    set_error("");
    if (!gh) return invalid("grid is NULL");
    if (!valid_path(path)) return invalid("unknown path");
    if (min_pts < 1) return invalid("min_pts must be >= 1");
    if (!ncore) return invalid("ncore is NULL");
    if (gh->g.n > 0 && !is_core) return invalid("is_core is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    Grid &g = gh->g;
    AllocScope scope(g.hook);
    const sj_path run = path_for(g, path);
    CountRun cr;
    if (!g.have_counts) compute_counts(g, run, false, cr, s);
    unsigned long long hc = 0;
    if (g.n > 0) {
        DevBuf<unsigned long long> dc(1, s);
        fill_zero(dc.p, sizeof(unsigned long long), s);
        hipLaunchKernelGGL(k_core_flags, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g.cnt, g.perm, g.n,
                           min_pts, is_core, dc.p);
        SJ_HIP(hipGetLastError());
        SJ_HIP(hipMemcpyAsync(&hc, dc.p, sizeof hc, hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
    }
    *ncore = (int64_t)hc;
    return SJ_OK;
    SJ_API_END
}

sj_status selfjoin_pairs(sj_grid *gh, sj_path path, int64_t cursor, int32_t *pairs, double *d2, int64_t capacity,
                         int64_t *written, int64_t *next_cursor, sj_stats *stats, void *stream) {
    set_error("");
    if (!gh) return invalid("grid is NULL");
    if (!valid_path(path)) return invalid("unknown path");
    if (!written || !next_cursor) return invalid("written / next_cursor is NULL");
    if (cursor < 0 || cursor > gh->g.n) return invalid("cursor out of range");
    if (capacity < 0) return invalid("capacity < 0");
    if (capacity > 0 && !pairs) return invalid("pairs is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    Grid &g = gh->g;
    AllocScope scope(g.hook);
    const sj_path run = path_for(g, path);
    if (cursor == g.n) {
        *written = 0;
        *next_cursor = g.n;
        if (stats) fill_stats(stats, g, 0, CountRun{}, run, 0.f, 0.f, nullptr, 0.0);
        return SJ_OK;
    }
    CallTimer tm(stats != nullptr, s);
    CountRun cr;
    if (!g.have_counts) compute_counts(g, run, stats != nullptr, cr, s);
    const ChunkPlan p = (cursor == 0 && capacity >= g.total) ? whole_plan(g) : plan_chunk(g, cursor, capacity, s);
    if (p.too_small) {
        *written = p.written;
        set_error("capacity too small for the next query's pairs");
        return SJ_ERR_CAPACITY;
    }
    DevBuf<DevCounters> ctr(1, s);
    RefineOut re;
    re.timed = stats != nullptr;
    re.ctr = ctr.p;
    refine_pairs(g, run, p, cursor, pairs, d2, re, s);
    *written = p.written;
    *next_cursor = p.next;
    if (stats) {
        DevCounters h{};
        SJ_HIP(hipMemcpyAsync(&h, ctr.p, sizeof h, hipMemcpyDeviceToHost, s));
        const float ms = tm.stop(s);  // synchronises the stream
        const HostCounters he = read_counters(h);
        double brel = re.band_rel;
        if (is_lowp(run)) {
            const double sc = lowp_scale(g);
            brel = g.eps2 > 0 ? he.max_delta / (g.eps2 * sc * sc) : 0.0;
        }
        fill_stats(stats, g, p.written, cr, run, ms, re.kt.ms(), &he, brel);
    }
    return SJ_OK;
    SJ_API_END
}

sj_status selfjoin_measure_error(sj_grid *gh, sj_path path, double *max_abs_err, double *max_band,
                                 int64_t *violations, void *stream) {
    set_error("");
    if (!gh) return invalid("grid is NULL");
    if (!valid_path(path)) return invalid("unknown path");
    if (!max_abs_err || !max_band || !violations) return invalid("NULL output");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    AllocScope scope(gh->g.hook);
    refine_measure(gh->g, path_for(gh->g, path), max_abs_err, max_band, violations, s);
    return SJ_OK;
    SJ_API_END
}

sj_status selfjoin_grid_info(sj_grid *gh, sj_grid_info *info, void *stream) {
    set_error("");
    if (!gh || !info) return invalid("NULL argument");
    SJ_API_BEGIN
    Grid &g = gh->g;
    AllocScope scope(g.hook);
    grid_cref(g, static_cast<hipStream_t>(stream));
    info->n = g.n;
    info->d = g.d;
    info->k = g.k;
    info->cells = g.cells;
    info->items = g.items;
    info->eps = g.eps;
    info->eps2 = g.eps2;
    info->cell_side = g.w;
    info->cand_ref = g.cand_ref;
    info->cand_items = g.cand_items;
    return SJ_OK;
    SJ_API_END
}

void selfjoin_free_grid(sj_grid *gh, void *stream) {
    if (!gh) return;
    try {
        AllocScope scope(gh->g.hook);
        free_grid(gh->g, static_cast<hipStream_t>(stream));
    } catch (...) {
    }
    delete gh;
}

sj_status selfjoin_count_noalloc(const double *points, int64_t n, int32_t d, double eps, sj_path path,
                                 int32_t *per_point, int64_t *total, void *stream) {
    set_error("");
    if (n < 0 || n > kMaxPoints) return invalid("n must be in [0, 2,000,000,000]");
    if (d < 1 || d > kMaxDims) return invalid("d must be in [1, 256]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return invalid("eps must be finite and > 0");
    if (n > 0 && !points) return invalid("points is NULL");
    if (!valid_path(path)) return invalid("unknown path");
    if (!total) return invalid("total is NULL");
    if (is_lowp(path) && d > kLpMaxD) {
        set_error("FP32/BF16 MFMA paths support d <= 64");
        return SJ_ERR_UNSUPPORTED;
    }
    const size_t need = lean_need(n, d);
    if (need > kScratchBytes) {
        set_error("n = " + std::to_string(n) + ", d = " + std::to_string(d) + " needs up to " +
                  std::to_string(need) + " bytes of scratch; the static scratch holds " +
                  std::to_string(kScratchBytes));
        return SJ_ERR_CAPACITY;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    ScratchDev &sd = scratch_for_current_device();
    std::lock_guard<std::mutex> lk(sd.mu);
    Arena arena;
    arena.base = static_cast<char *>(sd.ptr);
    arena.size = kScratchBytes;
    AllocScope scope(&arena);
    Grid g;
    g.lean = true;
    build_grid(g, points, n, d, eps, 0, s);
    const sj_path run = path_for(g, path);
    CountRun cr;
    compute_counts(g, run, false, cr, s);
    if (per_point && g.n > 0) {
        hipLaunchKernelGGL(k_scatter_counts, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, g.cnt, g.perm,
                           g.n, per_point);
        SJ_HIP(hipGetLastError());
    }
    // the next call may reuse the scratch as soon as this one returns
    SJ_HIP(hipStreamSynchronize(s));
    *total = g.total;
    return SJ_OK;
    SJ_API_END
}

const char *selfjoin_status_string(sj_status s) {
    switch (s) {
        case SJ_OK: return "ok";
        case SJ_ERR_INVALID: return "invalid argument";
        case SJ_ERR_OOM: return "out of memory";
        case SJ_ERR_HIP: return "HIP runtime error";
        case SJ_ERR_CAPACITY: return "output capacity too small";
        case SJ_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *selfjoin_last_error(void) { return last_error(); }

sj_status selfjoin_probe_peaks(int64_t bytes, sj_peaks *out, void *stream) {
    set_error("");
    if (!out) return invalid("out is NULL");
    if (bytes < 0 || (bytes > 0 && bytes < 16)) return invalid("bytes must be 0 or >= 16");
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJ_API_BEGIN
    sj_peaks r{};
    probe_peaks(bytes, r, s);
    *out = r;
    return SJ_OK;
    SJ_API_END
}

const char *selfjoin_version(void) { return "selfjoin-mi355x 0.2 (gfx950)"; }

}  // extern "C"

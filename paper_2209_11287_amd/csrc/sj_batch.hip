// Batched form: many independent self-joins (uneven n and d) refined by one
// persistent work-queue kernel whose items are ordered longest first, with
// the count pipeline (queue reset, persistent count kernel, per-problem
// prefix sums) captured once into a HIP graph and replayed; an optional
// autotuner picks the number of indexed dimensions per d by timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sj_internal.h"

namespace sj {

namespace {

// Cost of each work item, as a descending sort key: candidates x queries x
// K-steps; value = global item index.
__global__ void k_item_cost(const Item *__restrict__ items, const Range *__restrict__ ranges, int nitems,
                            int nranges, int ksteps, int64_t base, unsigned long long *__restrict__ key,
                            int32_t *__restrict__ val) {
    const int it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= nitems) return;
    const Item I = items[it];
    unsigned long long c = 0;
    for (int o = 0; o < nranges; ++o) {
        const Range r = ranges[(int64_t)it * nranges + o];
        c += (unsigned long long)((r.end - r.begin + 15) / 16);
    }
    c *= (unsigned long long)(ksteps > 0 ? ksteps : 1);
    const unsigned long long cap = 0xffffffffull;
    key[base + it] = cap - (c < cap ? c : cap);
    val[base + it] = (int32_t)(base + it);
}

struct TuneCache {
    std::mutex mu;
    std::map<std::string, int> k;  // "path/d/log2n" -> index_dims
};
TuneCache g_tune;

std::string tune_key(int path, int d, int64_t n) {
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= std::max<int64_t>(1, n)) ++lg;
    return std::to_string(path) + "/" + std::to_string(d) + "/" + std::to_string(lg);
}

void tune_load(const char *path) {
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[128];
    int v;
    // one "key value" pair per line
    while (std::fscanf(f, "%127s %d", key, &v) == 2) g_tune.k[key] = v;
    std::fclose(f);
}

void tune_save(const char *path) {
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune.k) std::fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
    std::fclose(f);
}

// Times the FP64 MFMA count kernel on one problem for k = 1..min(d, 4) and
// returns the fastest k (result-neutral).
int tune_index_dims(const double *pts, int64_t n, int d, double eps, hipStream_t s) {
    int best_k = std::min(d, kMaxIndexDims);
    float best = 1e30f;
    for (int k = 1; k <= std::min(d, kMaxIndexDims); ++k) {
        Grid g;
        try {
            build_grid(g, pts, n, d, eps, k, s);
            int32_t *cnt = dev_alloc_n<int32_t>((size_t)n + 1, s);
            RefineOut ro;
            ro.timed = true;
            ro.ctr = dev_alloc_n<DevCounters>(1, s);
            refine_count(g, SJ_FP64_MFMA, cnt, ro, s);  // warm
            ro.kt.ms();
            refine_count(g, SJ_FP64_MFMA, cnt, ro, s);
            const float ms = ro.kt.ms();
            dev_free(cnt, s);
            dev_free(ro.ctr, s);
            if (ms < best) {
                best = ms;
                best_k = k;
            }
        } catch (...) {
            free_grid(g, s);
            throw;
        }
        free_grid(g, s);
    }
    return best_k;
}

}  // namespace

struct Batch {
    int B = 0;
    std::vector<Grid *> grids;
    std::vector<int> kdims;
    int64_t total_items = 0;
    std::vector<int64_t> item_base;       // B + 1
    int64_t *item_base_dev = nullptr;     // B + 1
    int32_t *queue = nullptr;             // global item indices, longest first
    int *counter = nullptr;
    DevCounters *ctr = nullptr;
    BProb *probs_dev = nullptr;
    std::vector<BProb> probs;
    int64_t *totals_dev = nullptr;
    std::vector<int64_t> totals;
    bool counted = false;
    // count pipeline graphs, per path
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipStream_t graph_stream[2] = {nullptr, nullptr};
};

void batch_free(Batch &b, hipStream_t s) {
    for (int i = 0; i < 2; ++i)
        if (b.exec[i]) (void)hipGraphExecDestroy(b.exec[i]);
    for (Grid *g : b.grids) {
        if (!g) continue;
        if (g->cnt) {
            dev_free(g->cnt, s);
            g->cnt = nullptr;
        }
        if (g->off) {
            dev_free(g->off, s);
            g->off = nullptr;
        }
        free_grid(*g, s);
        delete g;
    }
    b.grids.clear();
    void *bufs[] = {b.item_base_dev, b.queue, b.counter, b.ctr, b.probs_dev, b.totals_dev};
    for (void *p : bufs)
        if (p) dev_free(p, s);
}

void batch_build(Batch &b, int B, const double *const *points, const int64_t *n, const int32_t *d, const double *eps,
                 const sj_opts *opts, hipStream_t s) {
    b.B = B;
    b.grids.assign(B, nullptr);
    b.kdims.assign(B, 0);
    const bool tune = opts && opts->tune;
    if (tune) {
        std::lock_guard<std::mutex> lk(g_tune.mu);
        tune_load(opts->tune_cache);
        // one representative (largest n) per d
        std::map<int, int> rep;
        for (int i = 0; i < B; ++i)
            if (n[i] > 0 && (!rep.count(d[i]) || n[i] > n[rep[d[i]]])) rep[d[i]] = i;
        for (auto &kv : rep) {
            const int i = kv.second;
            const std::string key = tune_key(SJ_FP64_MFMA, d[i], n[i]);
            if (!g_tune.k.count(key)) g_tune.k[key] = tune_index_dims(points[i], n[i], d[i], eps[i], s);
        }
        tune_save(opts->tune_cache);
        for (int i = 0; i < B; ++i) {
            auto it = g_tune.k.find(tune_key(SJ_FP64_MFMA, d[i], n[rep.count(d[i]) ? rep[d[i]] : i]));
            b.kdims[i] = it != g_tune.k.end() ? it->second : 0;
        }
    } else if (opts) {
        for (int i = 0; i < B; ++i) b.kdims[i] = opts->index_dims;
    }
    b.item_base.assign(B + 1, 0);
    for (int i = 0; i < B; ++i) {
        b.grids[i] = new Grid();
        build_grid(*b.grids[i], points[i], n[i], d[i], eps[i], b.kdims[i], s);
        Grid &g = *b.grids[i];
        g.cnt = dev_alloc_n<int32_t>((size_t)g.n + 1, s);
        g.off = dev_alloc_n<int64_t>((size_t)g.n + 1, s);
        b.item_base[i + 1] = b.item_base[i] + g.items;
    }
    b.total_items = b.item_base[B];
    if (b.total_items >= (int64_t(1) << 31)) throw std::string("too many work items in one batch");
    b.item_base_dev = dev_alloc_n<int64_t>(B + 1, s);
    SJ_HIP(hipMemcpyAsync(b.item_base_dev, b.item_base.data(), (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    // longest-first queue
    const int64_t T = std::max<int64_t>(1, b.total_items);
    unsigned long long *ka = dev_alloc_n<unsigned long long>(T, s), *kb = dev_alloc_n<unsigned long long>(T, s);
    int32_t *va = dev_alloc_n<int32_t>(T, s), *vb = dev_alloc_n<int32_t>(T, s);
    for (int i = 0; i < B; ++i) {
        const Grid &g = *b.grids[i];
        if (g.items == 0) continue;
        hipLaunchKernelGGL(k_item_cost, dim3((unsigned)((g.items + 255) / 256)), dim3(256), 0, s, g.item, g.ranges,
                           (int)g.items, g.nranges, g.da >> 2, b.item_base[i], ka, va);
        SJ_HIP(hipGetLastError());
    }
    unsigned long long *k_sorted = ka;
    int32_t *v_sorted = va;
    radix_sort_pairs(&k_sorted, &v_sorted, k_sorted == ka ? kb : ka, v_sorted == va ? vb : va, b.total_items, 32, s);
    b.queue = v_sorted;
    dev_free(v_sorted == va ? vb : va, s);
    dev_free(ka, s);
    dev_free(kb, s);
    b.counter = dev_alloc_n<int>(1, s);
    b.ctr = dev_alloc_n<DevCounters>(1, s);
    b.totals_dev = dev_alloc_n<int64_t>(B, s);
    b.probs.resize(B);
    for (int i = 0; i < B; ++i) {
        const Grid &g = *b.grids[i];
        BProb &p = b.probs[i];
        p.G = make_dev_grid(g);
        p.delta = fp64_mfma_delta(g);
        p.ks = g.da >> 2;
        p.slot = (g.d & 3) ? 1 : 0;
        p.cnt = g.cnt;
        p.off = g.off;
        p.pout = 0;
    }
    b.probs_dev = dev_alloc_n<BProb>(B, s);
    SJ_HIP(hipMemcpyAsync(b.probs_dev, b.probs.data(), B * sizeof(BProb), hipMemcpyHostToDevice, s));
    SJ_HIP(hipStreamSynchronize(s));
    b.totals.assign(B, 0);
}

// Count pipeline: captured into a graph on first use per (path, stream), then
// replayed. The graph holds only kernel nodes (no memset or copy nodes).
float batch_count(Batch &b, sj_path path, hipStream_t s, HostCounters *hc) {
    const int pi = path == SJ_FP64_MFMA ? 1 : 0;
    hipEvent_t e0, e1;
    SJ_HIP(hipEventCreate(&e0));
    SJ_HIP(hipEventCreate(&e1));
    if (!b.exec[pi] || b.graph_stream[pi] != s) {
        if (b.exec[pi]) (void)hipGraphExecDestroy(b.exec[pi]);
        b.exec[pi] = nullptr;
        hipStream_t cs = s;
        bool own = false;
        if (!cs) {  // the legacy null stream cannot be captured: capture on a private stream
            SJ_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            own = true;
        }
        hipGraph_t graph;
        SJ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        launch_batch(false, path, b.probs_dev, b.item_base_dev, b.B, b.queue, (int)b.total_items, b.counter, nullptr,
                     b.ctr, cs);
        launch_seg_scan(b.probs_dev, b.B, b.totals_dev, cs);
        SJ_HIP(hipStreamEndCapture(cs, &graph));
        SJ_HIP(hipGraphInstantiate(&b.exec[pi], graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        if (own) SJ_HIP(hipStreamDestroy(cs));
        b.graph_stream[pi] = s;
    }
    SJ_HIP(hipEventRecord(e0, s));
    SJ_HIP(hipGraphLaunch(b.exec[pi], s));
    SJ_HIP(hipEventRecord(e1, s));
    DevCounters hb{};
    SJ_HIP(hipMemcpyAsync(b.totals.data(), b.totals_dev, b.B * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(&hb, b.ctr, sizeof hb, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    float ms = 0;
    SJ_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *hc = read_counters(hb);
    for (int i = 0; i < b.B; ++i) {
        b.grids[i]->total = b.totals[i];
        b.grids[i]->have_counts = true;
    }
    b.counted = true;
    return ms;
}

// Emission of every problem's pairs into one buffer: problem i's rows at
// [offsets[i], offsets[i + 1]).
float batch_pairs(Batch &b, sj_path path, int32_t *pairs, hipStream_t s) {
    int64_t off = 0;
    for (int i = 0; i < b.B; ++i) {
        b.probs[i].pout = off;
        off += b.totals[i];
    }
    SJ_HIP(hipMemcpyAsync(b.probs_dev, b.probs.data(), b.B * sizeof(BProb), hipMemcpyHostToDevice, s));
    hipEvent_t e0, e1;
    SJ_HIP(hipEventCreate(&e0));
    SJ_HIP(hipEventCreate(&e1));
    SJ_HIP(hipEventRecord(e0, s));
    launch_batch(true, path, b.probs_dev, b.item_base_dev, b.B, b.queue, (int)b.total_items, b.counter, pairs,
                 b.ctr, s);
    SJ_HIP(hipEventRecord(e1, s));
    SJ_HIP(hipEventSynchronize(e1));
    float ms = 0;
    SJ_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace sj

struct sj_batch {
    sj::Batch b;
};

using namespace sj;

#define SJB_TRY try {
#define SJB_CATCH                                                                      \
    }                                                                                  \
    catch (const HipError &e) {                                                        \
        set_error(e.where + ": " + hipGetErrorString(e.code));                         \
        return SJ_ERR_HIP;                                                             \
    }                                                                                  \
    catch (const OomError &e) {                                                        \
        set_error("device allocation of " + std::to_string(e.bytes) + " bytes failed"); \
        return SJ_ERR_OOM;                                                             \
    }                                                                                  \
    catch (const Unsupported &u) {                                                     \
        set_error(u.what);                                                             \
        return SJ_ERR_UNSUPPORTED;                                                     \
    }                                                                                  \
    catch (const std::string &msg) {                                                   \
        set_error(msg);                                                                \
        return SJ_ERR_INVALID;                                                         \
    }                                                                                  \
    catch (...) {                                                                      \
        set_error("unexpected exception");                                             \
        return SJ_ERR_HIP;                                                             \
    }

extern "C" {

sj_status selfjoin_batch_build(int32_t B, const double *const *points, const int64_t *n, const int32_t *d,
                               const double *eps, const sj_opts *opts, void *stream, sj_batch **out) {
    set_error("");
    if (!out || B < 0 || (B > 0 && (!points || !n || !d || !eps))) {
        set_error("invalid batch arguments");
        return SJ_ERR_INVALID;
    }
    for (int i = 0; i < B; ++i) {
        if (n[i] < 0 || n[i] >= (int64_t(1) << 31) || d[i] < 1 || d[i] > kMaxDims || !(eps[i] > 0.0) ||
            !std::isfinite(eps[i]) || (n[i] > 0 && !points[i])) {
            set_error("invalid arguments for batch problem " + std::to_string(i));
            return SJ_ERR_INVALID;
        }
    }
    if (opts && (opts->index_dims < 0 || opts->index_dims > kMaxIndexDims)) {
        set_error("index_dims must be in [0, 4]");
        return SJ_ERR_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    sj_batch *h = new sj_batch();
    SJB_TRY
    try {
        batch_build(h->b, B, points, n, d, eps, opts, s);
    } catch (...) {
        batch_free(h->b, s);
        delete h;
        throw;
    }
    *out = h;
    return SJ_OK;
    SJB_CATCH
}

sj_status selfjoin_batch_count(sj_batch *bh, sj_path path, int64_t *totals, sj_stats *stats, void *stream) {
    set_error("");
    if (!bh || !totals) {
        set_error("NULL argument");
        return SJ_ERR_INVALID;
    }
    if (path != SJ_FP64_MFMA && path != SJ_FP64_VALU) {
        set_error("the batched form runs the FP64 paths");
        return SJ_ERR_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJB_TRY
    Batch &b = bh->b;
    HostCounters hc;
    const float ms = batch_count(b, path, s, &hc);
    int64_t sum = 0, cev = 0;
    for (int i = 0; i < b.B; ++i) {
        totals[i] = b.totals[i];
        sum += b.totals[i];
        cev += b.grids[i]->cand_items;
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->cand_ref = -1;
        stats->cand_eval = cev;
        stats->pairs = sum;
        stats->rechecked = hc.rechecked;
        stats->rechecked_in = hc.rechecked_in;
        stats->ms = ms;
        stats->ms_refine = ms;
        stats->tiles_pruned = hc.pruned;
        stats->path_run = (int32_t)path;
    }
    return SJ_OK;
    SJB_CATCH
}

sj_status selfjoin_batch_pairs(sj_batch *bh, sj_path path, int32_t *pairs, int64_t capacity, int64_t *offsets,
                               sj_stats *stats, void *stream) {
    set_error("");
    if (!bh || !offsets) {
        set_error("NULL argument");
        return SJ_ERR_INVALID;
    }
    if (path != SJ_FP64_MFMA && path != SJ_FP64_VALU) {
        set_error("the batched form runs the FP64 paths");
        return SJ_ERR_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    SJB_TRY
    Batch &b = bh->b;
    if (!b.counted) {
        HostCounters hc;
        batch_count(b, path, s, &hc);
    }
    int64_t sum = 0;
    for (int i = 0; i < b.B; ++i) sum += b.totals[i];
    if (sum > capacity) {
        offsets[b.B] = sum;
        set_error("capacity too small for the batch's pairs");
        return SJ_ERR_CAPACITY;
    }
    if (sum > 0 && !pairs) {
        set_error("pairs is NULL");
        return SJ_ERR_INVALID;
    }
    const float ms = batch_pairs(b, path, pairs, s);
    int64_t off = 0;
    for (int i = 0; i < b.B; ++i) {
        offsets[i] = off;
        off += b.totals[i];
    }
    offsets[b.B] = off;
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->cand_ref = -1;
        stats->pairs = sum;
        stats->ms = ms;
        stats->ms_emit = ms;
        stats->path_run = (int32_t)path;
    }
    return SJ_OK;
    SJB_CATCH
}

sj_status selfjoin_batch_info(const sj_batch *bh, int32_t i, int32_t *index_dims, int64_t *items) {
    if (!bh || i < 0 || i >= bh->b.B) {
        set_error("invalid batch index");
        return SJ_ERR_INVALID;
    }
    if (index_dims) *index_dims = bh->b.grids[i]->k;
    if (items) *items = bh->b.grids[i]->items;
    return SJ_OK;
}

void selfjoin_batch_free(sj_batch *bh, void *stream) {
    if (!bh) return;
    try {
        batch_free(bh->b, static_cast<hipStream_t>(stream));
    } catch (...) {
    }
    delete bh;
}

}  // extern "C"

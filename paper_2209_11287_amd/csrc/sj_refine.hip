// Refine kernels: distance tiles between a work item's queries and the
// candidates of its neighbouring cells (Section II-D "refine"; Section III-B:
// queries of one cell share one candidate set, so a tile's queries come from
// one run of cells).
//
// One wave (64 lanes) owns one work item of up to 16 queries.
//
//  V64 -- FP64 vector ALU, direct form (Eq. (1) in the order of Eq. (2)):
//         lane = candidate, loop over the item's queries; bit-exact with the
//         oracle's chain by construction. The paper's CUDA-core baseline role.
//  M64 -- FP64 MFMA, expanded form (Eq. (3), Fig. 2): one
//         v_mfma_f64_16x16x4_f64 per K-step computes, for 16 candidates (rows)
//         x 16 queries (columns), D' = |c|^2 - 2 c.q. The candidate norm rides
//         in a spare K slot (or the accumulator init when d % 4 == 0); the
//         query norm moves to the threshold side: in iff D' <= eps^2 - |q|^2.
//         A proven error bound Delta splits each value into in / out / band;
//         band pairs are re-evaluated with the exact FP64 chain, so the
//         result is the exact set. Fig. 2 needs CUDA-core steps because FP64
//         WMMA cannot feed an accumulator back; here the norms fold into the
//         contraction and only the threshold test stays on the vector ALU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "sj_internal.h"

// v_writelane_b32: lane `lane` of `old` takes the wave-uniform `val`.
__device__ int amdgcn_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace sj {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

typedef double double4_t __attribute__((ext_vector_type(4)));


// Output side of a refine launch.
struct RefOut {
    int32_t *cnt;                 // count: per-query counts, sorted order
    const int64_t *off;           // emit: exclusive prefix of counts
    int64_t base;                 // emit: off[qlo]
    int32_t qlo, qhi;             // emit: queries [qlo, qhi) write pairs
    int32_t *pairs;               // emit: rows (i, j), input indices
    double *d2;                   // emit: exact d2 per pair (nullable)
    unsigned long long *band;     // band pairs re-evaluated
    unsigned long long *meas;     // measure: [0] max err bits, [1] violations
    int32_t item_lo;              // first item of this launch
    unsigned long long *masks;    // count: per-tile in-masks to record (nullable)
};

enum { MODE_COUNT = 0, MODE_EMIT = 1, MODE_MEASURE = 2 };

// Blocks go round-robin over the 8 XCDs; give each XCD a contiguous run of
// logical blocks so spatially adjacent work items share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The oracle's chain: ascending dimensions from +0.0, fl(a - b) then fma.
__device__ __forceinline__ double exact_d2(const double *__restrict__ a, const double *__restrict__ b, int d) {
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        const double delta = __dsub_rn(a[t], b[t]);
        acc = __fma_rn(delta, delta, acc);
    }
    return acc;
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const unsigned lane = threadIdx.x & 63u;
    return lane ? ((~0ull) >> (64u - lane)) : 0ull;
}

// ------------------------------------------------------------ shared parts --
// Candidate ranges of a work item: lane o (< nranges) holds range o's bounds.
struct ItemRanges {
    int rb, re;
    int nr;
    __device__ __forceinline__ int begin(int o) const { return __builtin_amdgcn_readlane(rb, o); }
    __device__ __forceinline__ int end(int o) const { return __builtin_amdgcn_readlane(re, o); }
    __device__ __forceinline__ int first_nonempty(int o) const {
        while (o < nr && begin(o) >= end(o)) ++o;
        return o;
    }
};

__device__ __forceinline__ ItemRanges load_ranges(const DevGrid &G, int it, int lane) {
    ItemRanges r;
    r.nr = G.nranges;
    r.rb = 0;
    r.re = 0;
    if (lane < G.nranges) {
        const Range x = G.ranges[(int64_t)it * G.nranges + lane];
        r.rb = x.begin;
        r.re = x.end;
    }
    // Wait for the bounds once, here. The tile loops read them with
    // v_readlane while tile loads are in flight; without this the compiler
    // cannot tell those reads from the newer loads and waits for the
    // prefetched tiles at every range step.
    __asm__ volatile("" : "+v"(r.rb), "+v"(r.re));
    return r;
}

// Walks the item's candidate tiles (all ranges, in order) `step` rows at a time.
struct TileCursor {
    int o, t, ce;
    __device__ __forceinline__ bool live(const ItemRanges &rg) const { return o < rg.nr; }
    __device__ __forceinline__ void first(const ItemRanges &rg) {
        o = rg.first_nonempty(0);
        t = o < rg.nr ? rg.begin(o) : 0;
        ce = o < rg.nr ? rg.end(o) : 0;
    }
    __device__ __forceinline__ void advance(const ItemRanges &rg, int step) {
        t += step;
        if (t >= ce) {
            o = rg.first_nonempty(o + 1);
            if (o < rg.nr) {
                t = rg.begin(o);
                ce = rg.end(o);
            }
        }
    }
};

// Wave-local LDS ordering (stores by some lanes, loads by others).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Emission. Pairs go to exact offsets (prefix sums of the count pass), so a
// query's pairs form one run in candidate order.
//
// V64 (lane = candidate, one query at a time): flagged pairs are compacted,
// wave-wide, into an LDS ring (candidate, rank within its query, query
// column); whenever 64 are queued, one full-width store writes them, instead
// of one store per query with a few lanes active.
constexpr int kRing = 512;  // > 63 queued + 256 from one tile

struct EmitRing {
    uint32_t *cand;  // sorted index of the candidate
    uint32_t *rel;   // rank of the pair within its query's run
    uint32_t *col;   // query column (0..15)
    int head, tail;  // wave-uniform counters (entries flushed / appended)
    // The batch taken from the ring by the previous flush: its candidates'
    // input indices were requested then and are stored one flush later, so
    // that gather's latency overlaps the work in between.
    int pend_n;        // wave-uniform, 0 = none
    int64_t pend_pos;  // output row of lane's pair
    int32_t pend_pq;   // input index of the query
    int32_t pend_pc;   // input index of the candidate (in flight)
    uint32_t pend_c;   // sorted index of the candidate (distances)
    uint32_t pend_j;   // query column (distances)
};

__device__ __forceinline__ void ring_init(EmitRing &rb, uint32_t *base) {
    rb.cand = base;
    rb.rel = base + kRing;
    rb.col = base + 2 * kRing;
    rb.head = rb.tail = 0;
    rb.pend_n = 0;
    rb.pend_pos = 0;
    rb.pend_pq = rb.pend_pc = 0;
    rb.pend_c = rb.pend_j = 0;
}

// Stores the pending batch.
__device__ __forceinline__ void ring_store_pending(EmitRing &rb, const DevGrid &G, const RefOut &R, int lane, int q0) {
    if (lane < rb.pend_n) {
        reinterpret_cast<int2 *>(R.pairs)[rb.pend_pos] = make_int2(rb.pend_pq, rb.pend_pc);
        if (R.d2)
            R.d2[rb.pend_pos] = exact_d2(G.xs + (int64_t)(q0 + (int)rb.pend_j) * G.dp,
                                         G.xs + (int64_t)rb.pend_c * G.dp, G.d);
    }
    rb.pend_n = 0;
}

// Takes `n` ring entries starting at head (n <= 64), lane l one entry:
// stores the previous batch and leaves this one pending.
__device__ __forceinline__ void ring_flush(EmitRing &rb, int n, const DevGrid &G, const RefOut &R, int lane,
                                           int64_t pbase_of_lane, int32_t pq_of_lane, int q0) {
    wave_lds_sync();
    const int e = (rb.head + lane) & (kRing - 1);
    const uint32_t c = rb.cand[e], rel = rb.rel[e], j = rb.col[e];
    // the query's output base and input index live in lane j (j < 16)
    const int64_t pb = __shfl(pbase_of_lane, (int)j);
    const int32_t pq = __shfl(pq_of_lane, (int)j);
    int32_t pc = 0;
    if (lane < n) pc = G.perm[c];
    rb.head += n;
    wave_lds_sync();
    ring_store_pending(rb, G, R, lane, q0);
    rb.pend_n = n;
    rb.pend_pos = pb + rel;
    rb.pend_pq = pq;
    rb.pend_pc = pc;
    rb.pend_c = c;
    rb.pend_j = j;
}

__device__ __forceinline__ void ring_drain(EmitRing &rb, bool all, const DevGrid &G, const RefOut &R, int lane,
                                           int64_t pbase_of_lane, int32_t pq_of_lane, int q0) {
    while (rb.tail - rb.head >= 64) ring_flush(rb, 64, G, R, lane, pbase_of_lane, pq_of_lane, q0);
    if (all) {
        if (rb.tail > rb.head) ring_flush(rb, rb.tail - rb.head, G, R, lane, pbase_of_lane, pq_of_lane, q0);
        ring_store_pending(rb, G, R, lane, q0);
    }
}

// Direct emission of one 16 x 16 tile from its mask words (canonical
// layout, already restricted to the queries this launch emits): lane (g, j)
// writes pair (query g + 4r, candidate t + j) for each r whose bit it holds,
// at the query's base + pairs so far + the pair's rank among the set bits
// of its 16-bit group. `pc` = input index of candidate t + j.
struct RowOut {
    int64_t qb[4];  // output row of the first pair of query g + 4r (this launch)
    int32_t pq[4];  // input index of query g + 4r
    int cur[4];     // pairs of query g + 4r written so far
    unsigned jlt;   // (1 << j) - 1
};

__device__ __forceinline__ void row_out_init(RowOut &ro, const bool emit_r[4], const DevGrid &G, const RefOut &R,
                                             int q0, int g, int j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = q0 + g + 4 * r;
        ro.qb[r] = emit_r[r] ? R.off[q] - R.base : 0;
        ro.pq[r] = emit_r[r] ? G.perm[q] : 0;
        ro.cur[r] = 0;
    }
    ro.jlt = (1u << j) - 1u;
}

__device__ __forceinline__ void tile_store(const unsigned long long w[4], int t, int32_t pc, RowOut &ro, int g,
                                           int j, const DevGrid &G, const RefOut &R, int q0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const unsigned long long m = w[r];
        if (!m) continue;
        const unsigned ch = (unsigned)(m >> (16 * g)) & 0xffffu;
        if (__builtin_amdgcn_inverse_ballot_w64(m)) {
            const int64_t pos = ro.qb[r] + (ro.cur[r] + __popc(ch & ro.jlt));
            reinterpret_cast<int2 *>(R.pairs)[pos] = make_int2(ro.pq[r], pc);
            if (R.d2)
                R.d2[pos] = exact_d2(G.xs + (int64_t)(q0 + g + 4 * r) * G.dp, G.xs + (int64_t)(t + j) * G.dp, G.d);
        }
        ro.cur[r] += __popc(ch);
    }
}

// --------------------------------------------------------------------- V64 --
// lane = candidate (64 per tile), loop over the item's queries. D > 0: the
// candidate row is held in registers; D = 0: runtime d, read per dimension.
template <int D, int MODE>
__device__ __forceinline__ void v64_item(const DevGrid &G, const RefOut &R, int it, uint32_t *ring_lds) {
    const int lane = threadIdx.x & 63;
    const int wv = uniform_i32(threadIdx.x >> 6);
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int d = D > 0 ? D : G.d;
    const int dp = G.dp;
    const double eps2 = G.eps2;
    const double *__restrict__ xs = G.xs;
    const ItemRanges rg = load_ranges(G, it, lane);

    // emit state of query `lane` (lanes < nq)
    int64_t my_pbase = -1;
    int32_t my_pq = 0;
    bool emit_q = false;
    if (MODE == MODE_EMIT && lane < nq && q0 + lane >= R.qlo && q0 + lane < R.qhi) {
        my_pbase = R.off[q0 + lane] - R.base;
        my_pq = G.perm[q0 + lane];
        emit_q = true;
    }
    const unsigned long long emit_mask = __ballot(emit_q);
    EmitRing rb;
    ring_init(rb, ring_lds + (MODE == MODE_EMIT ? wv * 3 * kRing : 0));
    int my_cur = 0;
    const unsigned long long lt = lanemask_lt();
    int cnt[kTileQ];
#pragma unroll
    for (int jq = 0; jq < kTileQ; ++jq) cnt[jq] = 0;

    // in-mask recording (count): 16-candidate tile numbering of the item
    const bool rec = MODE == MODE_COUNT && R.masks != nullptr;
    const int64_t tile_base = rec ? G.tile_off[it] : 0;
    int kb = 0;  // tiles of the ranges before the current one
    TileCursor tc;
    tc.first(rg);
    int cur_o = tc.o, cur_cb = tc.t;
    double xn[D > 0 ? D : 1];
    if (D > 0 && tc.live(rg)) {
        const double *xc = xs + (int64_t)(tc.t + lane) * dp;  // rows are padded past n
#pragma unroll
        for (int u = 0; u < (D > 0 ? D : 1); ++u) xn[u] = xc[u];
    }
    while (tc.live(rg)) {
        const int t = tc.t, ce = tc.ce;
        if (rec && tc.o != cur_o) {
            kb += (rg.end(cur_o) - rg.begin(cur_o) + 15) / 16;
            cur_o = tc.o;
            cur_cb = tc.t;
        }
        const int k16 = kb + (t - cur_cb) / 16;  // first 16-tile of this 64-candidate tile
        unsigned long long qm[kTileQ];
#pragma unroll
        for (int jq = 0; jq < kTileQ; ++jq) qm[jq] = 0ull;
        const int c = t + lane;
        const bool valid = c < ce;
        double x[D > 0 ? D : 1];
#pragma unroll
        for (int u = 0; u < (D > 0 ? D : 1); ++u) x[u] = xn[u];
        tc.advance(rg, 64);
        if (D > 0 && tc.live(rg)) {  // prefetch the next tile
            const double *xc2 = xs + (int64_t)(tc.t + lane) * dp;
#pragma unroll
            for (int u = 0; u < (D > 0 ? D : 1); ++u) xn[u] = xc2[u];
        }
        const double *__restrict__ xc = xs + (int64_t)c * dp;
#pragma unroll
        for (int jq = 0; jq < kTileQ; ++jq) {
            if (jq < nq) {
                const double *__restrict__ xq = xs + (int64_t)(q0 + jq) * dp;
                double acc = 0.0;
                if (D > 0) {
#pragma unroll
                    for (int u = 0; u < (D > 0 ? D : 1); ++u) {
                        const double delta = __dsub_rn(xq[u], x[u]);
                        acc = __fma_rn(delta, delta, acc);
                    }
                } else {
                    for (int u = 0; u < d; ++u) {
                        const double delta = __dsub_rn(xq[u], xc[u]);
                        acc = __fma_rn(delta, delta, acc);
                    }
                }
                const bool in = valid && acc <= eps2;
                if (MODE == MODE_COUNT) {
                    cnt[jq] += in ? 1 : 0;
                    if (rec) qm[jq] = __ballot(in);
                } else if (MODE == MODE_EMIT) {
                    const unsigned long long m = __ballot(in);
                    if ((emit_mask >> jq) & 1ull) {
                        const int nm = __popcll(m);
                        if (nm) {
                            const int cur_j = __builtin_amdgcn_readlane(my_cur, jq);
                            if (in) {
                                const int e = (rb.tail + __popcll(m & lt)) & (kRing - 1);
                                rb.cand[e] = (uint32_t)c;
                                rb.rel[e] = (uint32_t)(cur_j + __popcll(m & lt));
                                rb.col[e] = (uint32_t)jq;
                            }
                            rb.tail += nm;
                            if (lane == jq) my_cur += nm;
                            ring_drain(rb, false, G, R, lane, my_pbase, my_pq, q0);
                        }
                    }
                }
            }
        }
        if (rec) {
            // four 16-candidate tiles: word r of sub-tile s collects the
            // 16-bit slices of queries 4r .. 4r + 3 (query g + 4r at bits
            // 16g); lane 4s + r stores it (the 16 words are contiguous)
            const int nsub = (min(64, ce - t) + 15) / 16;
            unsigned long long wl = 0;
#pragma unroll
            for (int sub = 0; sub < 4; ++sub) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    unsigned long long w = 0;
#pragma unroll
                    for (int gg = 0; gg < 4; ++gg) w |= ((qm[gg + 4 * r] >> (16 * sub)) & 0xffffull) << (16 * gg);
                    if (lane == 4 * sub + r) wl = w;
                }
            }
            if (lane < 4 * nsub) R.masks[(tile_base + k16) * 4 + lane] = wl;
        }
    }
    if (MODE == MODE_EMIT) ring_drain(rb, true, G, R, lane, my_pbase, my_pq, q0);
    if (MODE == MODE_COUNT) {
#pragma unroll
        for (int jq = 0; jq < kTileQ; ++jq) {
            int v = cnt[jq];
            for (int sh = 32; sh > 0; sh >>= 1) v += __shfl_xor(v, sh);
            if (lane == 0 && jq < nq) R.cnt[q0 + jq] = v;
        }
    }
}

template <int D, int MODE>
__global__ __launch_bounds__(kThreads) void k_v64(DevGrid G, RefOut R) {
    __shared__ uint32_t ring_lds[MODE == MODE_EMIT ? kWaves * 3 * kRing : 1];
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    v64_item<D, MODE>(G, R, it, ring_lds);
}

// --------------------------------------------------------------------- M64 --
// One v_mfma_f64_16x16x4f64 per K-step: rows = the item's 16 queries (the A
// operand, loaded once per item), columns = 16 candidates (the B operand,
// one row load per lane per K-step). Result layout (probed on gfx950):
// register r of lane (g, j) = lane 16g + j holds row g + 4r, column j.
//  SLOT (d % 4 != 0): the candidate norm rides in K slot d (A holds 1 there),
//    D = |c|^2 - 2 q.c, and the query norm moves to a per-row threshold:
//    in iff D <= eps^2 - |q|^2.
//  no slot (d % 4 == 0): the accumulator starts at |q|^2 (constant per
//    item), D = |q|^2 - 2 q.c, and the candidate norm moves to a per-column
//    threshold: in iff D <= eps^2 - |c|^2.
// KS = K-steps of 4 dimensions (0 = runtime).
// The 16-candidate tiles of a work item, in order (its ranges in order,
// ceil(len / 16) tiles each), as a table in registers: lane l holds the first
// candidate and the number of valid columns of tile 64c + l (chunk c). Tile
// loops then read a tile's bounds with two v_readlane instead of walking the
// ranges with scalar code.
struct TileTable {
    int tp;      // lane o < nr: first tile of range o
    int ntiles;  // tiles of the item (wave-uniform)
    int tt, tn;  // lane l: first candidate / valid columns of tile 64 * chunk + l
    int chunk;   // chunk held in tt / tn (-1: none)
};

__device__ __forceinline__ void tile_table_init(TileTable &T, const ItemRanges &rg, int lane) {
    int cnt = 0;
    if (lane < rg.nr) {
        const int len = rg.re - rg.rb;
        cnt = len > 0 ? (len + 15) >> 4 : 0;
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    T.tp = incl - cnt;
    T.ntiles = __builtin_amdgcn_readlane(incl, 63);
    T.tt = T.tn = 0;
    T.chunk = -1;
}

__device__ __forceinline__ void tile_table_chunk(TileTable &T, const ItemRanges &rg, int c, int lane) {
    const int K = 64 * c + lane;
    int oo = 0;  // last range whose first tile is <= K (empty ranges share it)
    for (int o = 1; o < rg.nr; ++o)
        if (K >= __builtin_amdgcn_readlane(T.tp, o)) oo = o;
    const int b = __shfl(rg.rb, oo), e = __shfl(rg.re, oo), p = __shfl(T.tp, oo);
    int t = b + 16 * (K - p);
    int n = min(16, e - t);
    if (K >= T.ntiles) t = n = 0;
    T.tt = t;
    T.tn = n;
    T.chunk = c;
}

// Tile k of the item: first candidate and valid columns (wave-uniform).
__device__ __forceinline__ void tile_at(TileTable &T, const ItemRanges &rg, int k, int lane, int &t, int &n) {
    if ((k >> 6) != T.chunk) tile_table_chunk(T, rg, k >> 6, lane);
    t = __builtin_amdgcn_readlane(T.tt, k & 63);
    n = __builtin_amdgcn_readlane(T.tn, k & 63);
}

template <int KS>
struct M64Tile {
    double b[KS > 0 ? KS : 1];
    double nc;   // candidate norm (no-slot form)
    int32_t pc;  // emit: input index of candidate t + j
    int t, n;    // first candidate, valid columns
};

// Issues the loads of tile (t, n); nothing here waits for them.
template <int KS, bool SLOT, int MODE>
__device__ __forceinline__ void m64_load(M64Tile<KS> &T, const DevGrid &G, int t, int n, unsigned boff, int j) {
    // rows up to t + 15 < n + 64 exist (padded). The tile's base address is
    // wave-uniform; the lane part (j * da + g doubles) is a fixed offset.
    T.t = t;
    T.n = n;
    if (KS > 0) {
        const char *__restrict__ base = reinterpret_cast<const char *>(G.xa + (int64_t)t * G.da);
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s)
            T.b[s] = *reinterpret_cast<const double *>(base + boff + 32u * (unsigned)s);
    }
    T.nc = SLOT ? 0.0 : (G.nrm + t)[j];
    if (MODE == MODE_EMIT) T.pc = G.perm[t + min(j, n - 1)];  // n >= 1
}

// Columns j >= n (past the range) must fail every test: SLOT puts +inf into
// the norm slot (the value becomes +inf), no-slot sets the column threshold
// to -inf (m64_colthr).
template <int KS, bool SLOT>
__device__ __forceinline__ double4_t m64_tile(const M64Tile<KS> &T, const DevGrid &G, const double *aq,
                                              double4_t cinit, int j, int g, int qa, bool slot_lane) {
    double4_t acc = cinit;
    if (KS > 0) {
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s) {
            double bv = T.b[s];
            if (SLOT && s == (KS > 0 ? KS : 1) - 1 && slot_lane && j >= T.n) bv = INFINITY;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], bv, acc, 0, 0, 0);
        }
    } else {
        const int d = G.d, da = G.da, ks = da >> 2;
        const double *__restrict__ brow = G.xa + (int64_t)(T.t + j) * da + g;
        const double *__restrict__ arow = G.xa + (int64_t)qa * da;
        const bool colok = j < T.n;
        for (int s = 0; s < ks; ++s) {
            const int kk = 4 * s + g;
            const double a = kk < d ? -2.0 * arow[kk] : ((SLOT && kk == d) ? 1.0 : 0.0);
            double bv = brow[4 * s];
            if (SLOT && kk == d && !colok) bv = INFINITY;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
        }
    }
    return acc;
}

// Per-lane classification state.
struct M64Thr {
    double mid[4];        // SLOT: threshold of row r, eps^2 - |q|^2 (-inf for absent rows)
    double lo[4], hi[4];  // SLOT: mid -/+ Delta (error measurement)
    double ecol;          // no slot: eps^2 for the column threshold
    double nq[4];         // |q|^2 of row r (for the error measurement)
};

// Returns the in-mask (bit r = row g + 4r) after the exact recheck of band
// elements. Columns past the range end are masked here.
template <bool SLOT, int MODE>
__device__ __forceinline__ unsigned m64_classify(double4_t acc, double nc, int t, int ce, int g, int j, int q0,
                                                 const M64Thr &th, double delta, const DevGrid &G,
                                                 unsigned long long &band, unsigned long long &viol,
                                                 double &maxerr) {
    double v0 = acc[0], v1 = acc[1], v2 = acc[2], v3 = acc[3];
    const bool colok = j < ce - t;
    double l0, l1, l2, l3, h0, h1, h2, h3;
    if (SLOT) {
        l0 = th.lo[0]; l1 = th.lo[1]; l2 = th.lo[2]; l3 = th.lo[3];
        h0 = th.hi[0]; h1 = th.hi[1]; h2 = th.hi[2]; h3 = th.hi[3];
        if (!colok) v0 = v1 = v2 = v3 = INFINITY;
    } else {
        const double tc = th.ecol - nc;
        const double lc = colok ? tc - delta : -INFINITY;
        const double hc = colok ? tc + delta : -INFINITY;
        l0 = l1 = l2 = l3 = lc;
        h0 = h1 = h2 = h3 = hc;
    }
    const bool i0 = v0 <= l0, i1 = v1 <= l1, i2 = v2 <= l2, i3 = v3 <= l3;
    const bool m0 = v0 <= h0, m1 = v1 <= h1, m2 = v2 <= h2, m3 = v3 <= h3;
    unsigned inm = (unsigned)i0 | ((unsigned)i1 << 1) | ((unsigned)i2 << 2) | ((unsigned)i3 << 3);
    if (MODE == MODE_MEASURE) {
        const double vv[4] = {v0, v1, v2, v3};
        const double hh[4] = {h0, h1, h2, h3};
        for (int r = 0; r < 4; ++r) {
            if (vv[r] < INFINITY && hh[r] > -INFINITY) {
                const int q = q0 + g + 4 * r;
                const double ex = exact_d2(G.xs + (int64_t)q * G.dp, G.xs + (int64_t)(t + j) * G.dp, G.d);
                if (ex <= 4.0 * G.eps2) {
                    const double err = fabs(vv[r] - (ex - (SLOT ? th.nq[r] : nc)));
                    maxerr = fmax(maxerr, err);
                    if (err > delta) ++viol;
                }
            }
        }
    }
    const bool anyband = (m0 != i0) | (m1 != i1) | (m2 != i2) | (m3 != i3);
    if (__builtin_expect(__any(anyband), 0)) {
        // rare: exact FP64 chain on the original coordinates
        const unsigned mbm = (unsigned)m0 | ((unsigned)m1 << 1) | ((unsigned)m2 << 2) | ((unsigned)m3 << 3);
        const unsigned bm = mbm & ~inm;
        for (int r = 0; r < 4; ++r) {
            if (bm & (1u << r)) {
                const int q = q0 + g + 4 * r;
                const double ex = exact_d2(G.xs + (int64_t)q * G.dp, G.xs + (int64_t)(t + j) * G.dp, G.d);
                if (ex <= G.eps2) inm |= 1u << r;
                ++band;
            }
        }
    }
    return inm;
}

// Count / emit classification on wave-wide compare masks: word r, bit
// 16g + j = (query g + 4r, candidate t + j) is within eps. A value at most
// Delta away from its threshold is decided by the exact FP64 chain; the rest
// by the threshold. `band` (wave-uniform) counts the rechecks.
template <int KS>
__device__ __forceinline__ double m64_colthr(const M64Tile<KS> &T, int j, double eps2) {
    return j < T.n ? eps2 - T.nc : -INFINITY;
}

template <bool SLOT>
__device__ __forceinline__ void m64_words(double4_t acc, double thr_col, int t, int g, int j, int q0,
                                          const M64Thr &th, double delta, const DevGrid &G,
                                          unsigned long long &band, unsigned long long w[4]) {
    double thr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) thr[r] = SLOT ? th.mid[r] : thr_col;
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = __ballot(acc[r] <= thr[r]);
    const double u = fmin(fmin(fabs(acc[0] - thr[0]), fabs(acc[1] - thr[1])),
                          fmin(fabs(acc[2] - thr[2]), fabs(acc[3] - thr[3])));
    if (__builtin_expect(__ballot(u <= delta) != 0ull, 0)) {
        // rare: exact FP64 chain on the original coordinates
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool bl = fabs(acc[r] - thr[r]) <= delta;
            const unsigned long long bm = __ballot(bl);
            if (!bm) continue;
            bool ok = false;
            if (bl) {
                const int q = q0 + g + 4 * r;
                ok = exact_d2(G.xs + (int64_t)q * G.dp, G.xs + (int64_t)(t + j) * G.dp, G.d) <= G.eps2;
            }
            w[r] = (w[r] & ~bm) | __ballot(ok);
            band += (unsigned long long)__popcll(bm);
        }
    }
}

template <int KS, bool SLOT, int MODE>
__device__ __forceinline__ void m64_item(const DevGrid &G, const RefOut &R, double delta, int it) {
    const int lane = threadIdx.x & 63;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int d = G.d, da = G.da;
    const int j = lane & 15;   // A row (query j) / result column (candidate t + j)
    const int g = lane >> 4;   // K index of the operands; row group of the result
    const int qa = q0 + (j < nq ? j : 0);
    const double *__restrict__ xa = G.xa;
    const ItemRanges rg = load_ranges(G, it, lane);
    const unsigned boff = (unsigned)(j * da + g) * 8u;  // lane's B element within a tile
    const bool slot_lane = SLOT && g == (d & 3);         // lane holding the norm slot's K index
    const double eps2 = G.eps2;

    // A operand (16 x K): A[i][k] = -2 q_i[k] for k < d, 1 in the norm slot.
    double aq[KS > 0 ? KS : 1];
    if (KS > 0) {
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s) {
            const int kk = 4 * s + g;
            aq[s] = (j < nq && kk < d) ? -2.0 * xa[(int64_t)qa * da + kk] : ((SLOT && kk == d) ? 1.0 : 0.0);
        }
    }
    // rows of this lane: queries g + 4r
    M64Thr th;
    double4_t cinit = (double4_t){0.0, 0.0, 0.0, 0.0};
    bool emit_r[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = g + 4 * r;
        const bool ok = i < nq;
        const double nq_r = ok ? G.nrm[q0 + i] : 0.0;
        th.nq[r] = nq_r;
        const double thr = eps2 - nq_r;
        th.mid[r] = ok ? thr : -INFINITY;
        th.lo[r] = ok ? thr - delta : -INFINITY;
        th.hi[r] = ok ? thr + delta : -INFINITY;
        if (!SLOT) cinit[r] = ok ? nq_r : INFINITY;
        emit_r[r] = MODE == MODE_EMIT && ok && q0 + i >= R.qlo && q0 + i < R.qhi;
    }
    th.ecol = eps2;
    unsigned long long ebal[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ebal[r] = __ballot(emit_r[r]);
    RowOut ro;
    if (MODE == MODE_EMIT) row_out_init(ro, emit_r, G, R, q0, g, j);
    int cnt[4] = {0, 0, 0, 0};  // in-pairs of row g + 4r in this lane's column
    unsigned long long band = 0, viol = 0;  // band: wave-uniform in count / emit
    double maxerr = 0.0;

    // in-mask recording (count): the words of 16 consecutive tiles gather in
    // one register pair (lane 4s + r = word r of tile s of the group) and
    // leave in one coalesced store
    const bool rec = MODE == MODE_COUNT && R.masks != nullptr;
    const int64_t tile_base = rec ? G.tile_off[it] : 0;
    unsigned mlo = 0, mhi = 0;
    auto consume = [&](const unsigned long long w[4], int k, int t, int32_t pc) {
        if (MODE == MODE_EMIT) {
            unsigned long long bal[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) bal[r] = w[r] & ebal[r];
            tile_store(bal, t, pc, ro, g, j, G, R, q0);
        } else {
            if ((w[0] | w[1] | w[2] | w[3]) != 0ull) {
#pragma unroll
                for (int r = 0; r < 4; ++r) cnt[r] += __builtin_amdgcn_inverse_ballot_w64(w[r]) ? 1 : 0;
                if (rec) {
                    const int sl = 4 * (k & 15);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        mlo = amdgcn_writelane((int)(unsigned)w[r], sl + r, (int)mlo);
                        mhi = amdgcn_writelane((int)(unsigned)(w[r] >> 32), sl + r, (int)mhi);
                    }
                }
            }
            if (rec && (k & 15) == 15) {
                R.masks[(tile_base + k - 15) * 4 + lane] = ((unsigned long long)mhi << 32) | mlo;
                mlo = mhi = 0;
            }
        }
    };

    TileTable TT;
    tile_table_init(TT, rg, lane);
    const int ntiles = TT.ntiles;
    auto load = [&](M64Tile<KS> &T, int k) {
        int tt, tn;
        tile_at(TT, rg, k, lane, tt, tn);
        m64_load<KS, SLOT, MODE>(T, G, tt, tn, boff, j);
    };
    auto classify = [&](const double4_t &acc, const M64Tile<KS> &T, int k) {
        if (MODE == MODE_MEASURE) {
            (void)m64_classify<SLOT, MODE>(acc, T.nc, T.t, T.t + T.n, g, j, q0, th, delta, G, band, viol, maxerr);
        } else {
            unsigned long long w[4];
            m64_words<SLOT>(acc, SLOT ? 0.0 : m64_colthr(T, j, eps2), T.t, g, j, q0, th, delta, G, band, w);
            consume(w, k, T.t, T.pc);
        }
    };
    // both products first, then both classifications
    auto run = [&](const M64Tile<KS> &TA, const M64Tile<KS> &TB, int k) {
        const bool h1 = k + 1 < ntiles;
        const double4_t a0 = m64_tile<KS, SLOT>(TA, G, aq, cinit, j, g, qa, slot_lane);
        double4_t a1;
        if (h1) a1 = m64_tile<KS, SLOT>(TB, G, aq, cinit, j, g, qa, slot_lane);
        classify(a0, TA, k);
        if (h1) classify(a1, TB, k + 1);
    };
    // Four tile buffers, two stages per iteration: a stage runs two tiles
    // while the next two load into the other pair of buffers (fixed roles, so
    // no register copies wait on loads in flight).
    // Loads past the last tile repeat the last tile (same instruction count
    // on every path, so each wait covers exactly the older tiles).
    M64Tile<KS> T0, T1, T2, T3;
    const int klast = ntiles - 1;
    if (ntiles > 0) {
        load(T0, 0);
        load(T1, min(1, klast));
    }
    for (int k = 0; k < ntiles; k += 4) {
        load(T2, min(k + 2, klast));
        load(T3, min(k + 3, klast));
        run(T0, T1, k);
        if (k + 2 >= ntiles) break;
        load(T0, min(k + 4, klast));
        load(T1, min(k + 5, klast));
        run(T2, T3, k + 2);
    }
    if (MODE == MODE_COUNT) {
        if (rec && (ntiles & 15) != 0 && lane < 4 * (ntiles & 15))
            R.masks[(tile_base + (ntiles & ~15)) * 4 + lane] = ((unsigned long long)mhi << 32) | mlo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int v = cnt[r];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            if (j == 0 && g + 4 * r < nq) R.cnt[q0 + g + 4 * r] = v;
        }
        if (lane == 0 && band) atomicAdd(R.band, band);
    }
    if (MODE == MODE_MEASURE) {
        for (int sh = 32; sh > 0; sh >>= 1) {
            viol += __shfl_xor(viol, sh);
            maxerr = fmax(maxerr, __shfl_xor(maxerr, sh));
        }
        if (lane == 0) {
            atomicMax(&R.meas[0], (unsigned long long)__double_as_longlong(maxerr));
            if (viol) atomicAdd(&R.meas[1], viol);
        }
    }
}

template <int KS, bool SLOT, int MODE>
__global__ __launch_bounds__(kThreads) void k_m64(DevGrid G, RefOut R, double delta) {
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    m64_item<KS, SLOT, MODE>(G, R, delta, it);
}

// ------------------------------------------------------------ mask emit --
// Emission from the in-masks recorded by an FP64 count pass (FP64 VALU or
// FP64 MFMA: both record the same canonical masks): per 16 x 16 tile of an
// item, word r, bit 16g + j says whether query g + 4r is within eps of
// candidate j. This pass evaluates no distance; it expands the masks into
// pairs at the exact offsets of the count, through the same LDS ring.
//
// The masks of 16 consecutive tiles arrive in one coalesced vector load (lane
// l holds word l % 4 of tile l / 4), the next 16 are loaded while these are
// expanded, and all-zero tiles are skipped without touching the ring.

// Moves the cursor forward by n >= 0 tiles of 16 candidates.
__device__ __forceinline__ void skip_tiles(TileCursor &tc, const ItemRanges &rg, int n) {
    while (n > 0) {
        const int rem = (tc.ce - tc.t + 15) >> 4;  // tiles left in this range, current included
        if (n < rem) {
            tc.t += 16 * n;
            return;
        }
        n -= rem;
        tc.o = rg.first_nonempty(tc.o + 1);
        if (tc.o >= rg.nr) return;
        tc.t = rg.begin(tc.o);
        tc.ce = rg.end(tc.o);
    }
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int lane) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ void mask_item(const DevGrid &G, const RefOut &R, const unsigned long long *masks,
                                          int it) {
    const int lane = threadIdx.x & 63;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int j = lane & 15;
    const int g = lane >> 4;
    const ItemRanges rg = load_ranges(G, it, lane);
    bool emit_r[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = g + 4 * r;
        emit_r[r] = i < nq && q0 + i >= R.qlo && q0 + i < R.qhi;
    }
    unsigned long long ebal[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ebal[r] = __ballot(emit_r[r]);
    RowOut ro;
    row_out_init(ro, emit_r, G, R, q0, g, j);
    const int64_t tile_base = G.tile_off[it];
    const int ntiles = uniform_i32((int)(G.tile_off[it + 1] - tile_base));
    const int nwords = 4 * ntiles;
    const unsigned long long *mb = masks + tile_base * 4;
    unsigned long long wnext = lane < nwords ? mb[lane] : 0ull;
    TileCursor tc;
    tc.first(rg);
    int at = 0;  // tile the cursor points at
    // one tile in hand: its candidates' input indices load while the next
    // non-empty tile is found
    bool hp = false;
    int tp = 0;
    int32_t pcp = 0;
    unsigned long long wp[4] = {0ull, 0ull, 0ull, 0ull};
    for (int b = 0; b < ntiles; b += 16) {
        const unsigned long long w = wnext;
        if (b + 16 < ntiles) {
            const int idx = 4 * (b + 16) + lane;
            wnext = idx < nwords ? mb[idx] : 0ull;
        }
        unsigned long long nz = __ballot(w != 0ull);
        while (nz) {
            const int k = uniform_i32(__builtin_ctzll(nz) >> 2);
            nz &= ~(0xfull << (4 * k));
            unsigned long long wk[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) wk[r] = readlane_u64(w, 4 * k + r) & ebal[r];
            if (!(wk[0] | wk[1] | wk[2] | wk[3])) continue;
            skip_tiles(tc, rg, b + k - at);
            at = b + k;
            const int t = tc.t;
            int32_t pck = 0;
            if (t + j < tc.ce) pck = G.perm[t + j];
            if (hp) tile_store(wp, tp, pcp, ro, g, j, G, R, q0);
#pragma unroll
            for (int r = 0; r < 4; ++r) wp[r] = wk[r];
            tp = t;
            pcp = pck;
            hp = true;
        }
    }
    if (hp) tile_store(wp, tp, pcp, ro, g, j, G, R, q0);
}

__global__ __launch_bounds__(kThreads) void k_mask_emit(DevGrid G, RefOut R, const unsigned long long *masks) {
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    mask_item(G, R, masks, it);
}

// ------------------------------------------------------------------ batch --
// Persistent work-queue kernel over the work items of many independent
// self-joins. Waves pop global item indices (ordered by descending cost: the
// longest items start first) and run the same per-item tile code as the
// single-problem kernels, with that problem's grid and outputs.
template <int MODE, int PATHV>
__global__ __launch_bounds__(kThreads) void k_batch(const BProb *__restrict__ probs,
                                                    const int64_t *__restrict__ item_base, int B,
                                                    const int32_t *__restrict__ queue, int total,
                                                    int *__restrict__ counter, int32_t *__restrict__ pairs,
                                                    unsigned long long *__restrict__ band) {
    __shared__ uint32_t ring_lds[MODE == MODE_EMIT ? kWaves * 3 * kRing : 1];
    const int lane = threadIdx.x & 63;
    for (;;) {
        int w = 0;
        if (lane == 0) w = atomicAdd(counter, 1);
        w = uniform_i32(__shfl(w, 0));
        if (w >= total) break;
        const int gi = queue[w];
        int lo = 0, hi = B;  // last problem p with item_base[p] <= gi
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (item_base[mid] <= gi) lo = mid;
            else hi = mid;
        }
        const int p = uniform_i32(lo);
        const BProb P = probs[p];
        RefOut R{};
        R.cnt = P.cnt;
        R.off = P.off;
        R.base = 0;
        R.qlo = 0;
        R.qhi = (int32_t)P.G.n;
        R.pairs = pairs + 2 * P.pout;
        R.d2 = nullptr;
        R.band = band;
        R.item_lo = 0;
        const int it = uniform_i32(gi - (int)item_base[p]);
        if (PATHV == SJ_FP64_MFMA) {
            switch (P.ks * 2 + P.slot) {
                case 3: m64_item<1, true, MODE>(P.G, R, P.delta, it); break;
                case 2: m64_item<1, false, MODE>(P.G, R, P.delta, it); break;
                case 5: m64_item<2, true, MODE>(P.G, R, P.delta, it); break;
                case 4: m64_item<2, false, MODE>(P.G, R, P.delta, it); break;
                case 7: m64_item<3, true, MODE>(P.G, R, P.delta, it); break;
                case 6: m64_item<3, false, MODE>(P.G, R, P.delta, it); break;
                case 9: m64_item<4, true, MODE>(P.G, R, P.delta, it); break;
                case 8: m64_item<4, false, MODE>(P.G, R, P.delta, it); break;
                default:
                    if (P.slot) m64_item<0, true, MODE>(P.G, R, P.delta, it);
                    else m64_item<0, false, MODE>(P.G, R, P.delta, it);
                    break;
            }
        } else {
            switch (P.G.d) {
                case 1: v64_item<1, MODE>(P.G, R, it, ring_lds); break;
                case 2: v64_item<2, MODE>(P.G, R, it, ring_lds); break;
                case 3: v64_item<3, MODE>(P.G, R, it, ring_lds); break;
                case 4: v64_item<4, MODE>(P.G, R, it, ring_lds); break;
                case 8: v64_item<8, MODE>(P.G, R, it, ring_lds); break;
                default: v64_item<0, MODE>(P.G, R, it, ring_lds); break;
            }
        }
    }
}

// One block per problem: exclusive scan of its counts (n + 1 entries, the
// last taken as 0) into its prefix array, and its total.
__global__ __launch_bounds__(kThreads) void k_seg_scan(const BProb *__restrict__ probs,
                                                       int64_t *__restrict__ totals) {
    __shared__ int64_t wsum[kWaves];
    __shared__ int64_t carry;
    const BProb P = probs[blockIdx.x];
    const int64_t n1 = P.G.n + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t t0 = 0; t0 < n1; t0 += kThreads) {
        const int64_t i = t0 + tid;
        const int64_t v = (i < P.G.n) ? (int64_t)P.cnt[i] : 0;
        int64_t x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int64_t pre = carry;
        for (int w = 0; w < wave; ++w) pre += wsum[w];
        if (i < n1) const_cast<int64_t *>(P.off)[i] = pre + x - v;
        __syncthreads();
        if (tid == kThreads - 1) carry = pre + x;
        __syncthreads();
    }
    if (tid == 0) totals[blockIdx.x] = carry;
}

__global__ void k_batch_reset(int *counter, unsigned long long *band) {
    *counter = 0;
    *band = 0;
}

DevGrid dev_grid(const Grid &g) {
    DevGrid G;
    G.xs = g.xs;
    G.xa = g.xa;
    G.nrm = g.nrm;
    G.perm = g.perm;
    G.ranges = g.ranges;
    G.items = g.item;
    G.n = g.n;
    G.d = g.d;
    G.dp = g.dp;
    G.da = g.da;
    G.nranges = g.nranges;
    G.nitems = (int32_t)g.items;
    G.eps2 = g.eps2;
    G.tile_off = g.tile_off;
    return G;
}

// Band half-width of the M64 test, from the error analysis of the Gram form:
// |(D' - (eps2 - Nq)) - (d2 - eps2)| <= Delta/2 for every pair whose exact
// distance is near eps (the only pairs whose classification it decides).
//  - stored centred rows x' = fl(x - mid): |x' - (x - mid)| <= u |x - mid|;
//  - norms (FP64 chain of d steps): relative error gamma_d;
//  - MFMA accumulation of d products plus one norm, any order, each step
//    with relative error at most 2u (twice round-to-nearest, for safety);
//  - the oracle's own chain: relative error gamma_{d+2} of |x - y|^2;
//  - threshold eps2 - Nq: one rounding.
// Delta doubles the sum of these terms.
double m64_delta(const Grid &g) {
    const double u = 0x1p-53;
    const int d = g.d;
    auto gam = [&](double m, double uu) { return m * uu / (1.0 - m * uu); };
    const double S = 2.0 * g.nmax * (1.0 + 1e-12);  // Nq + Nc upper bound
    const double E1 = (2.0 * gam(d + 1, 2 * u) + gam(d, u) + u) * S + u * g.eps2;
    const double e = u * 2.0 * std::sqrt(g.nmax) * (1.0 + 1e-12);
    const double tau = g.eps * (1.0 + 4 * u) + e;
    const double tiny = (d + 2) * 0x1p-1021;  // products flushed below the normal range
    return 2.0 * (E1 + 2.0 * tau * e + e * e + gam(d + 2, u) * tau * tau + tiny);
}

template <int MODE>
void launch_v64(const Grid &g, const RefOut &R, int nitems, hipStream_t s) {
    const DevGrid G = dev_grid(g);
    const unsigned blocks = (unsigned)((nitems + kWaves - 1) / kWaves);
    if (!blocks) return;
#define SJ_V64(DD) hipLaunchKernelGGL((k_v64<DD, MODE>), dim3(blocks), dim3(kThreads), 0, s, G, R)
    switch (g.d) {
        case 1: SJ_V64(1); break;
        case 2: SJ_V64(2); break;
        case 3: SJ_V64(3); break;
        case 4: SJ_V64(4); break;
        case 5: SJ_V64(5); break;
        case 6: SJ_V64(6); break;
        case 7: SJ_V64(7); break;
        case 8: SJ_V64(8); break;
        default: SJ_V64(0); break;
    }
#undef SJ_V64
    SJ_HIP(hipGetLastError());
}

template <int MODE>
void launch_m64(const Grid &g, const RefOut &R, int nitems, double delta, hipStream_t s) {
    const DevGrid G = dev_grid(g);
    const unsigned blocks = (unsigned)((nitems + kWaves - 1) / kWaves);
    if (!blocks) return;
    const bool slot = (g.d & 3) != 0;
    const int ks = g.da >> 2;
#define SJ_M64(KSV, SL) hipLaunchKernelGGL((k_m64<KSV, SL, MODE>), dim3(blocks), dim3(kThreads), 0, s, G, R, delta)
    if (slot) {
        switch (ks) {
            case 1: SJ_M64(1, true); break;
            case 2: SJ_M64(2, true); break;
            case 3: SJ_M64(3, true); break;
            case 4: SJ_M64(4, true); break;
            default: SJ_M64(0, true); break;
        }
    } else {
        switch (ks) {
            case 1: SJ_M64(1, false); break;
            case 2: SJ_M64(2, false); break;
            case 3: SJ_M64(3, false); break;
            case 4: SJ_M64(4, false); break;
            default: SJ_M64(0, false); break;
        }
    }
#undef SJ_M64
    SJ_HIP(hipGetLastError());
}

}  // namespace

void launch_batch(bool emit, sj_path path, const BProb *probs, const int64_t *item_base, int B,
                  const int32_t *queue, int total, int *counter, int32_t *pairs, unsigned long long *band,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, counter, band);
    SJ_HIP(hipGetLastError());
    if (total <= 0) return;
    int dev = 0, ncu = 256;
    SJ_HIP(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const unsigned blocks = (unsigned)std::min<int64_t>((total + kWaves - 1) / kWaves, (int64_t)ncu * 8);
#define SJ_B(M, P) hipLaunchKernelGGL((k_batch<M, P>), dim3(blocks), dim3(kThreads), 0, s, probs, item_base, B, queue, \
                                      total, counter, pairs, band)
    if (path == SJ_FP64_MFMA) {
        if (emit) SJ_B(MODE_EMIT, SJ_FP64_MFMA);
        else SJ_B(MODE_COUNT, SJ_FP64_MFMA);
    } else {
        if (emit) SJ_B(MODE_EMIT, SJ_FP64_VALU);
        else SJ_B(MODE_COUNT, SJ_FP64_VALU);
    }
#undef SJ_B
    SJ_HIP(hipGetLastError());
}

DevGrid make_dev_grid(const Grid &g) { return dev_grid(g); }
double fp64_mfma_delta(const Grid &g) { return m64_delta(g); }

void launch_seg_scan(const BProb *probs, int B, int64_t *totals, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_seg_scan, dim3(B), dim3(kThreads), 0, s, probs, totals);
    SJ_HIP(hipGetLastError());
}

// Enqueues the count kernel; the band counter lands in ro.band_dev (device,
// zeroed here) and is read by the caller together with the total.
void refine_count(Grid &g, sj_path path, int32_t *cnt_sorted, RefineOut &ro, hipStream_t s) {
    fill_zero(ro.band_dev, sizeof(unsigned long long), s);
    RefOut R{};
    R.cnt = cnt_sorted;
    R.band = ro.band_dev;
    R.item_lo = 0;
    R.masks = ro.masks;
    ro.cand_eval = g.cand_items;
    if (path == SJ_FP64_VALU) {
        ro.kt.start(ro.timed, s);
        launch_v64<MODE_COUNT>(g, R, (int)g.items, s);
        ro.kt.stop(s);
        ro.band_rel = 0.0;
    } else if (path == SJ_FP64_MFMA) {
        const double delta = m64_delta(g);
        ro.kt.start(ro.timed, s);
        launch_m64<MODE_COUNT>(g, R, (int)g.items, delta, s);
        ro.kt.stop(s);
        ro.band_rel = g.eps2 > 0 ? delta / g.eps2 : 0.0;
    } else {
        lowp_count(g, path, cnt_sorted, ro, s);
    }
}

namespace {

// Chunk plan (result batching, Section III-B): from `cursor`, the largest run
// of whole queries whose pairs fit in `capacity`, and the work items that
// cover it. One thread; binary searches over the prefix sums and the items.
__global__ void k_chunk_plan(const int64_t *__restrict__ off, const Item *__restrict__ items, int64_t n,
                             int64_t nitems, const int32_t *__restrict__ blocks, int64_t nblocks, int64_t cursor,
                             int64_t capacity, int64_t *__restrict__ out) {
    const int64_t base = off[cursor];
    const int64_t need = off[cursor + 1] - base;
    if (need > capacity) {
        out[0] = 1;
        out[1] = need;
        return;
    }
    int64_t a = cursor + 1, b = n;  // largest q in [a, b] with off[q] - base <= capacity
    while (a < b) {
        const int64_t mid = a + (b - a + 1) / 2;
        if (off[mid] - base <= capacity) a = mid;
        else b = mid - 1;
    }
    const int64_t next = a;
    int64_t lo = 0, hi = nitems;  // first item with qend > cursor
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (items[mid].qend <= cursor) lo = mid + 1;
        else hi = mid;
    }
    const int64_t ilo = lo;
    lo = ilo;
    hi = nitems;  // first item with qbegin >= next
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (items[mid].qbegin < next) lo = mid + 1;
        else hi = mid;
    }
    const int64_t ihi = lo;
    // block items: first with blocks[b + 1] > ilo; end = first with blocks[b] >= ihi
    int64_t x = 0, y = nblocks;
    while (x < y) {
        const int64_t mid = x + (y - x) / 2;
        if (blocks[mid + 1] <= ilo) x = mid + 1;
        else y = mid;
    }
    const int64_t blo = x;
    y = nblocks;
    while (x < y) {
        const int64_t mid = x + (y - x) / 2;
        if (blocks[mid] < ihi) x = mid + 1;
        else y = mid;
    }
    out[0] = 0;
    out[1] = off[next] - base;
    out[2] = next;
    out[3] = ilo;
    out[4] = ihi;
    out[5] = base;
    out[6] = blo;
    out[7] = x;
}

}  // namespace

ChunkPlan plan_chunk(Grid &g, int64_t cursor, int64_t capacity, hipStream_t s) {
    int64_t *d = dev_alloc_n<int64_t>(8, s);
    hipLaunchKernelGGL(k_chunk_plan, dim3(1), dim3(1), 0, s, g.off, g.item, g.n, g.items, g.blocks, g.nblocks,
                       cursor, capacity, d);
    SJ_HIP(hipGetLastError());
    int64_t h[8] = {0};
    SJ_HIP(hipMemcpyAsync(h, d, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    dev_free(d, s);
    ChunkPlan p;
    p.too_small = h[0] != 0;
    p.written = h[1];
    p.next = h[2];
    p.item_lo = h[3];
    p.item_hi = h[4];
    p.base = h[5];
    p.block_lo = h[6];
    p.block_hi = h[7];
    return p;
}

void refine_pairs(Grid &g, sj_path path, const ChunkPlan &p, int64_t qlo, int32_t *pairs, double *d2,
                  RefineOut &ro, hipStream_t s) {
    RefOut R{};
    R.off = g.off;
    R.base = p.base;
    R.qlo = (int32_t)qlo;
    R.qhi = (int32_t)p.next;
    R.pairs = pairs;
    R.d2 = d2;
    R.item_lo = (int32_t)p.item_lo;
    fill_zero(ro.band_dev, sizeof(unsigned long long), s);
    R.band = ro.band_dev;
    const int nitems = (int)(p.item_hi - p.item_lo);
    if ((path == SJ_FP64_VALU || path == SJ_FP64_MFMA) && g.masks_valid && g.masks) {
        ro.kt.start(ro.timed, s);
        const unsigned blocks = (unsigned)((nitems + kWaves - 1) / kWaves);
        if (blocks) {
            hipLaunchKernelGGL(k_mask_emit, dim3(blocks), dim3(kThreads), 0, s, dev_grid(g), R,
                               (const unsigned long long *)g.masks);
            SJ_HIP(hipGetLastError());
        }
        ro.kt.stop(s);
    } else if (path == SJ_FP64_VALU) {
        ro.kt.start(ro.timed, s);
        launch_v64<MODE_EMIT>(g, R, nitems, s);
        ro.kt.stop(s);
    } else if (path == SJ_FP64_MFMA) {
        const double delta = m64_delta(g);
        ro.kt.start(ro.timed, s);
        launch_m64<MODE_EMIT>(g, R, nitems, delta, s);
        ro.kt.stop(s);
        ro.band_rel = g.eps2 > 0 ? delta / g.eps2 : 0.0;
    } else {
        lowp_pairs(g, path, p, qlo, pairs, d2, ro, s);
    }
}

void refine_measure(Grid &g, sj_path path, double *max_err, double *max_band, int64_t *viol, hipStream_t s) {
    unsigned long long *meas = dev_alloc_n<unsigned long long>(3, s);
    fill_zero(meas, 3 * sizeof(unsigned long long), s);
    RefOut R{};
    R.meas = meas;
    R.band = meas + 2;
    R.item_lo = 0;
    double delta = 0.0;
    if (path == SJ_FP64_VALU) {
        // the direct form is the exact chain: no band, no error
        *max_err = 0.0;
        *max_band = 0.0;
        *viol = 0;
        dev_free(meas, s);
        return;
    } else if (path == SJ_FP64_MFMA) {
        delta = m64_delta(g);
        launch_m64<MODE_MEASURE>(g, R, (int)g.items, delta, s);
    } else {
        dev_free(meas, s);
        lowp_measure(g, path, max_err, max_band, viol, s);
        return;
    }
    unsigned long long h[2] = {0, 0};
    SJ_HIP(hipMemcpyAsync(h, meas, sizeof h, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    double e;
    std::memcpy(&e, &h[0], sizeof e);
    *max_err = e;
    *max_band = delta;
    *viol = (int64_t)h[1];
    dev_free(meas, s);
}

}  // namespace sj

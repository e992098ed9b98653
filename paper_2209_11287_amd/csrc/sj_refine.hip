// Refine kernels: distance tiles between a work item's queries and the
// candidates of its neighbouring cells (Section II-D "refine"; Section III-B:
// queries of one cell share one candidate set, so a tile's queries come from
// one run of cells).
//
// One wave (64 lanes) owns one work item of up to 16 queries; its candidates
// form one packed list walked in 16 x 16 tiles (rows = queries, columns =
// candidates). Lane (g, j) holds rows g + 4r (r = 0..3) of column j.
//
//  V64 -- FP64 vector ALU, direct form (Eq. (1) in the order of Eq. (2)):
//         each lane evaluates its four pairs with the oracle's chain, so the
//         result is bit-exact by construction. The paper's CUDA-core
//         baseline role.
//  M64 -- FP64 MFMA, expanded form (Eq. (3), Fig. 2): one
//         v_mfma_f64_16x16x4_f64 per K-step computes the tile's Gram part;
//         the candidate norm rides in a spare K slot (or the query norm in the
//         accumulator init when d % 4 == 0) and the other norm moves to the
//         threshold side. A proven error bound Delta splits each value into
//         in / out / band; band pairs are re-evaluated with the exact FP64
//         chain, so the result is the exact set. Fig. 2 needs CUDA-core steps
//         because FP64 WMMA cannot feed an accumulator back; here the norms
//         fold into the contraction and only the threshold test stays on the
//         vector ALU.
// Count passes record per-tile in-masks (nibble words); the pairs pass expands
// them (k_mask_emit) or, without masks, re-runs the tiles in emit mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "sj_internal.h"

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
    DevCounters *ctr;             // rechecks, pruned tiles, measurements
    int32_t item_lo;              // first item of this launch
    unsigned long long *masks;    // count: per-tile in-masks to record (nullable)
};

// MODE_SYM: the count with the half stencil (sym_cut / sym_mask below).
enum { MODE_COUNT = 0, MODE_EMIT = 1, MODE_MEASURE = 2, MODE_SYM = 3 };
constexpr bool is_count(int mode) { return mode == MODE_COUNT || mode == MODE_SYM; }

// Blocks go round-robin over the 8 XCDs (hardware block b runs on XCD b % 8).
// Logical blocks come in chunks of kXcdChunk consecutive ones, so spatially
// adjacent work items (which share candidates) share one XCD's L2; the chunks
// are dealt round-robin to the XCDs, so dense regions of the index (whose
// items are long) spread over all of them. A final partial round keeps the
// hardware order.
constexpr int kXcdChunk = 16;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int full = nb / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (b >= full) return b;
    const int x = b & 7, k = b >> 3;
    return ((k / kXcdChunk) * 8 + x) * kXcdChunk + (k % kXcdChunk);
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders one wave's LDS writes before its later reads of other lanes' slots
// (and those reads before the next writes).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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


// ------------------------------------------------------------ shared parts --
// Candidate ranges of a work item: lane o (< nranges) holds range o's bounds.
struct ItemRanges {
    int rb, re;
    int nr;
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

// The candidates of a work item as one list: its ranges in order, packed
// (a 16-candidate tile may span the end of one range and the start of the
// next; only the item's last tile can be partial). Tile k = list positions
// 16k .. 16k + 15; chunk c = positions 64c .. 64c + 63 (tiles 4c .. 4c + 3).
// A lane finds the sorted index at position P from the range holding P:
// index = P + (begin - first position) of that range. Chunks are visited in
// increasing order; only the ranges that start inside a chunk are read for
// it (typically one or two), the range carried over from the previous chunk
// covers the positions before them.
struct CandList {
    int cp, dlt;                  // lane o < nr: first list position of range o, begin - cp
    unsigned long long nonempty;  // ranges with candidates (wave-uniform)
    int total, ntiles;            // candidates, ceil(total / 16) (wave-uniform)
    int carry;                    // begin - cp of the range holding the next chunk's start
    int fill;                     // a valid sorted index (< n) for positions past the end
};

__device__ __forceinline__ void cand_init(CandList &L, const ItemRanges &rg, int lane, int fill) {
    int len = 0;
    if (lane < rg.nr) len = max(0, rg.re - rg.rb);
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    L.cp = incl - len;
    L.dlt = rg.rb - L.cp;
    L.nonempty = __ballot(len > 0);
    L.total = __builtin_amdgcn_readlane(incl, 63);
    L.ntiles = (L.total + 15) >> 4;
    L.carry = 0;
    L.fill = fill;
}

// Sorted indices at positions P[0..NP) (all inside chunk c) into idx[].
template <int NP>
__device__ __forceinline__ void cand_chunk(CandList &L, int c, const int P[NP], int idx[NP]) {
    const int base = 64 * c;
    unsigned long long st = __ballot(L.cp >= base && L.cp < base + 64) & L.nonempty;
    int dl[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) dl[p] = L.carry;
    while (st) {
        const int o = __builtin_ctzll(st);
        st &= st - 1;
        const int cpo = __builtin_amdgcn_readlane(L.cp, o);
        const int d = __builtin_amdgcn_readlane(L.dlt, o);
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (P[p] >= cpo) dl[p] = d;
        L.carry = d;
    }
    if (base + 64 <= L.total) {
#pragma unroll
        for (int p = 0; p < NP; ++p) idx[p] = P[p] + dl[p];
    } else {
#pragma unroll
        for (int p = 0; p < NP; ++p) idx[p] = P[p] < L.total ? P[p] + dl[p] : L.fill;
    }
}


// Emission. Pairs go to exact offsets (prefix sums of the count pass), so a
// query's pairs form one run in candidate order.
// Direct emission of one 16 x 16 tile from its mask words (canonical
// layout, already restricted to the queries this launch emits): lane (g, j)
// writes pair (query g + 4r, candidate of column j) for each r whose bit it
// holds, at the query's base + pairs so far + the pair's rank among the set
// bits of its 16-bit group. `c` / `pc` = sorted / input index of the lane's
// candidate.
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

__device__ __forceinline__ void tile_store(const unsigned long long w[4], int c, int32_t pc, RowOut &ro, int g,
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
                R.d2[pos] = exact_d2(G.xs + (int64_t)(q0 + g + 4 * r) * G.dp, G.xs + (int64_t)c * G.dp, G.d);
        }
        ro.cur[r] += __popc(ch);
    }
}

// Half-stencil count (symmetric evaluation, FP64 paths): each pair within
// eps is met once, from its smaller sorted index. A work item keeps only the
// candidates at or after its first query q0 (the ranges are cut at q0: a
// line with a smaller key lies wholly before the item's line in the sorted
// order, a larger one wholly after it), and a value (query i, candidate c)
// counts only for c > i, which matters only where the candidates are the
// item's own queries (or, on a shared block list, its block's earlier ones).
// The row sums go to the queries as before; each tile's column sums go to
// its candidates by atomics; every point adds 1 for itself.
__device__ __forceinline__ void sym_cut(ItemRanges &rg, int q0) {
    rg.rb = max(rg.rb, q0);
    rg.re = max(rg.re, rg.rb);
}

// Clears the values (query q0 + g + 4r, candidate c) with c <= that query;
// only tiles holding a candidate below q0 + 16 have any (wave-uniform test).
__device__ __forceinline__ void sym_mask(unsigned long long w[4], int c, int n, int q0, int g, int j) {
    if (__ballot(j < n && c < q0 + 16) == 0ull) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] &= __ballot(c > q0 + g + 4 * r);
}

// The tile's pairs of the lane's column (its four row bits are the low
// nibble of the accumulator right after nib_push), summed over the four row
// groups, added to the candidate's count.
__device__ __forceinline__ void sym_columns(unsigned nacc, int c, int32_t *cnt, int lane) {
    int v = __popc(nacc & 0xFu);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16 && v) atomicAdd(cnt + c, v);
}

// Per-query count of a finished item: the row sums reduced over the 16
// lanes of each row group; with the half stencil they are added (other
// items add their column sums to the same entries) with the point itself.
template <bool SYM>
__device__ __forceinline__ void write_counts(const int tot[4], const RefOut &R, int q0, int nq, int g, int j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int v = tot[r];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if (j == 0 && g + 4 * r < nq) {
            if (SYM) atomicAdd(R.cnt + q0 + g + 4 * r, v + 1);
            else R.cnt[q0 + g + 4 * r] = v;
        }
    }
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
// Operand registers of a tile: every K-step, or (KS > 4, count / emit) the
// current batch of 4.
constexpr int m64_nb(int ks, int mode) { return (ks > 4 && mode != MODE_MEASURE) ? 4 : (ks > 0 ? ks : 1); }

template <int KS, int NB>
struct M64Tile {
    double b[NB];
    double pn;   // candidate prefix norms (short-circuit): KS 2..4: at K-step KS / 2;
                 // KS > 4: lane (g, j) holds the one at K-step 4 t + g + 1 of the batch t in registers
    double nc;   // candidate norm (no-slot form)
    int32_t c;   // sorted index of the lane's column (a valid row past the end)
    int32_t pc;  // emit: input index of that candidate
    int n;       // valid columns (wave-uniform)
};

// Issues the loads of a tile whose column j is candidate c (n valid
// columns); nothing here waits for them.
template <int KS, bool SLOT, int MODE>
__device__ __forceinline__ void m64_load(M64Tile<KS, m64_nb(KS, MODE)> &T, int c, int n, const DevGrid &G, int g) {
    T.c = c;
    T.n = n;
    if (KS > 0) {
        // KS > 4 (count / emit): only the first batch of 4 K-steps ahead of
        // time; each further batch loads after the partial-distance tests of
        // the one before, for tiles that pass them
        constexpr int KL = (KS > 4 && MODE != MODE_MEASURE) ? 4 : (KS > 0 ? KS : 1);
        const double *__restrict__ brow = G.xa + (int64_t)c * G.da + g;
#pragma unroll
        for (int s = 0; s < KL; ++s) T.b[s] = brow[4 * s];
    }
    T.nc = SLOT ? 0.0 : G.nrm[c];
    if (MODE != MODE_MEASURE) {  // prefix norms exist for every grid with KS >= 2
        if (KS > 4) T.pn = G.pn[(int64_t)c * G.npc + g];
        else if (KS >= 2) T.pn = G.pn[(int64_t)c * G.npc + (KS / 2 - 1)];
    }
    if (MODE == MODE_EMIT) T.pc = G.perm[c];
}

template <int KS, bool SLOT>
__device__ __forceinline__ double4_t m64_tile(const M64Tile<KS, (KS > 0 ? KS : 1)> &T, const DevGrid &G, const double *aq,
                                              double4_t cinit, int g, int qa) {
    double4_t acc = cinit;
    if (KS > 0) {
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], T.b[s], acc, 0, 0, 0);
    } else {
        const int d = G.d, da = G.da, ks = da >> 2;
        const double *__restrict__ brow = G.xa + (int64_t)T.c * da + g;
        const double *__restrict__ arow = G.xa + (int64_t)qa * da;
        for (int s = 0; s < ks; ++s) {
            const int kk = 4 * s + g;
            const double a = kk < d ? -2.0 * arow[kk] : ((SLOT && kk == d) ? 1.0 : 0.0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, brow[4 * s], acc, 0, 0, 0);
        }
    }
    return acc;
}

// Per-lane classification state.
struct M64Thr {
    double lo[4], hi[4];  // SLOT: threshold of row r -/+ Delta (-inf for absent rows)
    double clo, chi;      // no slot: eps^2 -/+ Delta (the column norm is subtracted per tile)
    double nq[4];         // |q|^2 of row r (error measurement)
};

// Columns [0, n) of each 16-lane group.
__device__ __forceinline__ unsigned long long col_mask(int n) {
    if (n >= 16) return ~0ull;
    return ((1ull << n) - 1ull) * 0x0001000100010001ull;
}

// Error measurement: for every value whose exact distance is within 2 eps,
// the difference between the Gram value and the exact value (on the same
// side of the threshold equation), its maximum and the count above Delta.
template <bool SLOT, int KS, class TileT>
__device__ __forceinline__ void m64_measure(double4_t acc, const TileT &T, int g, int j, int q0,
                                            const M64Thr &th, double delta, const DevGrid &G,
                                            unsigned long long &viol, double &maxerr) {
    if (j >= T.n) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (th.hi[r] == -INFINITY && SLOT) continue;  // absent row
        if (!SLOT && acc[r] == INFINITY) continue;      // absent row
        const int q = q0 + g + 4 * r;
        const double ex = exact_d2(G.xs + (int64_t)q * G.dp, G.xs + (int64_t)T.c * G.dp, G.d);
        if (ex <= 4.0 * G.eps2) {
            const double err = fabs(acc[r] - (ex - (SLOT ? th.nq[r] : T.nc)));
            maxerr = fmax(maxerr, err);
            if (err > delta) ++viol;
        }
    }
}

// Count / emit classification on wave-wide compare masks: word r, bit
// 16g + j = (query g + 4r, candidate of column j) is within eps. Values at
// or below threshold - Delta are in, above threshold + Delta out; the rest
// are decided by the exact FP64 chain. `band` (wave-uniform) counts them.
template <bool SLOT, int KS, class TileT>
__device__ __forceinline__ void m64_words(double4_t acc, const TileT &T, int g, int q0, const M64Thr &th,
                                          const DevGrid &G, unsigned long long &band, unsigned long long &band_in,
                                          unsigned long long w[4], bool sym = false) {
    double lo[4], hi[4];
    if (SLOT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lo[r] = th.lo[r];
            hi[r] = th.hi[r];
        }
    } else {
        const double l = th.clo - T.nc, h = th.chi - T.nc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lo[r] = l;
            hi[r] = h;
        }
    }
    unsigned long long m[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w[r] = __ballot(acc[r] <= lo[r]);
        m[r] = __ballot(acc[r] <= hi[r]);
    }
    if (T.n < 16) {  // the item's last tile: columns past the end
        const unsigned long long cm = col_mask(T.n);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            w[r] &= cm;
            m[r] &= cm;
        }
    }
    if (sym) {  // half stencil: only candidates after the query
        unsigned long long keep[4] = {~0ull, ~0ull, ~0ull, ~0ull};
        sym_mask(keep, T.c, T.n, q0, g, threadIdx.x & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            w[r] &= keep[r];
            m[r] &= keep[r];
        }
    }
    if (__builtin_expect(((m[0] ^ w[0]) | (m[1] ^ w[1]) | (m[2] ^ w[2]) | (m[3] ^ w[3])) != 0ull, 0)) {
        // rare: exact FP64 chain on the original coordinates
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const unsigned long long bm = m[r] & ~w[r];
            if (!bm) continue;
            bool ok = false;
            if (__builtin_amdgcn_inverse_ballot_w64(bm)) {
                const int q = q0 + g + 4 * r;
                ok = exact_d2(G.xs + (int64_t)q * G.dp, G.xs + (int64_t)T.c * G.dp, G.d) <= G.eps2;
            }
            const unsigned long long okm = __ballot(ok);
            w[r] |= okm;
            band += (unsigned long long)__popcll(bm);
            band_in += (unsigned long long)__popcll(okm);
        }
    }
}

// In-mask words, nibble layout. A group of 16 consecutive tiles of an item
// is 64 words, one per lane (g, j): bit 4s + r says whether query g + 4r is
// within eps of the candidate in column j of tile s of the group.
// Built 8 tiles at a time in a 32-bit register: each tile's four row bits
// enter at the bottom through an add with carry (acc + acc + the lane's bit
// of the row's compare mask), so after t tiles bit 4t - 1 - (4s + r) holds
// (tile s, row r); shifted up and bit-reversed that is bit 4s + r.
__device__ __forceinline__ unsigned shift_in(unsigned acc, unsigned long long mask) {
    unsigned out;
    unsigned long long carry;
    __asm__("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(out), "=s"(carry) : "v"(acc), "s"(mask));
    return out;
}

__device__ __forceinline__ void nib_push(unsigned &acc, const unsigned long long w[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc = shift_in(acc, w[r]);
}

// t (1..8) tiles pushed since the last flush, into half h of the group word.
__device__ __forceinline__ void nib_flush(unsigned long long &nib, unsigned &acc, int t, int h) {
    nib |= (unsigned long long)__builtin_bitreverse32(acc << (32 - 4 * t)) << (32 * h);
    acc = 0;
}

// Pairs of the lane's rows r (queries g + 4r, column j) in a nibble word.
__device__ __forceinline__ void nibble_count(unsigned long long nib, int tot[4]) {
    const unsigned lo = (unsigned)nib, hi = (unsigned)(nib >> 32);
#pragma unroll
    for (int r = 0; r < 4; ++r) tot[r] += __popc(lo & (0x11111111u << r)) + __popc(hi & (0x11111111u << r));
}

template <int KS, bool SLOT, int MODE>
__device__ __forceinline__ void m64_item(const DevGrid &G, const RefOut &R, double delta, int it,
                                         double *tqs /* KS > 4: per-wave LDS, (KS - 1) x 16 */) {
    const int lane = threadIdx.x & 63;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int d = G.d, da = G.da;
    const int j = lane & 15;   // A row (query j) / result column (candidate of column j)
    const int g = lane >> 4;   // K index of the operands; row group of the result
    const int qa = q0 + (j < nq ? j : 0);
    const double *__restrict__ xa = G.xa;
    constexpr bool sym = MODE == MODE_SYM;
    const double eps2 = G.eps2;
    using Tile = M64Tile<KS, m64_nb(KS, MODE)>;
    const bool sc_on = MODE != MODE_MEASURE && KS >= 2 && G.sc != -1;

    // The item's loads first, all unconditional (indices clamped to valid
    // rows), so that one wait covers them: its ranges, the A operand rows,
    // the rows' norms and (one short-circuit check) prefix norms.
    const Range rx = G.ranges[(int64_t)it * G.nranges + min(lane, G.nranges - 1)];
    double xq[KS > 0 ? KS : 1];
    if (KS > 0) {
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s) xq[s] = xa[(int64_t)qa * da + 4 * s + g];  // 4s + g < da
    }
    double nrm4[4], pn4[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int qr = q0 + min(g + 4 * r, nq - 1);
        nrm4[r] = G.nrm[qr];
        pn4[r] = (KS >= 2 && KS <= 4 && sc_on) ? G.pn[(int64_t)qr * G.npc + (KS / 2 - 1)] : 0.0;
    }
    ItemRanges rg;
    rg.nr = G.nranges;
    rg.rb = lane < rg.nr ? rx.begin : 0;
    rg.re = lane < rg.nr ? rx.end : 0;
    // the bounds are settled here, before any tile load (see load_ranges)
    __asm__ volatile("" : "+v"(rg.rb), "+v"(rg.re));
    if (sym) sym_cut(rg, q0);

    // A operand (16 x K): A[i][k] = -2 q_i[k] for k < d, 1 in the norm slot.
    double aq[KS > 0 ? KS : 1];
    if (KS > 0) {
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s) {
            const int kk = 4 * s + g;
            aq[s] = (j < nq && kk < d) ? -2.0 * xq[s] : ((SLOT && kk == d) ? 1.0 : 0.0);
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
        const double nq_r = ok ? nrm4[r] : 0.0;
        th.nq[r] = nq_r;
        const double thr = eps2 - nq_r;
        th.lo[r] = ok ? thr - delta : -INFINITY;
        th.hi[r] = ok ? thr + delta : -INFINITY;
        if (!SLOT) cinit[r] = ok ? nq_r : INFINITY;
        emit_r[r] = MODE == MODE_EMIT && ok && q0 + i >= R.qlo && q0 + i < R.qhi;
    }
    th.clo = eps2 - delta;
    th.chi = eps2 + delta;
    // Partial-distance bound (Section III-B's short-circuit, filter only).
    // After s K-steps (s < KS: the norm slot lies in the last one) the
    // accumulator of row r is cinit_r - 2 q.c over the first 4s columns of
    // xa, so their squared distance is acc - cinit_r + pq_r + pc with the
    // prefix norms pq_r, pc at s. If it exceeds eps^2 + Delta for every value
    // of the tile, no pair of the tile is within eps (the columns' partial
    // distances only grow; Delta bounds the rounding of this partial form as
    // well, which has fewer terms and smaller norms than the full one), and
    // the tile is dropped: per row, acc > tq_r(s) - pc with tq_r(s) = eps^2 +
    // Delta + cinit_r - pq_r(s). Absent rows (tq = -inf) and columns past the
    // item's end never block.
    // KS 2..4: one check, after K-step KS / 2 (tq in registers); KS > 4: a
    // check every `every` K-steps (4 by default), tq of every K-step in a
    // per-wave LDS table [s][g][r], the candidates' prefix norms of a batch
    // of 4 K-steps spread over the lane's row group.
    const int every = G.sc > 0 ? G.sc : 4;
    double tq[4];
    if (KS >= 2 && KS <= 4 && sc_on) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = g + 4 * r;
            tq[r] = i < nq ? eps2 + delta + (SLOT ? 0.0 : th.nq[r]) - pn4[r] : -INFINITY;
        }
    }
    if (KS > 4 && sc_on) {
        for (int e = lane; e < (KS > 4 ? KS - 1 : 1) * 16; e += 64) {
            const int sidx = e >> 4, i = e & 15;
            const double v = i < nq ? eps2 + delta + (SLOT ? 0.0 : G.nrm[q0 + i]) -
                                          G.pn[(int64_t)(q0 + i) * G.npc + sidx]
                                    : -INFINITY;
            tqs[sidx * 16 + (i & 3) * 4 + (i >> 2)] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    unsigned long long npruned = 0;  // wave-uniform
    unsigned long long ebal[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ebal[r] = __ballot(emit_r[r]);
    RowOut ro;
    if (MODE == MODE_EMIT) row_out_init(ro, emit_r, G, R, q0, g, j);
    int tot[4] = {0, 0, 0, 0};  // count: pairs of query g + 4r in this lane's column
    unsigned long long band = 0, band_in = 0, viol = 0;  // band, band_in: wave-uniform
    double maxerr = 0.0;

    // count: the lane's nibbles of 16 consecutive tiles (one group) gather in
    // one 64-bit register; the counts come from it, and with recording on it
    // is stored (64 lanes = one coalesced 512-byte store per group)
    const bool rec = MODE == MODE_COUNT && R.masks != nullptr;
    const int64_t tile_base = rec ? G.tile_off[it] : 0;
    unsigned long long nib = 0;
    unsigned nacc = 0;  // bits of the current half group
    CandList L;
    cand_init(L, rg, lane, q0);
    const int ntiles = L.ntiles;
    const int nchunks = (ntiles + 3) >> 2;
    int flushed = 0;  // tiles whose group is counted (and stored)
    auto group_done = [&](int k0) {  // tiles k0 .. k0 + 15
        const int tg = min(ntiles - k0, 16);  // tiles of this group; those past the last flush are pending
        if (tg & 7) nib_flush(nib, nacc, tg & 7, (tg - 1) >> 3);
        nibble_count(nib, tot);
        if (rec) R.masks[(tile_base + k0) * 4 + lane] = nib;
        nib = 0;
        flushed = k0 + 16;
    };
    auto classify = [&](const double4_t &acc, const Tile &T, int k) {
        if (MODE == MODE_MEASURE) {
            m64_measure<SLOT, KS>(acc, T, g, j, q0, th, delta, G, viol, maxerr);
            return;
        }
        unsigned long long w[4];
        m64_words<SLOT, KS>(acc, T, g, q0, th, G, band, band_in, w, sym);
        if (MODE == MODE_EMIT) {
#pragma unroll
            for (int r = 0; r < 4; ++r) w[r] &= ebal[r];
            tile_store(w, T.c, T.pc, ro, g, j, G, R, q0);
        } else {
            nib_push(nacc, w);
            if (sym) sym_columns(nacc, T.c, R.cnt, lane);
            if ((k & 7) == 7) nib_flush(nib, nacc, 8, (k >> 3) & 1);
        }
    };
    // chunk c: lane (g, j) takes column j of its four tiles, positions 64c + 16s + j
    int cand[4];
    auto chunk = [&](int c) {
        int P[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[t] = 64 * c + 16 * t + j;
        cand_chunk<4>(L, c, P, cand);
    };
    auto load = [&](Tile &T, int k, int c) {
        m64_load<KS, SLOT, MODE>(T, c, min(16, L.total - 16 * k), G, g);
    };
    // a tile dropped by the partial-distance bound: no pairs, zero row bits
    auto prune = [&](int k) {
        ++npruned;
        if (is_count(MODE)) {
            nacc <<= 4;
            if ((k & 7) == 7) nib_flush(nib, nacc, 8, (k >> 3) & 1);
        }
    };
    // wave-uniform: every value of the tile is beyond its row's bound
    auto far_tile = [&](const double4_t &a, int n, const double t4[4], double pc) -> bool {
        const bool far = j >= n || (a[0] > t4[0] - pc && a[1] > t4[1] - pc && a[2] > t4[2] - pc &&
                                    a[3] > t4[3] - pc);
        return __ballot(!far) == 0ull;
    };
    // both products first, then both classifications
    auto run = [&](const Tile &TA, const Tile &TB, int k) {
        const bool h1 = k + 1 < ntiles;
        if constexpr (KS >= 2 && KS <= 4) {
            if (sc_on) {
                // first half of both tiles' K-steps, the bound, the rest
                constexpr int KC = KS / 2;
                double4_t a0 = cinit, a1 = cinit;
#pragma unroll
                for (int s = 0; s < KC; ++s) a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], TA.b[s], a0, 0, 0, 0);
                if (h1) {
#pragma unroll
                    for (int s = 0; s < KC; ++s)
                        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], TB.b[s], a1, 0, 0, 0);
                }
                const bool x0 = far_tile(a0, TA.n, tq, TA.pn);
                const bool x1 = h1 && far_tile(a1, TB.n, tq, TB.pn);
                if (!x0) {
#pragma unroll
                    for (int s = KC; s < KS; ++s)
                        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], TA.b[s], a0, 0, 0, 0);
                }
                if (h1 && !x1) {
#pragma unroll
                    for (int s = KC; s < KS; ++s)
                        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], TB.b[s], a1, 0, 0, 0);
                }
                if (x0) prune(k);
                else classify(a0, TA, k);
                if (h1) {
                    if (x1) prune(k + 1);
                    else classify(a1, TB, k + 1);
                }
                return;
            }
        }
        if constexpr (KS <= 4) {  // KS > 4 runs tiles one at a time (run1)
            const double4_t a0 = m64_tile<KS, SLOT>(TA, G, aq, cinit, g, qa);
            double4_t a1;
            if (h1) a1 = m64_tile<KS, SLOT>(TB, G, aq, cinit, g, qa);
            classify(a0, TA, k);
            if (h1) classify(a1, TB, k + 1);
        }
    };
    if constexpr (KS > 4) {
        // Many K-steps (d > 16): a tile's KS MFMAs dominate, so one tile is
        // in flight while the other runs (two buffers of KS operands each).
        int have = -1;
        auto cand_for = [&](int kk) -> int {
            const int c = kk >> 2;
            if (c != have) {
                chunk(c);
                have = c;
            }
            const int t = kk & 3;
            return t == 0 ? cand[0] : t == 1 ? cand[1] : t == 2 ? cand[2] : cand[3];
        };
        // K-steps s + 1 after which the bound is tested (bit s + 1)
        unsigned long long ckmask = 0;
        if (sc_on)
            for (int s1 = every; s1 < KS; s1 += every) ckmask |= 1ull << s1;
        auto run1 = [&](Tile &T, int k) {
            bool dropped = false;
            double4_t a = cinit;
            if constexpr (MODE == MODE_MEASURE) {
                a = m64_tile<KS, SLOT>(T, G, aq, cinit, g, qa);
            } else {
                // batches of 4 K-steps through the tile's 4 operand
                // registers; batch 0 was loaded ahead
                const double *__restrict__ brow = G.xa + (int64_t)T.c * G.da + g;
#pragma unroll
                for (int bt = 0; bt < (KS > 4 ? (KS + 3) / 4 : 1); ++bt) {
                    if (dropped) break;  // wave-uniform
                    if (bt > 0) {
                        // this batch's operands and candidate prefix norms
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (4 * bt + u < KS) T.b[u] = brow[4 * (4 * bt + u)];
                        if (sc_on) T.pn = 4 * bt + g < G.npc ? G.pn[(int64_t)T.c * G.npc + 4 * bt + g] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int s = 4 * bt + u;
                        if (s >= KS) break;
                        a = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], T.b[u & 3], a, 0, 0, 0);
                        if (s + 1 < KS && ((ckmask >> (s + 1)) & 1ull)) {
                            const double pc = __shfl(T.pn, 16 * u + j);
                            const double *tp = tqs + s * 16 + 4 * g;
                            const double t4[4] = {tp[0], tp[1], tp[2], tp[3]};
                            if (far_tile(a, T.n, t4, pc)) {
                                dropped = true;
                                break;
                            }
                        }
                    }
                }
            }
            if (dropped) prune(k);
            else classify(a, T, k);
            if (is_count(MODE) && (k & 15) == 15) group_done(k - 15);
        };
        const int klast = ntiles - 1;
        Tile TA, TB;
        if (ntiles > 0) load(TA, 0, cand_for(0));
        for (int k = 0; k < ntiles; k += 2) {
            const int k1 = min(k + 1, klast);
            load(TB, k1, cand_for(k1));
            run1(TA, k);
            if (k + 1 >= ntiles) break;
            const int k2 = min(k + 2, klast);
            load(TA, k2, cand_for(k2));
            run1(TB, k + 1);
        }
    } else {
    // Four tile buffers, two stages per chunk: a stage runs two tiles while
    // the next two load into the other pair of buffers (fixed roles, so no
    // register copy waits on a load in flight). Past the item's last tile the
    // loads repeat valid rows (same instruction count on every path, so each
    // wait covers exactly the older tiles) and nothing runs.
    Tile T0, T1, T2, T3;
    if (nchunks > 0) {
        chunk(0);
        load(T0, 0, cand[0]);
        load(T1, 1, cand[1]);
    }
    for (int c = 0; c < nchunks; ++c) {
        const int k = 4 * c;
        load(T2, k + 2, cand[2]);
        load(T3, k + 3, cand[3]);
        run(T0, T1, k);
        if (k + 2 >= ntiles) break;
        if (c + 1 < nchunks) chunk(c + 1);
        load(T0, k + 4, cand[0]);
        load(T1, k + 5, cand[1]);
        run(T2, T3, k + 2);
        if (is_count(MODE) && (c & 3) == 3) group_done(k - 12);
    }
    }
    if (is_count(MODE)) {
        if (flushed < ntiles) group_done(flushed);  // the last, partial group
        // the 16 lanes of row group g hold the columns of queries g + 4r
        write_counts<sym>(tot, R, q0, nq, g, j);
        if (lane == 0 && npruned) atomicAdd(&R.ctr->pruned, npruned);
    }
    if (MODE != MODE_MEASURE && lane == 0 && band) {
        atomicAdd(&R.ctr->rechecked, band);
        atomicAdd(&R.ctr->rechecked_in, band_in);
    }
    if (MODE == MODE_MEASURE) {
        for (int sh = 32; sh > 0; sh >>= 1) {
            viol += __shfl_xor(viol, sh);
            maxerr = fmax(maxerr, __shfl_xor(maxerr, sh));
        }
        if (lane == 0) {
            atomicMax(&R.ctr->max_err, (unsigned long long)__double_as_longlong(maxerr));
            if (viol) atomicAdd(&R.ctr->violations, viol);
        }
    }
}

// Count with LDS-shared candidate tiles, d = 5 .. 16 (2 to 4 K-steps). A
// block is one block item: up to 4 consecutive work items of one line, one
// per wave, which carry the same candidate list (for d > 4 the build unites
// the ranges of a block item's items). Each chunk of 4 tiles is staged once:
// wave w loads the B operand (and the columns' norms and prefix norms) of
// tile w of the chunk into LDS, and every wave then runs its 16 queries
// against all four tiles from LDS, so a candidate row leaves L2 once per 64
// queries instead of once per 16. The next chunk's loads are in flight while
// the current one computes; one barrier per chunk. Waves of a block without
// an item (a line's last block item) stage and wait like the others. The
// classification, in-masks, short-circuit and counts are those of m64_item.
constexpr int m64s_lds_doubles(int ks) { return 2 * 4 * (ks * 64 + 32); }

template <int KS, bool SLOT, bool SYM>
__device__ __forceinline__ void m64_block_count(const DevGrid &G, const RefOut &R, double delta, int bi,
                                                double *__restrict__ lds) {
    const int lane = threadIdx.x & 63;
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int ib = uniform_i32(G.blocks[bi] - G.item_base), ie = uniform_i32(G.blocks[bi + 1] - G.item_base);
    const bool active = ib + wv < ie;  // wave-uniform
    const int it = active ? ib + wv : ib;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = active ? uniform_i32(I.qend - I.qbegin) : 0;
    const int d = G.d, da = G.da;
    const int j = lane & 15, g = lane >> 4;
    const int qa = q0 + (j < nq ? j : 0);
    const double eps2 = G.eps2;
    using Tile = M64Tile<KS, KS>;
    double aq[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int kk = 4 * s + g;
        aq[s] = (j < nq && kk < d) ? -2.0 * G.xa[(int64_t)qa * da + kk] : ((SLOT && kk == d) ? 1.0 : 0.0);
    }
    M64Thr th;
    double4_t cinit = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = g + 4 * r;
        const bool ok = i < nq;
        const double nq_r = ok ? G.nrm[q0 + i] : 0.0;
        th.nq[r] = nq_r;
        th.lo[r] = ok ? eps2 - nq_r - delta : -INFINITY;
        th.hi[r] = ok ? eps2 - nq_r + delta : -INFINITY;
        if (!SLOT) cinit[r] = ok ? nq_r : INFINITY;
    }
    th.clo = eps2 - delta;
    th.chi = eps2 + delta;
    const bool sc_on = KS >= 2 && G.sc != -1;  // one check, after K-step KS / 2
    constexpr int KC = KS >= 2 ? KS / 2 : 1;
    double tq[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = g + 4 * r;
        tq[r] = (sc_on && i < nq) ? eps2 + delta + (SLOT ? 0.0 : th.nq[r]) - G.pn[(int64_t)(q0 + i) * G.npc + (KC - 1)]
                                  : -INFINITY;
    }
    unsigned long long npruned = 0, band = 0, band_in = 0;
    int tot[4] = {0, 0, 0, 0};
    const bool rec = R.masks != nullptr && active;
    const int64_t tile_base = rec ? G.tile_off[it] : 0;
    unsigned long long nib = 0;
    unsigned nacc = 0;
    // the block's list: every wave walks the first item's (united) ranges;
    // half stencil: cut at the block's first query, and each wave keeps the
    // candidates after its own queries (sym_mask)
    ItemRanges rg = load_ranges(G, ib, lane);
    constexpr bool sym = SYM;
    if (sym) sym_cut(rg, uniform_i32(G.items[ib].qbegin));
    CandList L;
    cand_init(L, rg, lane, q0);
    const int ntiles = L.ntiles;  // the same in every wave of the block
    const int nchunks = (ntiles + 3) >> 2;
    int flushed = 0;
    auto group_done = [&](int k0) {
        const int tg = min(ntiles - k0, 16);
        if (tg & 7) nib_flush(nib, nacc, tg & 7, (tg - 1) >> 3);
        nibble_count(nib, tot);
        if (rec) R.masks[(tile_base + k0) * 4 + lane] = nib;
        nib = 0;
        flushed = k0 + 16;
    };
    int cc[4], cn[4];  // sorted indices of the lane's column in the current / next chunk's tiles
    auto chunk = [&](int c, int out[4]) {
        int P[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[t] = 64 * c + 16 * t + j;
        cand_chunk<4>(L, c, P, out);
    };
    // staging registers: this wave's tile of a chunk (tile wv)
    double sb[KS], sx = 0.0;
    auto stage_load = [&](const int col4[4]) {
        const int col = wv == 0 ? col4[0] : wv == 1 ? col4[1] : wv == 2 ? col4[2] : col4[3];
        const double *__restrict__ brow = G.xa + (int64_t)col * da + g;
#pragma unroll
        for (int s = 0; s < KS; ++s) sb[s] = brow[4 * s];
        // lanes of row group 0: the column's norm (no slot); group 1: its prefix norm
        if (g == 0) sx = SLOT ? 0.0 : G.nrm[col];
        else if (g == 1 && KS >= 2) sx = G.pn[(int64_t)col * G.npc + (KC - 1)];
    };
    auto stage_store = [&](int buf) {
        double *t = lds + (buf * 4 + wv) * (KS * 64 + 32);
#pragma unroll
        for (int s = 0; s < KS; ++s) t[s * 64 + lane] = sb[s];
        if (g < 2) t[KS * 64 + g * 16 + j] = sx;
    };
    if (nchunks > 0) {
        chunk(0, cc);
        stage_load(cc);
        stage_store(0);
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {  // block-uniform trip count
        const int buf = c & 1;
        const bool more = c + 1 < nchunks;
        if (more) {
            chunk(c + 1, cn);
            stage_load(cn);  // in flight during this chunk's tiles
        }
        if (active) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = 4 * c + t;
                if (k >= ntiles) break;
                const double *tl = lds + (buf * 4 + t) * (KS * 64 + 32);
                Tile T;
                T.c = cc[t];
                T.n = min(16, L.total - 16 * k);
#pragma unroll
                for (int s = 0; s < KS; ++s) T.b[s] = tl[s * 64 + lane];
                T.nc = tl[KS * 64 + j];
                T.pn = tl[KS * 64 + 16 + j];
                double4_t a = cinit;
#pragma unroll
                for (int s = 0; s < (KS >= 2 ? KC : 0); ++s)
                    a = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], T.b[s], a, 0, 0, 0);
                bool far = false;
                if (sc_on) {
                    const bool f = j >= T.n || (a[0] > tq[0] - T.pn && a[1] > tq[1] - T.pn && a[2] > tq[2] - T.pn &&
                                                a[3] > tq[3] - T.pn);
                    far = __ballot(!f) == 0ull;
                }
                if (far) {
                    ++npruned;
                    nacc <<= 4;
                } else {
#pragma unroll
                    for (int s = (KS >= 2 ? KC : 0); s < KS; ++s)
                        a = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[s], T.b[s], a, 0, 0, 0);
                    unsigned long long w[4];
                    m64_words<SLOT, KS>(a, T, g, q0, th, G, band, band_in, w, sym);
                    nib_push(nacc, w);
                    if (sym) sym_columns(nacc, T.c, R.cnt, lane);
                }
                if ((k & 7) == 7) nib_flush(nib, nacc, 8, (k >> 3) & 1);
                if ((k & 15) == 15) group_done(k - 15);
            }
        }
        if (more) stage_store(buf ^ 1);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) cc[t] = cn[t];
    }
    if (!active) return;
    if (flushed < ntiles) group_done(flushed);
    write_counts<SYM>(tot, R, q0, nq, g, j);
    if (lane == 0) {
        if (npruned) atomicAdd(&R.ctr->pruned, npruned);
        if (band) {
            atomicAdd(&R.ctr->rechecked, band);
            atomicAdd(&R.ctr->rechecked_in, band_in);
        }
    }
}

// Five waves per SIMD (at most 96 VGPRs; the full-stencil forms do not
// spill) took the d = 16 count of a 1M-point Gaussian mixture from 9.5 to
// 8.8 ms against four, and the batched d = 8, 16 counts (k_batch_m64s) 7 %
// lower; six spill, and ran no faster in the batched form.
template <int KS, bool SLOT, bool SYM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_m64s(DevGrid G, RefOut R,
                                                                                             double delta, int nblocks) {
    __shared__ double lds[m64s_lds_doubles(KS)];
    const int bi = xcd_block(blockIdx.x, gridDim.x);
    if (bi >= nblocks) return;  // whole block
    m64_block_count<KS, SLOT, SYM>(G, R, delta, bi, lds);
}

template <int KS, bool SLOT, int MODE>
// d <= 4 (one K-step): six waves per SIMD (at most 80 VGPRs; a few spill in
// the d % 4 = 0 form) hide more of the candidate-load latency than five
// without the cap (~3.5 %). More K-steps: four waves (128 VGPRs, about no
// spills); capped at six they spilled 60-200 bytes per lane and ran 1.3-1.5x
// slower (Gaussian mixture, 1M points, d = 16, 32, 64), at five 1.2x slower.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KS == 1 ? 6 : 4, 8))) void k_m64(
    DevGrid G, RefOut R, double delta) {
    __shared__ double tqbuf[KS > 4 ? kWaves * (KS - 1) * 16 : 1];
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    m64_item<KS, SLOT, MODE>(G, R, delta, it, KS > 4 ? tqbuf + wv * (KS > 4 ? KS - 1 : 1) * 16 : nullptr);
}

// --------------------------------------------------------------------- V64 --
// The FP64 vector-ALU path, direct form (Eq. (1) in the order of Eq. (2)):
// the same 16 x 16 tiles, lane layout and in-mask words as M64, but every
// distance is the oracle's chain (fl(a - b), fma, dimensions ascending), so
// the result needs no band. Lane (g, j) evaluates its four rows (queries
// g + 4r) against its column's candidate. D > 0: the query rows sit in
// registers; D = 0: runtime d, read per dimension.
template <int D>
struct V64Tile {
    double x[D > 0 ? D : 1];
    int32_t c, pc;
    int n;
};

template <int D, int MODE>
__device__ __forceinline__ void v64_load(V64Tile<D> &T, int c, int n, const DevGrid &G) {
    T.c = c;
    T.n = n;
    if (D > 0) {
        const double *__restrict__ xc = G.xs + (int64_t)c * G.dp;
#pragma unroll
        for (int u = 0; u < (D > 0 ? D : 1); ++u) T.x[u] = xc[u];
    }
    if (MODE == MODE_EMIT) T.pc = G.perm[c];
}

// Runtime d (D = 0) up to this many dimensions: the item's query rows are
// staged in LDS (16 rows per wave) and each candidate value is read once per
// dimension for all four rows of the lane.
constexpr int kV64LdsD = 64;

template <int D, int MODE>
__device__ __forceinline__ void v64_item(const DevGrid &G, const RefOut &R, int it, double *qlds, double *cst) {
    const int lane = threadIdx.x & 63;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int j = lane & 15;
    const int g = lane >> 4;
    const int d = D > 0 ? D : G.d;
    const int dp = G.dp;
    const double eps2 = G.eps2;
    const double *__restrict__ xs = G.xs;
    constexpr bool sym = MODE == MODE_SYM;
    // short-circuit interval in dimensions (0 = off): every 4 by default
    const int cd = (MODE == MODE_MEASURE || d <= 4 || G.sc == -1) ? 0 : 4 * (G.sc > 0 ? G.sc : 1);

    // the item's loads first (ranges, query rows), one wait for them all
    const Range rx = G.ranges[(int64_t)it * G.nranges + min(lane, G.nranges - 1)];
    bool rowok[4], emit_r[4];
    int qrow[4];
    double xq[4][D > 0 ? D : 1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = g + 4 * r;
        rowok[r] = i < nq;
        qrow[r] = q0 + (rowok[r] ? i : 0);
        emit_r[r] = MODE == MODE_EMIT && rowok[r] && q0 + i >= R.qlo && q0 + i < R.qhi;
        if (D > 0) {
#pragma unroll
            for (int u = 0; u < (D > 0 ? D : 1); ++u) xq[r][u] = xs[(int64_t)qrow[r] * dp + u];
        }
    }
    ItemRanges rg;
    rg.nr = G.nranges;
    rg.rb = lane < rg.nr ? rx.begin : 0;
    rg.re = lane < rg.nr ? rx.end : 0;
    // the bounds are settled here, before any tile load (see load_ranges)
    __asm__ volatile("" : "+v"(rg.rb), "+v"(rg.re));
    if (sym) sym_cut(rg, q0);
    const bool use_lds = D == 0 && qlds != nullptr && d <= kV64LdsD;
    if (use_lds) {
        for (int i = 0; i < nq; ++i)
            for (int u = lane; u < d; u += 64) qlds[i * kV64LdsD + u] = xs[(int64_t)(q0 + i) * dp + u];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    unsigned long long npruned = 0;  // wave-uniform: tiles left early
    unsigned long long ebal[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ebal[r] = __ballot(emit_r[r]);
    RowOut ro;
    if (MODE == MODE_EMIT) row_out_init(ro, emit_r, G, R, q0, g, j);
    int tot[4] = {0, 0, 0, 0};
    const bool rec = MODE == MODE_COUNT && R.masks != nullptr;
    const int64_t tile_base = rec ? G.tile_off[it] : 0;
    unsigned long long nib = 0;
    unsigned nacc = 0;  // bits of the current half group
    int flushed = 0;
    CandList L;
    cand_init(L, rg, lane, q0);
    const int ntiles = L.ntiles;
    const int nchunks = (ntiles + 3) >> 2;
    auto group_done = [&](int k0) {
        const int tg = min(ntiles - k0, 16);  // tiles of this group; those past the last flush are pending
        if (tg & 7) nib_flush(nib, nacc, tg & 7, (tg - 1) >> 3);
        nibble_count(nib, tot);
        if (rec) R.masks[(tile_base + k0) * 4 + lane] = nib;
        nib = 0;
        flushed = k0 + 16;
    };
    auto run1 = [&](const V64Tile<D> &T, int k) {
        unsigned long long w[4];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        // Every pair's chain runs over the dimensions in order. Each step adds
        // a non-negative square with round-to-nearest, so the chain never
        // decreases: once every value of the tile is above eps^2 (checked
        // every cd dimensions) the tile is out, exactly (Section III-B's
        // short-circuit, with no margin needed); its values stay above eps^2,
        // so the classification below gives zero bits.
        auto all_far = [&]() -> bool {
            bool far = true;
#pragma unroll
            for (int r = 0; r < 4; ++r) far = far && (!rowok[r] || acc[r] > eps2);
            return __ballot(!(far || j >= T.n)) == 0ull;
        };
        if (D > 0) {
            // d <= 8: the query rows sit in registers and the chain runs
            // without checks (a check after 4 dimensions needs more
            // registers than it saves: one wave fewer per SIMD, slower even
            // where half the tiles could leave early)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int u = 0; u < (D > 0 ? D : 1); ++u) {
                    const double dl = __dsub_rn(xq[r][u], T.x[u]);
                    acc[r] = __fma_rn(dl, dl, acc[r]);
                }
        } else {
            const double *__restrict__ b = xs + (int64_t)T.c * dp;
            int next_ck = cd > 0 ? cd : d + 1;  // dimensions after which the next check runs
            auto chain = [&](auto from_lds) {
                for (int u0 = 0; u0 < d; u0 += 16) {
                    // the block's 16 candidate values of the lane's column
                    double bv[16];
                    if (cst) {
                        // lane (g, j) fetches dimensions u0 + 4g .. + 3 of its
                        // candidate in two 16-byte loads (rows are 32-byte
                        // aligned, zero-padded to dp, and followed by padding
                        // rows); the column's 16 values meet in LDS
                        const double2 *__restrict__ src = reinterpret_cast<const double2 *>(b + u0 + 4 * g);
                        const double2 v0 = src[0], v1 = src[1];
                        wave_lds_sync();
                        double2 *dst = reinterpret_cast<double2 *>(cst + 16 * j + 4 * g);
                        dst[0] = v0;
                        dst[1] = v1;
                        wave_lds_sync();
                        const double2 *rd = reinterpret_cast<const double2 *>(cst + 16 * j);
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const double2 pr = rd[t];
                            bv[2 * t] = pr.x;
                            bv[2 * t + 1] = pr.y;
                        }
                    } else {
                        // indices clamped into the row; steps past d skipped
#pragma unroll
                        for (int t = 0; t < 16; ++t) bv[t] = b[min(u0 + t, d - 1)];
                    }
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        const int u = u0 + t;
                        if (u < d) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                double qv;
                                if constexpr (decltype(from_lds)::value) qv = qlds[(g + 4 * r) * kV64LdsD + u];
                                else qv = xs[(int64_t)qrow[r] * dp + u];
                                const double dl = __dsub_rn(qv, bv[t]);
                                acc[r] = __fma_rn(dl, dl, acc[r]);
                            }
                        }
                        if (u + 1 == next_ck) {  // wave-uniform
                            next_ck += cd;
                            if (u + 1 < d && all_far()) {
                                ++npruned;
                                return;
                            }
                        }
                    }
                }
            };
            if (use_lds) chain(std::true_type{});
            else chain(std::false_type{});
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = __ballot(rowok[r] && acc[r] <= eps2);
        if (T.n < 16) {
            const unsigned long long cm = col_mask(T.n);
#pragma unroll
            for (int r = 0; r < 4; ++r) w[r] &= cm;
        }
        if (sym) sym_mask(w, T.c, T.n, q0, g, j);
        if (MODE == MODE_EMIT) {
#pragma unroll
            for (int r = 0; r < 4; ++r) w[r] &= ebal[r];
            tile_store(w, T.c, T.pc, ro, g, j, G, R, q0);
        } else {
            nib_push(nacc, w);
            if (sym) sym_columns(nacc, T.c, R.cnt, lane);
            if ((k & 7) == 7) nib_flush(nib, nacc, 8, (k >> 3) & 1);
        }
    };
    int cand[4];
    auto chunk = [&](int c) {
        int P[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[t] = 64 * c + 16 * t + j;
        cand_chunk<4>(L, c, P, cand);
    };
    auto load = [&](V64Tile<D> &T, int k, int c) { v64_load<D, MODE>(T, c, min(16, L.total - 16 * k), G); };
    auto run = [&](const V64Tile<D> &TA, const V64Tile<D> &TB, int k) {
        run1(TA, k);
        if (k + 1 < ntiles) run1(TB, k + 1);
    };
    // the M64 pipeline: four tile buffers, two stages per chunk
    V64Tile<D> T0, T1, T2, T3;
    if (nchunks > 0) {
        chunk(0);
        load(T0, 0, cand[0]);
        load(T1, 1, cand[1]);
    }
    for (int c = 0; c < nchunks; ++c) {
        const int k = 4 * c;
        load(T2, k + 2, cand[2]);
        load(T3, k + 3, cand[3]);
        run(T0, T1, k);
        if (k + 2 >= ntiles) break;
        if (c + 1 < nchunks) chunk(c + 1);
        load(T0, k + 4, cand[0]);
        load(T1, k + 5, cand[1]);
        run(T2, T3, k + 2);
        if (is_count(MODE) && (c & 3) == 3) group_done(k - 12);
    }
    if (is_count(MODE)) {
        if (flushed < ntiles) group_done(flushed);
        write_counts<sym>(tot, R, q0, nq, g, j);
        if (lane == 0 && npruned) atomicAdd(&R.ctr->pruned, npruned);
    }
}

template <int D, int MODE>
__global__ __launch_bounds__(kThreads) void k_v64(DevGrid G, RefOut R) {
    __shared__ double qbuf[D == 0 ? kWaves * 16 * kV64LdsD : 1];
    __shared__ double cbuf[D == 0 ? kWaves * 256 : 1];
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    v64_item<D, MODE>(G, R, it, D == 0 ? qbuf + wv * 16 * kV64LdsD : nullptr, D == 0 ? cbuf + wv * 256 : nullptr);
}

// ------------------------------------------------------------ mask emit --
// Emission from the in-masks recorded by an FP64 count pass (FP64 VALU or
// FP64 MFMA: both record the same nibble words). This pass evaluates no
// distance; it expands the masks into pairs at the exact offsets of the
// count.
//
// Tiles are taken one group (16 tiles) at a time: the lane's nibble word in
// one coalesced load and the input indices of the group's candidates in four
// (load q = chunk 4G + q of the candidate list, lane l = position 64 (4G + q)
// + l), all issued one group ahead; groups with nothing to write are skipped.
struct MaskBatch {
    unsigned long long w;  // the lane's nibble word
    int32_t pc[4];         // input index of the candidate
    int32_t c[4];          // sorted index of the candidate
};

// D2 (distances requested): the sorted indices (rows for the exact chain;
// the input index is looked up per pair); otherwise the input indices.
template <bool D2>
__device__ __forceinline__ void mask_batch_load(MaskBatch &B, CandList &L, const unsigned long long *mb,
                                                const DevGrid &G, int gi, int lane) {
    B.w = mb[64 * gi + lane];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = 4 * gi + q;
        const int P[1] = {64 * c + lane};
        int idx[1];
        cand_chunk<1>(L, c, P, idx);
        if (D2) B.c[q] = idx[0];
        else B.pc[q] = G.perm[idx[0]];
    }
}

template <int CTRL>
__device__ __forceinline__ unsigned dpp(unsigned x) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, true);
}

// Value of lane (lane ^ B), B in {1, 2, 4, 8}: quad permutes, a half-row
// mirror followed by a quad reversal (i ^ 7 ^ 3 = i ^ 4), a row rotate by 8.
template <int B>
__device__ __forceinline__ unsigned lane_xor(unsigned x) {
    if constexpr (B == 1) return dpp<0xB1>(x);
    else if constexpr (B == 2) return dpp<0x4E>(x);
    else if constexpr (B == 4) return dpp<0x1B>(dpp<0x141>(x));
    else return dpp<0x128>(x);
}

// Exchanges bit positions p and p + D of v for the positions p in M.
template <int D, unsigned M>
__device__ __forceinline__ unsigned delta_swap(unsigned v) {
    const unsigned t = ((v >> D) ^ v) & M;
    return v ^ t ^ (t << D);
}

// 32 bits as 8 nibbles (bit 4s + r) to 4 bytes (bit 8r + s): the bit index
// [s2 s1 s0 r1 r0] rotated to [r1 r0 s2 s1 s0] by four index-bit exchanges.
__device__ __forceinline__ unsigned nibbles_to_bytes(unsigned v) {
    v = delta_swap<14, 0x0000CCCCu>(v);  // index bits 4 and 1
    v = delta_swap<7, 0x00AA00AAu>(v);   // 3 and 0
    v = delta_swap<2, 0x0C0C0C0Cu>(v);   // 2 and 1
    return delta_swap<1, 0x22222222u>(v);  // 1 and 0
}

// One step of a 16 x 16 bit transpose across the lanes of each row (two
// matrices, one per 16-bit half): lanes with bit B set take the partner's
// bits of the other column block, rotated into place.
template <int B, unsigned LO>
__device__ __forceinline__ unsigned transpose_step(unsigned x, int lane) {
    const unsigned p = lane_xor<B>(x);
    const bool up = (lane & B) != 0;
    const unsigned rot = __builtin_amdgcn_alignbit(p, p, up ? B : 32 - B);
    const unsigned m = up ? LO : ~LO;
    return (rot & m) | (x & ~m);
}

__device__ __forceinline__ unsigned transpose16x2(unsigned x, int lane) {
    x = transpose_step<8, 0x00FF00FFu>(x, lane);
    x = transpose_step<4, 0x0F0F0F0Fu>(x, lane);
    x = transpose_step<2, 0x33333333u>(x, lane);
    return transpose_step<1, 0x55555555u>(x, lane);
}

__device__ __forceinline__ unsigned popc16x2(unsigned v) {
    return (unsigned)__popc(v & 0xFFFFu) | ((unsigned)__popc(v >> 16) << 16);
}

constexpr int kSlot = 256;  // LDS pair slots per row group (one query's pairs of a group)

// The pairs of one group of 16 tiles. Lane (g, j) holds the nibble word w
// (bit 4s + r: query g + 4r, column j of tile s). Per-lane nibbles become
// row-major bits (x_r, bit s); a transpose within each row group gives lane
// (g, s) the column bits y_r of tile s, and a scan over s the rank of the
// tile's first pair in the query's run. Then, row by row, each lane (g, s)
// drops its tile's candidates at consecutive ranks in the row group's LDS
// slot (candidate order), and the query's run leaves the slot as contiguous
// stores, 16 lanes per row group.
template <bool D2>
__device__ __forceinline__ void emit_group(unsigned long long w, const MaskBatch &cur, int64_t base[4],
                                           const int32_t pq[4], int g, int j, int lane, const DevGrid &G,
                                           const RefOut &R, int q0, int32_t *stage, int32_t *slot) {
    if (__ballot(w != 0ull) == 0ull) return;
    const unsigned rl = nibbles_to_bytes((unsigned)w), rh = nibbles_to_bytes((unsigned)(w >> 32));
    const unsigned y01 = transpose16x2(__builtin_amdgcn_perm(rh, rl, 0x05010400u), lane);
    const unsigned y23 = transpose16x2(__builtin_amdgcn_perm(rh, rl, 0x07030602u), lane);
    const unsigned c01 = popc16x2(y01), c23 = popc16x2(y23);
    unsigned i01 = c01, i23 = c23;  // inclusive scans over s (16-bit halves)
    i01 += dpp<0x111>(i01);
    i23 += dpp<0x111>(i23);
    i01 += dpp<0x112>(i01);
    i23 += dpp<0x112>(i23);
    i01 += dpp<0x114>(i01);
    i23 += dpp<0x114>(i23);
    i01 += dpp<0x118>(i01);
    i23 += dpp<0x118>(i23);
    unsigned t01 = c01, t23 = c23;  // pairs per query of the row group
    t01 += lane_xor<1>(t01);
    t23 += lane_xor<1>(t23);
    t01 += lane_xor<2>(t01);
    t23 += lane_xor<2>(t23);
    t01 += lane_xor<4>(t01);
    t23 += lane_xor<4>(t23);
    t01 += lane_xor<8>(t01);
    t23 += lane_xor<8>(t23);
    const unsigned p01 = i01 - c01, p23 = i23 - c23;
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) stage[64 * q + lane] = D2 ? cur.c[q] : cur.pc[q];
    int32_t *const own = slot + kSlot * g;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sh = 16 * (r & 1);
        const unsigned T = ((r < 2 ? t01 : t23) >> sh) & 0xFFFFu;
        if (__ballot(T != 0u) == 0ull) continue;
        wave_lds_sync();
        unsigned yy = ((r < 2 ? y01 : y23) >> sh) & 0xFFFFu;
        int32_t *at = own + (((r < 2 ? p01 : p23) >> sh) & 0xFFFFu);
        const int32_t *const tile = stage + 16 * j;
        while (yy) {
            const int col = __builtin_ctz(yy);
            yy &= yy - 1u;
            *at++ = tile[col];
        }
        wave_lds_sync();
        for (unsigned m = 0; m < T; m += 16) {
            const unsigned k = m + j;
            if (k < T) {
                const int32_t v = own[k];
                const int64_t pos = base[r] + k;
                if (D2) {
                    reinterpret_cast<int2 *>(R.pairs)[pos] = make_int2(pq[r], G.perm[v]);
                    R.d2[pos] = exact_d2(G.xs + (int64_t)(q0 + g + 4 * r) * G.dp, G.xs + (int64_t)v * G.dp, G.d);
                } else {
                    reinterpret_cast<int2 *>(R.pairs)[pos] = make_int2(pq[r], v);
                }
            }
        }
        base[r] += T;
    }
}

template <bool D2>
__device__ __forceinline__ void mask_item(const DevGrid &G, const RefOut &R, const unsigned long long *masks,
                                          int it, int32_t *stage, int32_t *slot) {
    const int lane = threadIdx.x & 63;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int j = lane & 15;
    const int g = lane >> 4;
    // the item's loads first, all unconditional (indices clamped to valid
    // rows), one wait for them all: its ranges, its rows' output offsets
    // and input indices, its first in-mask slot
    const Range rx = G.ranges[(int64_t)it * G.nranges + min(lane, G.nranges - 1)];
    bool emit_r[4];
    unsigned erows = 0;  // rows of this lane that this launch emits
    int64_t offr[4];
    int32_t pqr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = g + 4 * r;
        const int q = q0 + min(i, nq - 1);
        offr[r] = R.off[q];
        pqr[r] = G.perm[q];
        emit_r[r] = i < nq && q0 + i >= R.qlo && q0 + i < R.qhi;
        erows |= emit_r[r] ? 1u << r : 0u;
    }
    const int64_t toff = G.tile_off[it];
    ItemRanges rg;
    rg.nr = G.nranges;
    rg.rb = lane < rg.nr ? rx.begin : 0;
    rg.re = lane < rg.nr ? rx.end : 0;
    // the bounds are settled here, before the group loads (see load_ranges)
    __asm__ volatile("" : "+v"(rg.rb), "+v"(rg.re));
    const unsigned long long ekeep = 0x1111111111111111ull * erows;
    RowOut ro;  // as row_out_init
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ro.qb[r] = emit_r[r] ? offr[r] - R.base : 0;
        ro.pq[r] = emit_r[r] ? pqr[r] : 0;
        ro.cur[r] = 0;
    }
    ro.jlt = (1u << j) - 1u;
    int64_t base[4] = {ro.qb[0], ro.qb[1], ro.qb[2], ro.qb[3]};
    CandList L;
    cand_init(L, rg, lane, q0);
    const int ngroups = (L.ntiles + 15) >> 4;
    const unsigned long long *mb = masks + toff * 4;
    MaskBatch nxt;
    if (ngroups > 0) mask_batch_load<D2>(nxt, L, mb, G, 0, lane);
    for (int gi = 0; gi < ngroups; ++gi) {
        const MaskBatch cur = nxt;
        if (gi + 1 < ngroups) mask_batch_load<D2>(nxt, L, mb, G, gi + 1, lane);
        emit_group<D2>(cur.w & ekeep, cur, base, ro.pq, g, j, lane, G, R, q0, stage, slot);
    }
}

// Seven waves per SIMD (72 VGPRs; no spill without distances, 20 KB of LDS
// per block) hide more of the group loads than six (~5 %).
template <bool D2>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_mask_emit(DevGrid G,
                                                                                                 RefOut R,
                                                                                                 const unsigned long long *masks) {
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    __shared__ int32_t stage[kWaves * 256];
    __shared__ int32_t slot[kWaves * 4 * kSlot];
    if (it >= G.nitems) return;
    mask_item<D2>(G, R, masks, it, stage + 256 * wv, slot + 4 * kSlot * wv);
}

// ------------------------------------------------------------------ batch --
// Work items of many independent self-joins. The queue holds global item
// indices grouped by tile form (the problems' d) and, within a form, by
// descending cost. One launch per form: wave w of W takes queue positions
// lo + w, lo + w + W, ... (W = the waves the grid holds: either every wave
// the GPU keeps resident, a persistent grid dealing the longest items first
// round-robin, or one wave per item, the dispatcher handing out items in
// queue order). Each item runs the single-problem tile code with its
// problem's grid and outputs.
__device__ __forceinline__ int batch_problem(const int64_t *__restrict__ item_base, int B, int gi) {
    int lo = 0, hi = B;  // last problem p with item_base[p] <= gi
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (item_base[mid] <= gi) lo = mid;
        else hi = mid;
    }
    return uniform_i32(lo);
}

__device__ __forceinline__ RefOut batch_out(const BProb &P, int32_t *pairs, DevCounters *ctr, int mode) {
    RefOut R{};
    R.cnt = P.cnt;
    R.off = P.off;
    R.base = 0;
    R.qlo = 0;
    R.qhi = (int32_t)P.G.n;
    R.pairs = pairs ? pairs + 2 * P.pout : nullptr;
    R.d2 = nullptr;
    R.ctr = ctr;
    R.item_lo = 0;
    R.masks = mode == MODE_COUNT ? P.masks : nullptr;
    return R;
}

template <int KS, bool SLOT, int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KS == 1 ? 6 : 4, 8))) void k_batch_m64(
    const BProb *__restrict__ probs, const int64_t *__restrict__ item_base, int B, const int32_t *__restrict__ queue,
    int lo, int hi, int32_t *__restrict__ pairs, DevCounters *__restrict__ ctr) {
    __shared__ double tqbuf[KS > 4 ? kWaves * (KS - 1) * 16 : 1];
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int W = gridDim.x * kWaves;
    for (int w = lo + uniform_i32(blockIdx.x * kWaves + wv); w < hi; w += W) {
        const int gi = queue[w];
        const int p = batch_problem(item_base, B, gi);
        const BProb &P = probs[p];
        const RefOut R = batch_out(P, pairs, ctr, MODE);
        const int it = uniform_i32(gi - (int)item_base[p]);
        m64_item<KS, SLOT, MODE>(P.G, R, P.delta, it, KS > 4 ? tqbuf + wv * (KS > 4 ? KS - 1 : 1) * 16 : nullptr);
    }
}

template <int D, int MODE>
__global__ __launch_bounds__(kThreads) void k_batch_v64(const BProb *__restrict__ probs,
                                                        const int64_t *__restrict__ item_base, int B,
                                                        const int32_t *__restrict__ queue, int lo, int hi,
                                                        int32_t *__restrict__ pairs, DevCounters *__restrict__ ctr) {
    __shared__ double qbuf[D == 0 ? kWaves * 16 * kV64LdsD : 1];
    __shared__ double cbuf[D == 0 ? kWaves * 256 : 1];
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int W = gridDim.x * kWaves;
    for (int w = lo + uniform_i32(blockIdx.x * kWaves + wv); w < hi; w += W) {
        const int gi = queue[w];
        const int p = batch_problem(item_base, B, gi);
        const BProb &P = probs[p];
        const RefOut R = batch_out(P, pairs, ctr, MODE);
        const int it = uniform_i32(gi - (int)item_base[p]);
        v64_item<D, MODE>(P.G, R, it, D == 0 ? qbuf + wv * 16 * kV64LdsD : nullptr,
                          D == 0 ? cbuf + wv * 256 : nullptr);
    }
}

// FP64 MFMA count of the block items of many problems (d = 5 .. 16, united
// candidate lists): as k_m64s, one block item per block at a time, the block
// queue's positions [lo, hi) taken round-robin by the grid's blocks.
template <int KS, bool SLOT, bool SYM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_batch_m64s(
    const BProb *__restrict__ probs, const int64_t *__restrict__ block_base, int B, const int32_t *__restrict__ bqueue,
    int lo, int hi, DevCounters *__restrict__ ctr) {
    __shared__ double lds[m64s_lds_doubles(KS)];
    for (int w = lo + (int)blockIdx.x; w < hi; w += (int)gridDim.x) {  // block-uniform
        const int gb = bqueue[w];
        const int p = batch_problem(block_base, B, gb);
        const BProb &P = probs[p];
        const RefOut R = batch_out(P, nullptr, ctr, SYM ? MODE_SYM : MODE_COUNT);
        m64_block_count<KS, SLOT, SYM>(P.G, R, P.delta, uniform_i32(gb - (int)block_base[p]), lds);
    }
}

// Every problem's per-point counts set to zero before a half-stencil count
// adds into them (a kernel, so that the count graph holds no memset node):
// problems blockIdx.y, blockIdx.y + gridDim.y, ..., each swept along x.
__global__ __launch_bounds__(kThreads) void k_batch_zero_cnt(const BProb *__restrict__ probs, int B) {
    for (int p = (int)blockIdx.y; p < B; p += (int)gridDim.y) {
        int32_t *const c = probs[p].cnt;
        const int64_t n = probs[p].G.n;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            c[i] = 0;
    }
}

// Pairs of every item from the in-masks its problem's count pass recorded
// (no distance is recomputed), at the problem's output rows.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_batch_emit(
    const BProb *__restrict__ probs, const int64_t *__restrict__ item_base, int B, const int32_t *__restrict__ queue,
    int lo, int hi, int32_t *__restrict__ pairs) {
    __shared__ int32_t stage[kWaves * 256];
    __shared__ int32_t slot[kWaves * 4 * kSlot];
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int W = gridDim.x * kWaves;
    for (int w = lo + uniform_i32(blockIdx.x * kWaves + wv); w < hi; w += W) {
        const int gi = queue[w];
        const int p = batch_problem(item_base, B, gi);
        const BProb &P = probs[p];
        const RefOut R = batch_out(P, pairs, nullptr, MODE_EMIT);
        const int it = uniform_i32(gi - (int)item_base[p]);
        mask_item<false>(P.G, R, P.masks, it, stage + 256 * wv, slot + 4 * kSlot * wv);
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

__global__ void k_batch_reset(DevCounters *ctr) { *ctr = DevCounters{}; }

DevGrid dev_grid(const Grid &g) {
    DevGrid G;
    G.xs = g.xs;
    G.xa = g.xa;
    G.nrm = g.nrm;
    G.pn = g.pn;
    G.perm = g.perm;
    G.ranges = g.ranges;
    G.items = g.item;
    G.n = g.n;
    G.d = g.d;
    G.dp = g.dp;
    G.da = g.da;
    G.nranges = g.nranges;
    G.nitems = (int32_t)g.items;
    G.blocks = g.blocks;
    G.item_base = g.item_base;
    G.nblocks = (int32_t)g.nblocks;
    G.united = g.united ? 1 : 0;
    G.npc = g.npc;
    G.sc = g.npc > 0 ? g.sc : -1;
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

}  // namespace

bool m64_in_range(const Grid &g) { return g.nmax >= 0.0 && g.nmax <= 0x1p1000; }

sj_path effective_path(const Grid &g, sj_path requested) {
    sj_path p = requested;
    if (is_lowp(p) && g.d <= kLpMaxD && !lowp_in_range(g, p))
        p = SJ_FP64_MFMA;
    if (p == SJ_FP64_MFMA && !m64_in_range(g)) p = SJ_FP64_VALU;
    return p;
}

namespace {

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
    // count of every item, 2 to 4 K-steps, united block items: LDS-shared tiles
    if (is_count(MODE) && g.united && g.nblocks > 0 && ks >= 2 && ks <= 4 && R.item_lo == 0 &&
        nitems == (int)g.items) {
        const unsigned nb = (unsigned)g.nblocks;
#define SJ_M64S(KSV, SL) hipLaunchKernelGGL((k_m64s<KSV, SL, MODE == MODE_SYM>), dim3(nb), dim3(kThreads), 0, s, G, R, delta, (int)nb)
        if (slot) {
            if (ks == 2) SJ_M64S(2, true);
            else if (ks == 3) SJ_M64S(3, true);
            else SJ_M64S(4, true);
        } else {
            if (ks == 2) SJ_M64S(2, false);
            else if (ks == 3) SJ_M64S(3, false);
            else SJ_M64S(4, false);
        }
#undef SJ_M64S
        SJ_HIP(hipGetLastError());
        return;
    }
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
            case 6: SJ_M64(6, false); break;
            case 8: SJ_M64(8, false); break;
            case 12: SJ_M64(12, false); break;
            case 16: SJ_M64(16, false); break;
            default: SJ_M64(0, false); break;
        }
    }
#undef SJ_M64
    SJ_HIP(hipGetLastError());
}

}  // namespace

// Launches of the batched form (see k_batch_m64): sched 0 = a persistent
// grid of the waves the GPU keeps resident for this kernel, 1 = one wave per
// item.
template <typename... P, typename... A>
static void batch_launch(void (*kernel)(P...), int n, int sched, hipStream_t s, A... args) {
    if (n <= 0) return;
    int want = n;
    if (sched == 0) {
        int dev = 0, ncu = 256, per_cu = 0;
        SJ_HIP(hipGetDevice(&dev));
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel), kThreads, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        want = std::min(n, ncu * per_cu * kWaves);
    }
    const unsigned blocks = (unsigned)((want + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kThreads), 0, s, args...);
    SJ_HIP(hipGetLastError());
}

void batch_reset(DevCounters *ctr, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, ctr);
    SJ_HIP(hipGetLastError());
}

template <int MODE>
static void batch_form_mode(const BatchForm &f, sj_path path, const BProb *probs, const int64_t *item_base, int B,
                            const int32_t *queue, int32_t *pairs, DevCounters *ctr, hipStream_t s) {
    const int n = f.hi - f.lo;
    if (path == SJ_FP64_MFMA) {
#define SJ_BM(KSV, SL)                                                                                   \
    batch_launch(k_batch_m64<KSV, SL, MODE>, n, f.sched, s, probs, item_base, B, queue, f.lo, f.hi, pairs, \
                 ctr)
        const bool slot = (f.d & 3) != 0;
        const int da = slot ? ((f.d + 1 + 3) & ~3) : f.d;
        const int ks = da >> 2;
        if (slot) {
            switch (ks) {
                case 1: SJ_BM(1, true); break;
                case 2: SJ_BM(2, true); break;
                case 3: SJ_BM(3, true); break;
                case 4: SJ_BM(4, true); break;
                default: SJ_BM(0, true); break;
            }
        } else {
            switch (ks) {
                case 1: SJ_BM(1, false); break;
                case 2: SJ_BM(2, false); break;
                case 3: SJ_BM(3, false); break;
                case 4: SJ_BM(4, false); break;
                case 6: SJ_BM(6, false); break;
                case 8: SJ_BM(8, false); break;
                case 12: SJ_BM(12, false); break;
                case 16: SJ_BM(16, false); break;
                default: SJ_BM(0, false); break;
            }
        }
#undef SJ_BM
    } else {
#define SJ_BV(DD) \
    batch_launch(k_batch_v64<DD, MODE>, n, f.sched, s, probs, item_base, B, queue, f.lo, f.hi, pairs, ctr)
        switch (f.d) {
            case 1: SJ_BV(1); break;
            case 2: SJ_BV(2); break;
            case 3: SJ_BV(3); break;
            case 4: SJ_BV(4); break;
            case 5: SJ_BV(5); break;
            case 6: SJ_BV(6); break;
            case 7: SJ_BV(7); break;
            case 8: SJ_BV(8); break;
            default: SJ_BV(0); break;
        }
#undef SJ_BV
    }
}

void launch_batch_form(bool emit, bool sym, const BatchForm &f, sj_path path, const BProb *probs,
                       const int64_t *item_base, int B, const int32_t *queue, int32_t *pairs, DevCounters *ctr,
                       hipStream_t s, const int64_t *block_base, const int32_t *bqueue) {
    if (!emit && path == SJ_FP64_MFMA && bqueue && f.bhi > f.blo) {
        const bool slot = (f.d & 3) != 0;
        const int ks = (slot ? ((f.d + 1 + 3) & ~3) : f.d) >> 2;
        const int nb = f.bhi - f.blo;
#define SJ_BS(KSV, SL)                                                                                           \
    sym ? batch_launch(k_batch_m64s<KSV, SL, true>, 4 * nb, f.sched, s, probs, block_base, B, bqueue, f.blo, f.bhi, \
                       ctr)                                                                                      \
        : batch_launch(k_batch_m64s<KSV, SL, false>, 4 * nb, f.sched, s, probs, block_base, B, bqueue, f.blo,    \
                       f.bhi, ctr)
        if (slot) {
            if (ks == 2) SJ_BS(2, true);
            else if (ks == 3) SJ_BS(3, true);
            else SJ_BS(4, true);
        } else {
            if (ks == 2) SJ_BS(2, false);
            else if (ks == 3) SJ_BS(3, false);
            else SJ_BS(4, false);
        }
#undef SJ_BS
        return;
    }
    if (emit) batch_form_mode<MODE_EMIT>(f, path, probs, item_base, B, queue, pairs, ctr, s);
    else if (sym) batch_form_mode<MODE_SYM>(f, path, probs, item_base, B, queue, pairs, ctr, s);
    else batch_form_mode<MODE_COUNT>(f, path, probs, item_base, B, queue, pairs, ctr, s);
}

void launch_batch_zero_counts(const BProb *probs, int B, int64_t max_n, hipStream_t s) {
    if (B <= 0 || max_n <= 0) return;
    const int64_t bx = std::min<int64_t>(1024, (max_n + 4 * kThreads - 1) / (4 * kThreads));
    hipLaunchKernelGGL(k_batch_zero_cnt, dim3((unsigned)bx, (unsigned)std::min(B, 1024)), dim3(kThreads), 0, s, probs,
                       B);
    SJ_HIP(hipGetLastError());
}

void launch_batch_emit(const BProb *probs, const int64_t *item_base, int B, const int32_t *queue, int total,
                       int sched, int32_t *pairs, hipStream_t s) {
    batch_launch(k_batch_emit, total, sched, s, probs, item_base, B, queue, 0, total, pairs);
}

DevGrid make_dev_grid(const Grid &g) { return dev_grid(g); }
double fp64_mfma_delta(const Grid &g) { return m64_delta(g); }

void launch_seg_scan(const BProb *probs, int B, int64_t *totals, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_seg_scan, dim3(B), dim3(kThreads), 0, s, probs, totals);
    SJ_HIP(hipGetLastError());
}

HostCounters read_counters(const DevCounters &c) {
    HostCounters h;
    h.rechecked = (int64_t)c.rechecked;
    h.rechecked_in = (int64_t)c.rechecked_in;
    h.pruned = (int64_t)c.pruned;
    h.violations = (int64_t)c.violations;
    std::memcpy(&h.max_delta, &c.max_delta, sizeof(double));
    std::memcpy(&h.max_err, &c.max_err, sizeof(double));
    return h;
}

namespace {

// Candidate pairs a half-stencil count evaluates: per item, its ranges cut
// at its first query, times its queries (grid-stride over item x range; one
// atomic per block: same-address atomics serialise).
__global__ __launch_bounds__(kThreads) void k_sym_cand(DevGrid G, unsigned long long *out) {
    __shared__ unsigned long long part[kWaves];
    unsigned long long acc = 0;
    const int64_t total = (int64_t)G.nitems * G.nranges;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t it = t / G.nranges;
        const Item I = G.items[it];
        const Range r = G.ranges[t];
        const int32_t b = max(r.begin, I.qbegin);
        if (r.end > b) acc += (unsigned long long)(I.qend - I.qbegin) * (unsigned long long)(r.end - b);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < kWaves; ++w) sum += part[w];
        if (sum) atomicAdd(out, sum);
    }
}

}  // namespace

void launch_sym_cand(const Grid &g, unsigned long long *acc, hipStream_t s) {
    if (g.items <= 0) return;
    hipLaunchKernelGGL(k_sym_cand, dim3(64), dim3(kThreads), 0, s, dev_grid(g), acc);
    SJ_HIP(hipGetLastError());
}

// Enqueues the count kernel of `path` (already range-checked); its counters
// land in ro.ctr (device, zeroed here), read back by the caller with the
// total.
void refine_count(Grid &g, sj_path path, int32_t *cnt_sorted, RefineOut &ro, hipStream_t s) {
    fill_zero(ro.ctr, sizeof(DevCounters), s);
    RefOut R{};
    R.cnt = cnt_sorted;
    R.ctr = ro.ctr;
    R.item_lo = 0;
    R.masks = ro.masks;
    const bool sym = ro.sym && (path == SJ_FP64_VALU || path == SJ_FP64_MFMA);
    ro.cand_eval = g.cand_items;
    if (sym) launch_sym_cand(g, &ro.ctr->spare[0], s);
    if (path == SJ_FP64_VALU) {
        ro.kt.start(ro.timed, s);
        if (sym) launch_v64<MODE_SYM>(g, R, (int)g.items, s);
        else launch_v64<MODE_COUNT>(g, R, (int)g.items, s);
        ro.kt.stop(s);
        ro.band_rel = 0.0;
    } else if (path == SJ_FP64_MFMA) {
        const double delta = m64_delta(g);
        ro.kt.start(ro.timed, s);
        if (sym) launch_m64<MODE_SYM>(g, R, (int)g.items, delta, s);
        else launch_m64<MODE_COUNT>(g, R, (int)g.items, delta, s);
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
    fill_zero(ro.ctr, sizeof(DevCounters), s);
    R.ctr = ro.ctr;
    const int nitems = (int)(p.item_hi - p.item_lo);
    if ((path == SJ_FP64_VALU || path == SJ_FP64_MFMA) && g.masks_valid && g.masks) {
        ro.kt.start(ro.timed, s);
        const unsigned blocks = (unsigned)((nitems + kWaves - 1) / kWaves);
        if (blocks) {
            if (R.d2)
                hipLaunchKernelGGL(k_mask_emit<true>, dim3(blocks), dim3(kThreads), 0, s, dev_grid(g), R,
                                   (const unsigned long long *)g.masks);
            else
                hipLaunchKernelGGL(k_mask_emit<false>, dim3(blocks), dim3(kThreads), 0, s, dev_grid(g), R,
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
    if (path == SJ_FP64_VALU) {
        // the direct form is the exact chain: no band, no error
        *max_err = 0.0;
        *max_band = 0.0;
        *viol = 0;
        return;
    }
    if (path != SJ_FP64_MFMA) {
        lowp_measure(g, path, max_err, max_band, viol, s);
        return;
    }
    DevCounters *ctr = dev_alloc_n<DevCounters>(1, s);
    fill_zero(ctr, sizeof(DevCounters), s);
    RefOut R{};
    R.ctr = ctr;
    R.item_lo = 0;
    const double delta = m64_delta(g);
    launch_m64<MODE_MEASURE>(g, R, (int)g.items, delta, s);
    DevCounters h{};
    SJ_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    dev_free(ctr, s);
    const HostCounters hc = read_counters(h);
    *max_err = hc.max_err;
    *max_band = delta;
    *viol = hc.violations;
}

}  // namespace sj

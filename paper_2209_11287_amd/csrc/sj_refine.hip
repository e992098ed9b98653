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

namespace sj {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

typedef double double4_t __attribute__((ext_vector_type(4)));

struct DevGrid {
    const double *xs;
    const double *xa;
    const double *nrm;
    const int32_t *perm;
    const Range *ranges;
    const Item *items;
    int64_t n;
    int32_t d, dp, da, nranges;
    int32_t nitems;
    double eps2;
};

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

// --------------------------------------------------------------------- V64 --
// Candidate coordinates of one lane, D known at compile time (0 = runtime d,
// read from memory per dimension).
template <int D, int MODE>
__global__ __launch_bounds__(kThreads) void k_v64(DevGrid G, RefOut R) {
    const int lane = threadIdx.x & 63;
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int d = D > 0 ? D : G.d;
    const int dp = G.dp;
    const double eps2 = G.eps2;
    const double *__restrict__ xs = G.xs;

    int cnt[kTileQ];
#pragma unroll
    for (int jq = 0; jq < kTileQ; ++jq) cnt[jq] = 0;
    // emit state of query `lane` (lanes < nq): output window and cursor
    int64_t my_pbase = -1, my_pend = 0;
    int my_cur = 0;
    if (MODE == MODE_EMIT && lane < nq && q0 + lane >= R.qlo && q0 + lane < R.qhi) {
        my_pbase = R.off[q0 + lane] - R.base;
        my_pend = R.off[q0 + lane + 1] - R.base;
    }
    const unsigned long long lt = lanemask_lt();
    for (int o = 0; o < G.nranges; ++o) {
        const int cb = uniform_i32(G.ranges[(int64_t)I.cell_first * G.nranges + o].begin);
        const int ce = uniform_i32(G.ranges[(int64_t)I.cell_last * G.nranges + o].end);
        for (int t = cb; t < ce; t += 64) {
            const int c = t + lane;  // < n + 64: rows are padded
            const bool valid = c < ce;
            const double *__restrict__ xc = xs + (int64_t)c * dp;
            double x[D > 0 ? D : 1];
            if (D > 0) {
#pragma unroll
                for (int u = 0; u < (D > 0 ? D : 1); ++u) x[u] = xc[u];
            }
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
                    } else if (MODE == MODE_EMIT) {
                        const unsigned long long m = __ballot(in);
                        const int64_t pb = readlane_i64(my_pbase, jq);
                        if (pb >= 0) {
                            const int64_t pos = pb + __builtin_amdgcn_readlane(my_cur, jq) + __popcll(m & lt);
                            if (in && pos < readlane_i64(my_pend, jq)) {
                                R.pairs[2 * pos] = G.perm[q0 + jq];
                                R.pairs[2 * pos + 1] = G.perm[c];
                                if (R.d2) R.d2[pos] = acc;
                            }
                            if (lane == jq) my_cur += __popcll(m);
                        }
                    }
                }
            }
        }
    }
    if (MODE == MODE_COUNT) {
#pragma unroll
        for (int jq = 0; jq < kTileQ; ++jq) {
            int v = cnt[jq];
            for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
            if (lane == 0 && jq < nq) R.cnt[q0 + jq] = v;
        }
    }
}

// --------------------------------------------------------------------- M64 --
// KS = K-steps of 4 dimensions (0 = runtime, read per step), SLOT = the
// candidate norm occupies xa slot d (d % 4 != 0).
template <int KS, bool SLOT, int MODE>
__global__ __launch_bounds__(kThreads) void k_m64(DevGrid G, RefOut R, double delta) {
    const int lane = threadIdx.x & 63;
    const int wv = uniform_i32(threadIdx.x >> 6);
    const int it = uniform_i32(R.item_lo + xcd_block(blockIdx.x, gridDim.x) * kWaves + wv);
    if (it >= G.nitems) return;
    const Item I = G.items[it];
    const int q0 = uniform_i32(I.qbegin);
    const int nq = uniform_i32(I.qend - I.qbegin);
    const int d = G.d, da = G.da, dp = G.dp;
    const int ks = KS > 0 ? KS : (da >> 2);
    const int j = lane & 15;   // query column
    const int g = lane >> 4;   // K index of the operands; row group of the result
    const bool qvalid = j < nq;
    const int qj = q0 + (qvalid ? j : 0);
    const double *__restrict__ xa = G.xa;
    const double *__restrict__ xs = G.xs;

    // B operand (K x 16): B[k][j] = -2 q_j[k] for k < d, 1 in the norm slot.
    double bq[KS > 0 ? KS : 1];
    if (KS > 0) {
#pragma unroll
        for (int s = 0; s < (KS > 0 ? KS : 1); ++s) {
            const int kk = 4 * s + g;
            bq[s] = kk < d ? -2.0 * xa[(int64_t)qj * da + kk] : ((SLOT && kk == d) ? 1.0 : 0.0);
        }
    }
    const double thr = G.eps2 - G.nrm[qj];
    const double lo = thr - delta, hi = thr + delta;

    int64_t pbase = -1, pend = 0;
    if (MODE == MODE_EMIT && qvalid && qj >= R.qlo && qj < R.qhi) {
        pbase = R.off[qj] - R.base;
        pend = R.off[qj + 1] - R.base;
    }
    const int32_t pq = MODE == MODE_EMIT ? G.perm[qj] : 0;
    int64_t cur = 0;
    int cnt = 0;
    unsigned long long band = 0, viol = 0;
    double maxerr = 0.0;

    for (int o = 0; o < G.nranges; ++o) {
        const int cb = uniform_i32(G.ranges[(int64_t)I.cell_first * G.nranges + o].begin);
        const int ce = uniform_i32(G.ranges[(int64_t)I.cell_last * G.nranges + o].end);
        for (int t = cb; t < ce; t += 16) {
            double4_t acc;
            if (SLOT) {
                acc = (double4_t){0.0, 0.0, 0.0, 0.0};
            } else {
                const double *nr = G.nrm + t + g;
                acc = (double4_t){nr[0], nr[4], nr[8], nr[12]};
            }
            const double *__restrict__ arow = xa + (int64_t)(t + j) * da + g;
            if (KS > 0) {
#pragma unroll
                for (int s = 0; s < (KS > 0 ? KS : 1); ++s)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[4 * s], bq[s], acc, 0, 0, 0);
            } else {
                for (int s = 0; s < ks; ++s) {
                    const int kk = 4 * s + g;
                    const double b = kk < d ? -2.0 * xa[(int64_t)qj * da + kk]
                                            : ((SLOT && kk == d) ? 1.0 : 0.0);
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[4 * s], b, acc, 0, 0, 0);
                }
            }
            // Result layout of v_mfma_f64_16x16x4f64: register r of lane
            // (g, j) holds row g + 4r, column j. Element r is candidate
            // t + g + 4r against query j.
            const int rowlim = ce - t;
            unsigned inm = 0, bandm = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool valid = qvalid && (g + 4 * r) < rowlim;
                const double v = acc[r];
                if (valid && v <= lo) inm |= 1u << r;
                else if (valid && v <= hi) bandm |= 1u << r;
                if (MODE == MODE_MEASURE && valid) {
                    const double ex = exact_d2(xs + (int64_t)qj * dp, xs + (int64_t)(t + g + 4 * r) * dp, d);
                    if (ex <= 4.0 * G.eps2) {
                        const double err = fabs(v - (ex - G.nrm[qj]));
                        maxerr = fmax(maxerr, err);
                        if (err > delta) ++viol;
                    }
                }
            }
            if (__any(bandm != 0)) {
                // rare: exact FP64 chain on the original coordinates
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (bandm & (1u << r)) {
                        const double ex = exact_d2(xs + (int64_t)qj * dp, xs + (int64_t)(t + g + 4 * r) * dp, d);
                        if (ex <= G.eps2) inm |= 1u << r;
                        ++band;
                    }
                }
            }
            cnt += __popc(inm);
            if (MODE == MODE_EMIT) {
                // candidate order per query: row i = g + 4r, so the rank of
                // (g, r) counts every flagged row of lower level r, then the
                // flagged rows of level r in lower lane groups.
                const unsigned long long sel = 0x0001000100010001ull << j;
                const unsigned long long below = (1ull << (16 * g)) - 1ull;
                int rank_base = 0;
                int rank[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned long long x = __ballot((inm >> r) & 1u) & sel;
                    rank[r] = rank_base + __popcll(x & below);
                    rank_base += __popcll(x);
                }
                if (pbase >= 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t pos = pbase + cur + rank[r];
                        if (((inm >> r) & 1u) && pos < pend) {
                            const int cand = t + g + 4 * r;
                            R.pairs[2 * pos] = pq;
                            R.pairs[2 * pos + 1] = G.perm[cand];
                            if (R.d2) R.d2[pos] = exact_d2(xs + (int64_t)qj * dp, xs + (int64_t)cand * dp, d);
                        }
                    }
                }
                cur += rank_base;
            }
        }
    }
    if (MODE == MODE_COUNT) {
        cnt += __shfl_xor(cnt, 16);
        cnt += __shfl_xor(cnt, 32);
        if (g == 0 && qvalid) R.cnt[qj] = cnt;
    }
    if (MODE != MODE_MEASURE) {
        for (int s = 32; s > 0; s >>= 1) band += __shfl_xor(band, s);
        if (lane == 0 && band) atomicAdd(R.band, band);
    } else {
        for (int s = 32; s > 0; s >>= 1) {
            viol += __shfl_xor(viol, s);
            maxerr = fmax(maxerr, __shfl_xor(maxerr, s));
        }
        if (lane == 0) {
            atomicMax(&R.meas[0], (unsigned long long)__double_as_longlong(maxerr));
            if (viol) atomicAdd(&R.meas[1], viol);
        }
    }
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

void refine_count(Grid &g, sj_path path, int32_t *cnt_sorted, RefineOut &ro, hipStream_t s) {
    unsigned long long *band = dev_alloc_n<unsigned long long>(1, s);
    fill_zero(band, sizeof(unsigned long long), s);
    RefOut R{};
    R.cnt = cnt_sorted;
    R.band = band;
    R.item_lo = 0;
    ro.cand_eval = g.cand_items;
    KernelTimer kt;
    if (path == SJ_FP64_VALU) {
        kt.start(ro.timed, s);
        launch_v64<MODE_COUNT>(g, R, (int)g.items, s);
        kt.stop(s);
        ro.band_rel = 0.0;
    } else if (path == SJ_FP64_MFMA) {
        const double delta = m64_delta(g);
        kt.start(ro.timed, s);
        launch_m64<MODE_COUNT>(g, R, (int)g.items, delta, s);
        kt.stop(s);
        ro.band_rel = g.eps2 > 0 ? delta / g.eps2 : 0.0;
    } else {
        dev_free(band, s);
        throw Unsupported{"path not supported by this build"};
    }
    ro.ms_kernel = kt.ms();
    unsigned long long hb = 0;
    SJ_HIP(hipMemcpyAsync(&hb, band, sizeof hb, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    ro.band_pairs = (int64_t)hb;
    dev_free(band, s);
}

namespace {

// Chunk plan (result batching, Section III-B): from `cursor`, the largest run
// of whole queries whose pairs fit in `capacity`, and the work items that
// cover it. One thread; binary searches over the prefix sums and the items.
__global__ void k_chunk_plan(const int64_t *__restrict__ off, const Item *__restrict__ items, int64_t n,
                             int64_t nitems, int64_t cursor, int64_t capacity, int64_t *__restrict__ out) {
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
    out[0] = 0;
    out[1] = off[next] - base;
    out[2] = next;
    out[3] = ilo;
    out[4] = lo;
    out[5] = base;
}

}  // namespace

ChunkPlan plan_chunk(Grid &g, int64_t cursor, int64_t capacity, hipStream_t s) {
    int64_t *d = dev_alloc_n<int64_t>(8, s);
    hipLaunchKernelGGL(k_chunk_plan, dim3(1), dim3(1), 0, s, g.off, g.item, g.n, g.items, cursor, capacity, d);
    SJ_HIP(hipGetLastError());
    int64_t h[8] = {0};
    SJ_HIP(hipMemcpyAsync(h, d, 6 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    dev_free(d, s);
    ChunkPlan p;
    p.too_small = h[0] != 0;
    p.written = h[1];
    p.next = h[2];
    p.item_lo = h[3];
    p.item_hi = h[4];
    p.base = h[5];
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
    unsigned long long *band = dev_alloc_n<unsigned long long>(1, s);
    fill_zero(band, sizeof(unsigned long long), s);
    R.band = band;
    const int nitems = (int)(p.item_hi - p.item_lo);
    KernelTimer kt;
    if (path == SJ_FP64_VALU) {
        kt.start(ro.timed, s);
        launch_v64<MODE_EMIT>(g, R, nitems, s);
        kt.stop(s);
    } else if (path == SJ_FP64_MFMA) {
        const double delta = m64_delta(g);
        kt.start(ro.timed, s);
        launch_m64<MODE_EMIT>(g, R, nitems, delta, s);
        kt.stop(s);
        ro.band_rel = g.eps2 > 0 ? delta / g.eps2 : 0.0;
    } else {
        dev_free(band, s);
        throw Unsupported{"path not supported by this build"};
    }
    dev_free(band, s);
    ro.ms_kernel = kt.ms();
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
        throw Unsupported{"path not supported by this build"};
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

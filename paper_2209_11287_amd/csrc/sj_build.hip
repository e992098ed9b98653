// Grid index build on the GPU: the "search" structure of the self-join
// (Section II-D: a grid is searched for candidates, which are then refined;
// Section III-B: cells of side eps, every query of a cell shares the cell's
// candidate set, so queries must be grouped by cell).
//
// Steps: bounding box -> cell keys -> LSD radix sort (key, index) -> gather of
// sorted rows and squared norms (the precomputed P of Section III-A) -> cell
// table -> grid lines and work items -> per-cell neighbour ranges.
//
// Grid geometry (the paper fixes the cell side only): origin = per-dimension
// minimum, cell side w = eps * (1 + 2^-19) (a pair within eps then never lands
// two cells apart after rounding), k leading dimensions indexed, last indexed
// dimension fastest in the key, so the three cells along it that neighbour a
// cell are contiguous in sorted order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <utility>
#include <vector>

#include "sj_internal.h"

namespace sj {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const unsigned lane = threadIdx.x & 63u;
    return lane ? ((~0ull) >> (64u - lane)) : 0ull;
}

// Order-preserving integer image of a double (for min/max reductions).
__device__ __forceinline__ unsigned long long dbl_to_ord(double v) {
    unsigned long long u = __double_as_longlong(v);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double ord_to_dbl(unsigned long long u) {
    unsigned long long b = (u & 0x8000000000000000ull) ? (u & 0x7fffffffffffffffull) : ~u;
    double r;
    std::memcpy(&r, &b, sizeof r);
    return r;
}

__global__ void k_fill_u8(unsigned char *p, size_t bytes, unsigned char v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < bytes; i += stride) p[i] = v;
}

// Zeroes up to eight segments (4-byte aligned, whole 4-byte words) in one
// launch: the build's small pads and counters.
struct FillList {
    uint32_t *p[8];
    unsigned long long words[8];
    int n;
};

__global__ void k_fill_many(FillList L) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (int k = 0; k < L.n; ++k)
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.words[k]; i += stride) L.p[k][i] = 0u;
}

static void fill_zero_many(std::initializer_list<std::pair<void *, size_t>> segs, hipStream_t s) {
    FillList L{};
    size_t most = 0;
    for (const auto &sg : segs) {
        if (!sg.first || !sg.second) continue;
        L.p[L.n] = static_cast<uint32_t *>(sg.first);
        L.words[L.n] = sg.second / 4;
        most = std::max(most, sg.second / 4);
        ++L.n;
    }
    if (!L.n) return;
    const unsigned blocks = (unsigned)std::min<size_t>((most + kThreads - 1) / kThreads, 1024);
    hipLaunchKernelGGL(k_fill_many, dim3(blocks), dim3(kThreads), 0, s, L);
    SJ_HIP(hipGetLastError());
}

// What the host reads back after the grid build's device work: the table
// sizes, the radix sort's error flag, the largest squared norm and the
// item candidate / tile totals.
struct BuildReadback {
    int32_t c[4];  // ncells, nlines, nitems, nblocks
    int32_t err;
    int32_t pad;
    double nmax;
    unsigned long long acc[3];  // item candidates, tiles, united candidates
};

__global__ void k_build_readback(const int32_t *__restrict__ counters, const int32_t *__restrict__ err,
                                 const double *__restrict__ nmax, const unsigned long long *__restrict__ acc,
                                 BuildReadback *__restrict__ out) {
    BuildReadback r;
    for (int i = 0; i < 4; ++i) r.c[i] = counters[i];
    r.err = *err;
    r.pad = 0;
    r.nmax = *nmax;
    for (int i = 0; i < 3; ++i) r.acc[i] = acc[i];
    *out = r;
}

void fill_ones(void *p, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    unsigned blocks = (unsigned)std::min<size_t>((bytes + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(kThreads), 0, s, (unsigned char *)p, bytes, (unsigned char)0xff);
    SJ_HIP(hipGetLastError());
}


// ---------------------------------------------------------------- bbox ----
// Each block reduces a contiguous run of rows. Threads walk the run's
// elements with a stride that is a multiple of d, so each thread sees a single
// dimension; per-dimension partials then go to memory. MOM: also the sums of
// (x - x_0) and (x - x_0)^2 per dimension (x_0 = the first row's value), for
// the variance order of the filter's dimensions (only an ordering: their
// rounding does not matter).
template <bool MOM>
__global__ void k_bbox_partial(const double *__restrict__ X, int64_t n, int d, int64_t rows_per_block,
                               double *__restrict__ pmin, double *__restrict__ pmax, double *__restrict__ psum,
                               double *__restrict__ psq, int *__restrict__ bad) {
    __shared__ double smin[kThreads], smax[kThreads];
    __shared__ double ssum[MOM ? kThreads : 1], ssq[MOM ? kThreads : 1];
    const int S = (kThreads / d) * d;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    double mn = INFINITY, mx = -INFINITY, s1 = 0.0, s2 = 0.0;
    int nonfinite = 0;
    if (tid < S && r0 < r1) {
        const int64_t e0 = r0 * d, e1 = r1 * d;
        const double x0 = MOM ? X[tid % d] : 0.0;
#pragma unroll 4
        for (int64_t e = e0 + tid; e < e1; e += S) {
            double v = X[e];
            nonfinite |= !isfinite(v);
            mn = fmin(mn, v);
            mx = fmax(mx, v);
            if (MOM) {
                const double c = v - x0;
                s1 += c;
                s2 = fma(c, c, s2);
            }
        }
    }
    smin[tid] = mn;
    smax[tid] = mx;
    if (MOM) {
        ssum[tid] = s1;
        ssq[tid] = s2;
    }
    if (nonfinite) atomicOr(bad, 1);
    __syncthreads();
    if (tid < d) {
        double a = INFINITY, b = -INFINITY, c1 = 0.0, c2 = 0.0;
        for (int t = tid; t < S; t += d) {
            a = fmin(a, smin[t]);
            b = fmax(b, smax[t]);
            if (MOM) {
                c1 += ssum[t];
                c2 += ssq[t];
            }
        }
        pmin[(int64_t)blockIdx.x * d + tid] = a;
        pmax[(int64_t)blockIdx.x * d + tid] = b;
        if (MOM) {
            psum[(int64_t)blockIdx.x * d + tid] = c1;
            psq[(int64_t)blockIdx.x * d + tid] = c2;
        }
    }
}

// One block per dimension j: out[j] = min, out[d + j] = max and, with the
// moments (psum non-null), out[2d + j], out[3d + j] = their sums.
__global__ void k_bbox_final(const double *__restrict__ pmin, const double *__restrict__ pmax,
                             const double *__restrict__ psum, const double *__restrict__ psq, int nb, int d,
                             double *__restrict__ out) {
    __shared__ double smin[kThreads], smax[kThreads], s1[kThreads], s2[kThreads];
    const int j = blockIdx.x;
    double a = INFINITY, b = -INFINITY, c1 = 0.0, c2 = 0.0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) {
        a = fmin(a, pmin[(int64_t)t * d + j]);
        b = fmax(b, pmax[(int64_t)t * d + j]);
        if (psum) {
            c1 += psum[(int64_t)t * d + j];
            c2 += psq[(int64_t)t * d + j];
        }
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    s1[threadIdx.x] = c1;
    s2[threadIdx.x] = c2;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[j] = smin[0];
        out[d + j] = smax[0];
        if (psum) {
            out[2 * d + j] = s1[0];
            out[3 * d + j] = s2[0];
        }
    }
}

// ---------------------------------------------------------------- keys ----
struct KeyGeom {
    int k, d;
    int sb;  // sub-cell bits appended (last indexed dimension)
    double w;
    double lo[kMaxIndexDims];
    int64_t m[kMaxIndexDims];
    int64_t stride[kMaxIndexDims];
};

// Position of t = fl(fl(x - lo) / w) inside cell c in 2^sb steps, clamped
// (monotone in x, like the cell itself).
__device__ __forceinline__ unsigned long long sub_cell(double t, int64_t c, int sb) {
    if (sb == 0) return 0;
    const double f = floor((t - (double)c) * (double)(1ull << sb));
    const double top = (double)((1ull << sb) - 1);
    return (unsigned long long)(f < 0.0 ? 0.0 : (f > top ? top : f));
}

// ----------------------------------------------------------- radix sort ----
// Stable LSD radix sort of (64-bit key, int32 value), 8-bit digits. Each
// block owns a tile of kThreads * kRsItems keys. Pass = per-tile digit
// histogram -> exclusive scan in digit-major order -> stable scatter where a
// key's rank inside its tile comes from a wave-wide match of its digit (eight
// ballots) plus per-wave digit counts combined in LDS.
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;

__global__ void k_rs_hist(const unsigned long long *__restrict__ key, int64_t n, int shift,
                          int32_t *__restrict__ hist, int nblocks) {
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_rs_scatter(const unsigned long long *__restrict__ kin, const int32_t *__restrict__ vin,
                             unsigned long long *__restrict__ kout, int32_t *__restrict__ vout,
                             int64_t n, int shift, const int32_t *__restrict__ hist_ex, int nblocks) {
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[kThreads / 64][256];
    __shared__ int32_t wpre[kThreads / 64][256];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    run[tid] = hist_ex[(int64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kRsTile;
    const unsigned long long lt = lanemask_lt();
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + tid;
        const bool valid = i < n;
        unsigned long long kk = 0;
        int32_t vv = 0;
        unsigned digit = 0;
        if (valid) {
            kk = kin[i];
            vv = vin[i];
            digit = (unsigned)((kk >> shift) & 255u);
        }
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][digit] = __popcll(peers);
        __syncthreads();
        {
            int32_t acc = run[tid];
            for (int w = 0; w < kThreads / 64; ++w) {
                wpre[w][tid] = acc;
                acc += wcnt[w][tid];
                wcnt[w][tid] = 0;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const int32_t pos = wpre[wave][digit] + rank;
            kout[pos] = kk;
            vout[pos] = vv;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ one-sweep sort ----
// The build's sort of (cell key, point index): LSD radix sort, 8-bit digits,
// one launch per digit. The key kernel also counts every digit of every key
// (all passes' digit histograms in one read). A pass kernel takes one tile
// of kOsTile keys (tile numbers handed out in launch order by a counter, so
// every tile's predecessors have started), ranks its keys stably by digit
// (wave-wide digit match, as in k_rs_scatter), publishes its per-digit counts
// and finds the counts of all tiles before it by looking back over their
// published words (decoupled look-back; each word = flag + count, read and
// written as one 64-bit atomic). The tile's keys are reordered by digit in
// LDS first, so the stores of one digit's run are contiguous.
// Keys of at most 32 bits travel packed with their index in one 64-bit word
// (key in the high half); the last pass then writes the key and the index
// to separate arrays. Wider keys travel as (64-bit key, 32-bit index).
// A look-back that does not see its predecessor's word after kOsSpin polls
// sets *err (the host reports it) instead of waiting on; with tile numbers
// handed out in order it cannot happen.
constexpr int kOsItems = 16;
constexpr int kOsTile = kThreads * kOsItems;
constexpr int kOsMaxPasses = 8;
constexpr unsigned long long kOsAgg = 1ull << 32;     // word flag: the tile's own count
constexpr unsigned long long kOsIncl = 2ull << 32;    // word flag: count of this tile and all before it
constexpr int kOsSpin = 1 << 16;

enum { OS_PACKED = 0, OS_PACKED_SPLIT = 1, OS_WIDE = 2 };

// Cell keys plus the digit histograms of every sort pass. Key of point i:
// c_j = floor(fl(fl(x_j - lo_j) / w)) clamped to [0, m_j - 1] (the same two
// roundings as the reference grid definition; clamped in double before the
// conversion, so an infinite quotient converts to nothing out of range),
// key = sum c_j stride_j, followed by sb sub-cell bits (the position inside
// the cell along the last indexed dimension). hist[p][v] = keys whose digit p
// is v (p < passes). PACKED: out[i] = key << 32 | i.
template <bool PACKED>
__global__ __launch_bounds__(kThreads) void k_keys_hist(const double *__restrict__ X, int64_t n, KeyGeom geo,
                                                        unsigned long long *__restrict__ key,
                                                        int32_t *__restrict__ idx, int passes,
                                                        int32_t *__restrict__ hist) {
    __shared__ int32_t h[kOsMaxPasses * 256];
    for (int t = threadIdx.x; t < passes * 256; t += kThreads) h[t] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long kk = 0, sub = 0;
        for (int j = 0; j < geo.k; ++j) {
            const double t = __ddiv_rn(__dsub_rn(X[i * geo.d + j], geo.lo[j]), geo.w);
            double q = floor(t);
            q = !(q >= 0.0) ? 0.0 : (q > (double)(geo.m[j] - 1) ? (double)(geo.m[j] - 1) : q);
            const int64_t c = (int64_t)q;
            kk += (unsigned long long)c * (unsigned long long)geo.stride[j];
            if (j == geo.k - 1) sub = sub_cell(t, c, geo.sb);
        }
        const unsigned long long full = (kk << geo.sb) | sub;
        if (PACKED) {
            key[i] = (full << 32) | (unsigned long long)(uint32_t)i;
        } else {
            key[i] = full;
            idx[i] = (int32_t)i;
        }
        for (int p = 0; p < passes; ++p) atomicAdd(&h[p * 256 + (int)((full >> (8 * p)) & 255u)], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < passes * 256; t += kThreads)
        if (h[t]) atomicAdd(&hist[t], h[t]);
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_onesweep(const unsigned long long *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       unsigned long long *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t n, int shift,
                                                       const int32_t *__restrict__ hist,
                                                       unsigned long long *__restrict__ status,
                                                       int32_t *__restrict__ tile_ctr, int32_t *__restrict__ err) {
    __shared__ unsigned long long skey[kOsTile];
    __shared__ int32_t sval[MODE == OS_WIDE ? kOsTile : 1];
    __shared__ int32_t dcnt[256];   // the tile's keys per digit
    __shared__ int32_t dexc[256];   // their exclusive prefix: first LDS slot of each digit
    __shared__ int32_t gbase[256];  // first output position of the tile's keys of each digit
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[kThreads / 64][256];
    __shared__ int32_t wpre[kThreads / 64][256];
    __shared__ int32_t wsum[kThreads / 64];
    __shared__ int32_t tile_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int dshift = (MODE == OS_WIDE ? 0 : 32) + shift;
    if (tid == 0) tile_sh = atomicAdd(tile_ctr, 1);
    dcnt[tid] = 0;
    run[tid] = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int tile = tile_sh;
    const int64_t t0 = (int64_t)tile * kOsTile;
    // the tile's keys, all loads in flight together
    unsigned long long kk[kOsItems];
    int32_t vv[kOsItems];
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + tid;
        kk[r] = i < n ? kin[i] : 0ull;
        if (MODE == OS_WIDE) vv[r] = i < n ? vin[i] : 0;
    }
    // digit counts of the tile
#pragma unroll
    for (int r = 0; r < kOsItems; ++r)
        if (t0 + (int64_t)r * kThreads + tid < n) atomicAdd(&dcnt[(int)((kk[r] >> dshift) & 255u)], 1);
    __syncthreads();
    // publish them at once (the first tile publishes its inclusive count)
    const int agg = dcnt[tid];
    __hip_atomic_store(&status[(int64_t)tile * 256 + tid],
                       (tile == 0 ? kOsIncl : kOsAgg) | (unsigned long long)(uint32_t)agg, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    // exclusive prefix of the counts over digits (LDS slots) and of the
    // pass's histogram (the digit's first output position)
    {
        int x = agg, y = hist[tid];
        int xi = x, yi = y;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int a = __shfl_up(xi, o), b = __shfl_up(yi, o);
            if (lane >= o) {
                xi += a;
                yi += b;
            }
        }
        if (lane == 63) wsum[wave] = xi;
        __syncthreads();
        int xo = 0;
        for (int w = 0; w < wave; ++w) xo += wsum[w];
        __syncthreads();
        if (lane == 63) wsum[wave] = yi;
        __syncthreads();
        int yo = 0;
        for (int w = 0; w < wave; ++w) yo += wsum[w];
        dexc[tid] = xo + xi - x;
        gbase[tid] = yo + yi - y;  // completed by the look-back below
    }
    __syncthreads();
    // stable ranks, round by round (round r = keys t0 + 256 r ..): digit match
    // within the wave, per-wave counts combined per digit in LDS
    const unsigned long long lt = lane ? ((~0ull) >> (64u - (unsigned)lane)) : 0ull;
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const bool valid = t0 + (int64_t)r * kThreads + tid < n;
        const unsigned digit = valid ? (unsigned)((kk[r] >> dshift) & 255u) : 0u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (digit >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][digit] = __popcll(peers);
        __syncthreads();
        {
            int acc = run[tid];
#pragma unroll
            for (int w = 0; w < kThreads / 64; ++w) {
                wpre[w][tid] = acc;
                acc += wcnt[w][tid];
                wcnt[w][tid] = 0;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const int slot = dexc[digit] + wpre[wave][digit] + rank;
            skey[slot] = kk[r];
            if (MODE == OS_WIDE) sval[slot] = vv[r];
        }
    }
    // look back over the earlier tiles' words of this thread's digit
    if (tile > 0) {
        int excl = 0, spins = 0;
        for (int k = tile - 1; k >= 0;) {
            const unsigned long long w =
                __hip_atomic_load(&status[(int64_t)k * 256 + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long f = w & ~0xffffffffull;
            if (f == 0ull) {
                if (++spins > kOsSpin) {
                    atomicOr(err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += (int)(uint32_t)w;
            if (f == kOsIncl) break;
            --k;
        }
        __hip_atomic_store(&status[(int64_t)tile * 256 + tid], kOsIncl | (unsigned long long)(uint32_t)(excl + agg),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        gbase[tid] += excl;
    }
    __syncthreads();
    // stores in LDS order: each digit's run of the tile is contiguous
    const int cnt = (int)min<int64_t>(kOsTile, n - t0);
#pragma unroll
    for (int r = 0; r < kOsItems; ++r) {
        const int sidx = r * kThreads + tid;
        if (sidx < cnt) {
            const unsigned long long k = skey[sidx];
            const int d = (int)((k >> dshift) & 255u);
            const int64_t pos = (int64_t)gbase[d] + (sidx - dexc[d]);
            if (MODE == OS_PACKED) {
                kout[pos] = k;
            } else if (MODE == OS_PACKED_SPLIT) {
                kout[pos] = k >> 32;
                vout[pos] = (int32_t)(uint32_t)k;
            } else {
                kout[pos] = k;
                vout[pos] = sval[sidx];
            }
        }
    }
}

// ---------------------------------------------------------------- scans ----
// Exclusive scan, three phases: per-tile sums, scan of the tile sums
// (recursively), per-tile scan plus carry. Tile = kThreads * kScanItems.
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

template <typename Tin, typename Tacc>
__global__ void k_scan_sums(const Tin *__restrict__ in, int64_t n, Tacc *__restrict__ sums) {
    __shared__ Tacc part[kThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    Tacc acc = 0;
    if (sizeof(Tin) == 4 && t0 + kScanTile <= n) {
        // whole tile: 16-byte loads, each wave reading 1 KB runs (the tile
        // starts at a 16 KB offset)
        const int4 *p4 = reinterpret_cast<const int4 *>(in + t0);
#pragma unroll
        for (int r = 0; r < kScanItems / 4; ++r) {
            const int4 w = p4[r * kThreads + threadIdx.x];
            acc += (Tacc)w.x + (Tacc)w.y + (Tacc)w.z + (Tacc)w.w;
        }
    } else {
        for (int r = 0; r < kScanItems; ++r) {
            int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
            if (i < n) acc += (Tacc)in[i];
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        Tacc s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += part[w];
        sums[blockIdx.x] = s;
    }
}

// Exclusive scan of one tile with a carry-in: carry[tile] (scanned tile
// sums), or the sum of sums[0 .. tile) taken here (raw tile sums), or none.
// Each thread scans kScanItems consecutive elements, the thread totals are
// scanned across the wave and the block.
template <typename Tin, typename Tacc>
__global__ void k_scan_tiles(const Tin *__restrict__ in, Tacc *__restrict__ out, int64_t n,
                             const Tacc *__restrict__ carry, const Tacc *__restrict__ sums) {
    __shared__ Tacc wsum[kThreads / 64];
    __shared__ Tacc csum[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    Tacc c = 0;
    if (!carry && sums) {
        for (int64_t t = tid; t < (int64_t)blockIdx.x; t += kThreads) c += sums[t];
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
        if (lane == 0) csum[wave] = c;
    }
    const int64_t e0 = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    Tacc v[kScanItems];
    Tacc sum = 0;
    const bool full = e0 + kScanItems <= n;
    if (full && sizeof(Tin) == 4) {
        // whole run of 16: four 16-byte loads (the run starts at a 64-byte offset)
        const int4 *p4 = reinterpret_cast<const int4 *>(in + e0);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const int4 w = p4[q];
            v[4 * q] = (Tacc)w.x;
            v[4 * q + 1] = (Tacc)w.y;
            v[4 * q + 2] = (Tacc)w.z;
            v[4 * q + 3] = (Tacc)w.w;
        }
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) sum += v[i];
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = e0 + i < n ? (Tacc)in[e0 + i] : (Tacc)0;
            sum += v[i];
        }
    }
    Tacc x = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const Tacc y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    Tacc pre = 0;
    if (carry) pre = carry[blockIdx.x];
    else if (sums)
        for (int w = 0; w < kThreads / 64; ++w) pre += csum[w];
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    Tacc run = pre + x - sum;
    if (full && sizeof(Tacc) == 4) {
        int4 *o4 = reinterpret_cast<int4 *>(out + e0);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            int4 w;
            w.x = (int)run;
            run += v[4 * q];
            w.y = (int)run;
            run += v[4 * q + 1];
            w.z = (int)run;
            run += v[4 * q + 2];
            w.w = (int)run;
            run += v[4 * q + 3];
            o4[q] = w;
        }
    } else if (full && sizeof(Tacc) == 8) {
        longlong2 *o2 = reinterpret_cast<longlong2 *>(out + e0);
#pragma unroll
        for (int q = 0; q < kScanItems / 2; ++q) {
            longlong2 w;
            w.x = (long long)run;
            run += v[2 * q];
            w.y = (long long)run;
            run += v[2 * q + 1];
            o2[q] = w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (e0 + i < n) out[e0 + i] = run;
            run += v[i];
        }
    }
}

template <typename Tin, typename Tacc>
void exclusive_scan(const Tin *in, Tacc *out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        hipLaunchKernelGGL((k_scan_tiles<Tin, Tacc>), dim3(1), dim3(kThreads), 0, s, in, out, n,
                           (const Tacc *)nullptr, (const Tacc *)nullptr);
        SJ_HIP(hipGetLastError());
        return;
    }
    if (tiles <= 8192) {  // two launches: tile sums, then tiles that add up the sums before them
        Tacc *sums = dev_alloc_n<Tacc>(tiles, s);
        hipLaunchKernelGGL((k_scan_sums<Tin, Tacc>), dim3((unsigned)tiles), dim3(kThreads), 0, s, in, n, sums);
        SJ_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_scan_tiles<Tin, Tacc>), dim3((unsigned)tiles), dim3(kThreads), 0, s, in, out, n,
                           (const Tacc *)nullptr, (const Tacc *)sums);
        SJ_HIP(hipGetLastError());
        dev_free(sums, s);
        return;
    }
    Tacc *sums = dev_alloc_n<Tacc>(tiles, s);
    Tacc *sums_ex = dev_alloc_n<Tacc>(tiles, s);
    hipLaunchKernelGGL((k_scan_sums<Tin, Tacc>), dim3((unsigned)tiles), dim3(kThreads), 0, s, in, n, sums);
    SJ_HIP(hipGetLastError());
    exclusive_scan<Tacc, Tacc>(sums, sums_ex, tiles, s);
    hipLaunchKernelGGL((k_scan_tiles<Tin, Tacc>), dim3((unsigned)tiles), dim3(kThreads), 0, s, in, out, n,
                       (const Tacc *)sums_ex, (const Tacc *)nullptr);
    SJ_HIP(hipGetLastError());
    dev_free(sums, s);
    dev_free(sums_ex, s);
}

// ---------------------------------------------------------- gather/norms ----
// Sorted copies: xs = original rows (stride dp, zero padded), xa = rows
// centred on `mid` (stride da); nrm = squared norm of the xa row, the FP64
// chain over dimensions in order; pn (d > 16, else null) = that chain after
// the first 16 dimensions: the prefix norm of the refine pass's
// partial-distance bound. When d % 4 != 0 the norm also sits in xa's
// slot d, where the MFMA tile multiplies it by 1 (Eq. (4) keeps the norms off
// the tensor cores; here a spare K slot takes them).
// Per-block maximum of non-negative doubles into part[blockIdx.x] (a
// single-address atomic from tens of thousands of blocks serialises).
__device__ __forceinline__ void block_max_out(double v, double *__restrict__ part_out) {
    __shared__ double part[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = part[0];
        for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, part[w]);
        part_out[blockIdx.x] = m;
    }
}

// One block: maximum of `nb` partials into *out.
__global__ void k_max_final(const double *__restrict__ part, int64_t nb, double *__restrict__ out) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) v = fmax(v, part[i]);
    __shared__ double red[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, red[w]);
        *out = m;
    }
}

struct GatherArgs {
    int d, dp, da;
    int npc;                 // prefix norms per row (0: none)
    uint8_t fo[kMaxDims];    // column t of xa holds input dimension fo[t]
    double mid[kMaxDims];
};

// Sorted rows (xs, input order), centred rows in the tile order (xa: column
// t = input dimension fo[t] minus its centre; slot d = the norm when d % 4 !=
// 0), norms and the prefix norms over the first 4s columns, s = 1 .. npc
// (the same FP64 chain, stopped at each K-step boundary).
__global__ void k_gather(const double *__restrict__ X, const int32_t *__restrict__ perm, int64_t n,
                         const GatherArgs ga_v, double *__restrict__ xs,
                         double *__restrict__ xa, double *__restrict__ nrm, double *__restrict__ pn,
                         double *__restrict__ nmax_part) {
    const GatherArgs *ga = &ga_v;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double nn = 0.0;
    if (i < n) {
        const int d = ga->d, dp = ga->dp, da = ga->da, npc = ga->npc;
        const double *src = X + (int64_t)perm[i] * d;
        double *ps = xs + i * dp;
        double *pa = xa + i * da;
        for (int t = 0; t < d; ++t) ps[t] = src[t];
        for (int t = 0; t < d; ++t) {
            const int u = ga->fo[t];
            const double c = __dsub_rn(src[u], ga->mid[u]);
            pa[t] = c;
            nn = __fma_rn(c, c, nn);
            if ((t & 3) == 3 && (t >> 2) < npc) pn[i * npc + (t >> 2)] = nn;
        }
        for (int t = d; t < dp; ++t) ps[t] = 0.0;
        for (int t = d; t < da; ++t) pa[t] = 0.0;
        if (d & 3) pa[d] = nn;
        nrm[i] = nn;
    }
    block_max_out(nn, nmax_part);
}

// The same rows, norms and prefix norms as k_gather (the same FP64
// operations in the same order, so the same bits) for 16 <= d <= 64, with
// every row read and written whole by one wave instruction: one wave per
// block, 32 rows per block staged in LDS. Lane t handles column t of a row
// (raw value, then the centred value of input dimension fo[t]); the norm
// chain runs per row in one lane over the staged columns in order, and the
// prefix norms leave through LDS as whole rows too. With fewer dimensions a
// row per lane (k_gather) needs far fewer memory instructions for the same
// bytes.
constexpr int kGatherRows = 32;
constexpr int kGatherLdsD = 64;

__global__ __launch_bounds__(64) void k_gather_lds(const double *__restrict__ X, const int32_t *__restrict__ perm,
                                                   int64_t n, const GatherArgs ga_v, double *__restrict__ xs,
                                                   double *__restrict__ xa, double *__restrict__ nrm,
                                                   double *__restrict__ pn, double *__restrict__ nmax_part) {
    __shared__ double row[kGatherRows][kGatherLdsD + 1];  // +1: a column of the rows falls in distinct banks
    const GatherArgs *ga = &ga_v;
    const int lane = threadIdx.x;
    const int d = ga->d, dp = ga->dp, da = ga->da, npc = ga->npc;
    // this lane's column: its input dimension and centre (uniform loop, no
    // lane-indexed access to the argument block)
    int my_fo = 0;
    double my_mid = 0.0;
    for (int t = 0; t < d; ++t) {
        const int u = ga->fo[t];
        const double m = ga->mid[u];
        if (lane == t) {
            my_fo = u;
            my_mid = m;
        }
    }
    const int64_t i0 = (int64_t)blockIdx.x * kGatherRows;
    const int nr = (int)min<int64_t>(kGatherRows, n - i0);
    // rows in, whole; sorted rows out, whole
    for (int r = 0; r < nr; ++r) {
        const int64_t src = (int64_t)perm[i0 + r] * d;
        const double v = lane < d ? X[src + lane] : 0.0;
        if (lane < d) row[r][lane] = v;
        if (lane < dp) xs[(i0 + r) * dp + lane] = v;  // zero past d
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // centred rows in the tile order, whole (in place: each row's permuted
    // reads complete before its writes; one wave)
    for (int r = 0; r < nr; ++r) {
        const double c = lane < d ? __dsub_rn(row[r][my_fo], my_mid) : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < d) row[r][lane] = c;
        if (lane < da && !((d & 3) && lane == d)) xa[(i0 + r) * da + lane] = c;  // slot d: the norm, below
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the norm chain of row `lane`; prefix norms back into the row's first
    // npc columns (each written after the columns it covers were read)
    double nn = 0.0;
    if (lane < nr) {
        for (int t = 0; t < d; ++t) {
            const double c = row[lane][t];
            nn = __fma_rn(c, c, nn);
            if ((t & 3) == 3 && (t >> 2) < npc) row[lane][t >> 2] = nn;
        }
        nrm[i0 + lane] = nn;
        if (d & 3) xa[(i0 + lane) * da + d] = nn;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (npc > 0)
        for (int r = 0; r < nr; ++r)
            if (lane < npc) pn[(i0 + r) * npc + lane] = row[r][lane];
    double v = nn;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if (lane == 0) nmax_part[blockIdx.x] = v;
}

// d <= 4 (dp = da = 4): four lanes per point, lane t = dimension t, so each
// wave stores 16 whole rows of xs and of xa contiguously. Same values as
// k_gather (the norm chain runs over the dimensions in order in every lane).
struct Mid4 {
    double m[4];
};

__global__ void k_gather4(const double *__restrict__ X, const int32_t *__restrict__ perm, int64_t n, int d,
                          Mid4 mid, double *__restrict__ xs, double *__restrict__ xa, double *__restrict__ nrm,
                          double *__restrict__ nmax_part) {
    const int t = threadIdx.x & 3;
    double mx = 0.0;
    // grid-stride over elements (point e / 4, dimension e % 4); the stride is
    // a multiple of 4, so a lane keeps its dimension
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 4 * ((n + 63) & ~int64_t(63));
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e >> 2;
        double v = 0.0, c = 0.0;
        if (i < n && t < d) {
            v = X[(int64_t)perm[i] * d + t];
            c = __dsub_rn(v, mid.m[t]);
        }
        double cc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cc[u] = __shfl(c, u, 4);
        double nn = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < d) nn = __fma_rn(cc[u], cc[u], nn);
        if (i < n) {
            xs[e] = t < d ? v : 0.0;
            xa[e] = t < d ? c : ((t == d) ? nn : 0.0);
            if (t == 0) nrm[i] = nn;
            mx = fmax(mx, nn);
        }
    }
    block_max_out(mx, nmax_part);
}

// ----------------------------------------------------------- cell table ----
// Sorted keys carry `sb` sub-cell bits below the cell key.
__global__ void k_cell_flags(const unsigned long long *__restrict__ key, int64_t n, int sb,
                             int32_t *__restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (i == 0 || (key[i] >> sb) != (key[i - 1] >> sb)) ? 1 : 0;
}

__global__ void k_cell_write(const unsigned long long *__restrict__ key, int sb, const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ cid, int64_t n, int64_t *__restrict__ cell_key,
                             int32_t *__restrict__ cell_start, int32_t *__restrict__ ncells) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (flag[i]) {
        cell_key[cid[i]] = (int64_t)(key[i] >> sb);
        cell_start[cid[i]] = (int32_t)i;
    }
    if (i == n - 1) {
        const int32_t c = cid[i] + flag[i];
        *ncells = c;
        cell_start[c] = (int32_t)n;
    }
}

// Line of a cell: its key without the last indexed coordinate.
__global__ void k_line_flags(const int64_t *__restrict__ cell_key, const int32_t *__restrict__ ncells_p,
                             int64_t m_last, int32_t *__restrict__ lflag) {
    const int64_t ncells = *ncells_p;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    lflag[c] = (c == 0 || cell_key[c] / m_last != cell_key[c - 1] / m_last) ? 1 : 0;
}

// Per line: first cell, and the number of work items (ceil(points / kTileQ)).
__global__ void k_line_write(const int32_t *__restrict__ lflag, const int32_t *__restrict__ lid,
                             const int32_t *__restrict__ cell_start, const int32_t *__restrict__ ncells_p,
                             int32_t *__restrict__ line_first, int32_t *__restrict__ nlines_p) {
    const int64_t ncells = *ncells_p;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    if (lflag[c]) line_first[lid[c]] = (int32_t)c;
    if (c == ncells - 1) {
        const int32_t L = lid[c] + lflag[c];
        *nlines_p = L;
        line_first[L] = (int32_t)ncells;
    }
}

__global__ void k_line_items(const int32_t *__restrict__ line_first, const int32_t *__restrict__ cell_start,
                             const int32_t *__restrict__ nlines_p, int32_t *__restrict__ nitem) {
    const int64_t L = *nlines_p;
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    const int32_t pts = cell_start[line_first[l + 1]] - cell_start[line_first[l]];
    nitem[l] = (pts + kTileQ - 1) / kTileQ;
}

__global__ void k_items_total(const int32_t *__restrict__ nitem, const int32_t *__restrict__ item_off,
                              const int32_t *__restrict__ nlines_p, int32_t *__restrict__ nitems_p) {
    const int32_t L = *nlines_p;
    *nitems_p = L > 0 ? item_off[L - 1] + nitem[L - 1] : 0;
}

// Largest index p in [a, b) with v[p] <= x (v ascending, v[a] <= x).
__device__ __forceinline__ int32_t last_le(const int32_t *v, int32_t a, int32_t b, int32_t x) {
    while (b - a > 1) {
        const int32_t mid = a + (b - a) / 2;
        if (v[mid] <= x) a = mid;
        else b = mid;
    }
    return a;
}

__global__ void k_items(const int32_t *__restrict__ line_first, const int32_t *__restrict__ item_off,
                        const int32_t *__restrict__ cell_start, const int32_t *__restrict__ nlines_p,
                        const int32_t *__restrict__ nitems_p, Item *__restrict__ items,
                        int32_t *__restrict__ bflag) {
    const int32_t L = *nlines_p;
    const int32_t I = *nitems_p;
    int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= I) return;
    // line of this item: last l with item_off[l] <= it
    const int32_t l = last_le(item_off, 0, L, (int32_t)it);
    const int32_t c0 = line_first[l], c1 = line_first[l + 1];
    const int32_t p0 = cell_start[c0], p1 = cell_start[c1];
    const int32_t qb = p0 + ((int32_t)it - item_off[l]) * kTileQ;
    const int32_t qe = min(qb + kTileQ, p1);
    Item r;
    r.qbegin = qb;
    r.qend = qe;
    r.cell_first = last_le(cell_start, c0, c1, qb);
    r.cell_last = last_le(cell_start, c0, c1, qe - 1);
    items[it] = r;
    // groups of kBlockItems consecutive items of one line form a block item
    bflag[it] = (((int32_t)it - item_off[l]) % kBlockItems) == 0 ? 1 : 0;
}

// Block items: first item of each group, and the end sentinel.
__global__ void k_blocks(const int32_t *__restrict__ bflag, const int32_t *__restrict__ bid,
                         const int32_t *__restrict__ nitems_p, int32_t *__restrict__ blocks,
                         int32_t *__restrict__ nblocks_p) {
    const int32_t I = *nitems_p;
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= I) return;
    if (bflag[it]) blocks[bid[it]] = (int32_t)it;
    if (it == I - 1) {
        const int32_t nb = bid[it] + bflag[it];
        blocks[nb] = I;
        *nblocks_p = nb;
    }
}

// ------------------------------------------------------- neighbour ranges ----
// For a cell with coordinates c and each offset o in {-1,0,1}^(k-1) of the
// leading indexed coordinates, the cells whose leading coordinates are c's
// plus o and whose last coordinate is within one of c's are adjacent in key
// order, hence one contiguous range of sorted points. A work item (queries of
// cells first..last of one line) takes, per offset, the union of those
// ranges of its first and last cell: last coordinates from first - 1 to
// last + 1. Out-of-grid offsets give an empty range.
struct RangeGeom {
    int k, nranges;
    int64_t m[kMaxIndexDims];
    int64_t stride[kMaxIndexDims];
    int sb;  // sub-cell bits of the sorted keys (0: no trimming)
};

// In the sorted v[a, b): x = first index with v >= lo, y = first index with
// v > hi (lo <= hi). The two binary searches run in lock-step, so their loads
// issue together (these searches are latency chains).
template <typename T>
__device__ __forceinline__ void bounds2(const T *__restrict__ v, int64_t a, int64_t b, T lo, T hi, int64_t &x,
                                        int64_t &y) {
    int64_t x0 = a, y0 = b, x1 = a, y1 = b;
    while (x0 < y0 || x1 < y1) {
        const int64_t m0 = x0 + (y0 - x0) / 2, m1 = x1 + (y1 - x1) / 2;
        const T v0 = v[min(m0, b - 1)], v1 = v[min(m1, b - 1)];  // b > a here
        if (x0 < y0) {
            if (v0 < lo) x0 = m0 + 1;
            else y0 = m0;
        }
        if (x1 < y1) {
            if (v1 <= hi) x1 = m1 + 1;
            else y1 = m1;
        }
    }
    x = x0;
    y = x1;
}

// Sorted-point range [begin, end) of the cells of line `base` (key of the
// line with last coordinate 0) whose last coordinate is in [lo_c, hi_c].
__device__ __forceinline__ Range line_segment(const int64_t *__restrict__ cell_key,
                                              const int32_t *__restrict__ cell_start, int64_t ncells,
                                              const int32_t *__restrict__ line_of_key,
                                              const int32_t *__restrict__ line_first, int64_t base, int64_t mlast,
                                              int64_t lo_c, int64_t hi_c) {
    Range r{0, 0};
    int64_t a = 0, b = ncells;
    if (line_of_key) {
        const int32_t lid = line_of_key[base / mlast];
        if (lid < 0) return r;
        a = line_first[lid];
        b = line_first[lid + 1];
    }
    int64_t ca, cb;  // first cell with key >= base + lo_c, first with key > base + hi_c
    bounds2<int64_t>(cell_key, a, b, base + lo_c, base + hi_c, ca, cb);
    r.begin = cell_start[ca];
    r.end = cell_start[cb];
    return r;
}

__device__ __forceinline__ void decode_key(int64_t key, const RangeGeom &geo, int64_t *cc) {
    for (int j = 0; j < geo.k; ++j) {
        cc[j] = key / geo.stride[j];
        key -= cc[j] * geo.stride[j];
    }
}

// Neighbouring line of offset o (base key, or -1 if outside the grid).
__device__ __forceinline__ int64_t neighbour_line(const int64_t *cc, int o, const RangeGeom &geo) {
    int64_t base = 0;
    for (int j = 0; j < geo.k - 1; ++j) {
        const int64_t cj = cc[j] + (o % 3) - 1;
        o /= 3;
        if (cj < 0 || cj >= geo.m[j]) return -1;
        base += cj * geo.stride[j];
    }
    return base;
}

// Block sum then one atomic per block.
__device__ __forceinline__ void block_add(unsigned long long v, unsigned long long *out) {
    __shared__ unsigned long long part[kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += part[w];
        if (t) atomicAdd(out, t);
    }
}

// Ranges of every work item (grid-stride over item x offset), plus the
// number of candidate pairs the items see. A range starts as the cells
// c_first - 1 .. c_last + 1 of a neighbour line. With sub-cell bits a point's
// position along the line is p = c_last * 2^sb + sub = floor(t 2^sb) (clamped,
// monotone), t = fl(fl(x - lo) / w); a pair within eps differs by less than
// w on the last indexed dimension, so by at most 2^sb in p. The range is cut
// to positions [p(first query) - 2^sb - 1, p(last query) + 2^sb + 1] (the
// item's queries are in key order) by two binary searches over the sorted
// keys.
__global__ void k_item_ranges(const Item *__restrict__ items, const int32_t *__restrict__ nitems_p,
                              const int64_t *__restrict__ cell_key, const int32_t *__restrict__ cell_start,
                              const int32_t *__restrict__ ncells_p, RangeGeom geo,
                              const int32_t *__restrict__ line_of_key, const int32_t *__restrict__ line_first,
                              const unsigned long long *__restrict__ skey, Range *__restrict__ ranges,
                              unsigned long long *__restrict__ cand_items) {
    const int64_t total = (int64_t)(*nitems_p) * geo.nranges;
    const int64_t ncells = *ncells_p;
    const int kl = geo.k - 1;
    const int64_t mlast = geo.m[kl];
    unsigned long long acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t it = t / geo.nranges;
        const int o = (int)(t - it * geo.nranges);
        const Item I = items[it];
        // keys of the item's first and last query (read ahead of the searches)
        const unsigned long long kf = geo.sb > 0 ? skey[I.qbegin] : 0ull;
        const unsigned long long kb = geo.sb > 0 ? skey[I.qend - 1] : 0ull;
        int64_t c0[kMaxIndexDims], c1[kMaxIndexDims];
        decode_key(cell_key[I.cell_first], geo, c0);
        decode_key(cell_key[I.cell_last], geo, c1);
        const int64_t base = neighbour_line(c0, o, geo);
        Range r{0, 0};
        if (base >= 0) {
            const int64_t lo_c = c0[kl] > 0 ? c0[kl] - 1 : 0;
            const int64_t hi_c = c1[kl] < mlast - 1 ? c1[kl] + 1 : c1[kl];
            r = line_segment(cell_key, cell_start, ncells, line_of_key, line_first, base, mlast, lo_c, hi_c);
            if (geo.sb > 0 && r.end > r.begin) {
                const unsigned long long sub = (1ull << geo.sb) - 1ull;
                const int64_t pf = (int64_t)((((kf >> geo.sb) % (unsigned long long)mlast) << geo.sb) | (kf & sub));
                const int64_t pb = (int64_t)((((kb >> geo.sb) % (unsigned long long)mlast) << geo.sb) | (kb & sub));
                const int64_t span = int64_t(1) << geo.sb, pmax = mlast * span - 1;
                const int64_t plo = max(pf - span - 1, int64_t(0)), phi = min(pb + span + 1, pmax);
                const unsigned long long klo = ((unsigned long long)base << geo.sb) + (unsigned long long)plo;
                const unsigned long long khi = ((unsigned long long)base << geo.sb) + (unsigned long long)phi;
                int64_t x0, x1;  // first key >= klo, first key > khi
                bounds2<unsigned long long>(skey, r.begin, r.end, klo, khi, x0, x1);
                r.begin = (int32_t)x0;
                r.end = (int32_t)x1;
            }
        }
        ranges[t] = r;
        acc += (unsigned long long)(I.qend - I.qbegin) * (unsigned long long)(r.end - r.begin);
    }
    block_add(acc, cand_items);
}

// d > 4: the ranges of every item become the union of its block item's
// (up to kBlockItems consecutive items of one line, starting where bflag is
// set): per neighbour line the smallest begin and largest end of the
// block's non-empty ranges. A superset of each item's own candidates (the
// tiles decide every pair), and the same list for the whole block item, so
// the FP64 MFMA count can stage each candidate tile once for all four items.
// Also the candidate pairs the items then see.
__global__ void k_unite_ranges(const Item *__restrict__ items, const int32_t *__restrict__ nitems_p,
                               const int32_t *__restrict__ bflag, int nranges, const Range *__restrict__ in,
                               Range *__restrict__ out, unsigned long long *__restrict__ cand_items) {
    const int64_t I = *nitems_p;
    unsigned long long acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < I * nranges;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t it = t / nranges;
        const int o = (int)(t - it * nranges);
        int64_t b0 = it;
        while (b0 > 0 && !bflag[b0]) --b0;
        int64_t b1 = b0 + 1;
        while (b1 < I && !bflag[b1]) ++b1;
        Range u{0, 0};
        bool any = false;
        for (int64_t i = b0; i < b1; ++i) {
            const Range r = in[i * nranges + o];
            if (r.end <= r.begin) continue;
            u.begin = any ? min(u.begin, r.begin) : r.begin;
            u.end = any ? max(u.end, r.end) : r.end;
            any = true;
        }
        out[t] = u;
        const Item m = items[it];
        acc += (unsigned long long)(m.qend - m.qbegin) * (unsigned long long)(u.end - u.begin);
    }
    block_add(acc, cand_items);
}

// Mask slots of each work item: its candidates (the ranges in order) form one
// packed list of ceil(sum of range lengths / 16) tiles, and its in-masks take
// whole groups of 16 tile slots (64 words of 64 bits per group); entry nitems
// is 0 so that an exclusive scan ends with the total.
__global__ void k_item_tiles(const Range *__restrict__ ranges, const int32_t *__restrict__ nitems_p, int nranges,
                             int32_t *__restrict__ tiles) {
    const int64_t I = *nitems_p;
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it > I) return;
    int64_t c = 0;
    if (it < I)
        for (int o = 0; o < nranges; ++o) {
            const Range r = ranges[it * nranges + o];
            c += r.end > r.begin ? r.end - r.begin : 0;
        }
    const int64_t nt = (c + 15) / 16;
    tiles[it] = (int32_t)((nt + 15) / 16 * 16);
}

__global__ void k_tiles_total(const int64_t *__restrict__ tile_off, const int32_t *__restrict__ nitems_p,
                              unsigned long long *__restrict__ out) {
    *out = (unsigned long long)tile_off[*nitems_p];
}

// C_ref = sum over non-empty cells c of |c| * (points in the 3^k cells around
// c): the implementation-free work unit (grid-stride over cell x offset).
__global__ void k_cell_cref(const int64_t *__restrict__ cell_key, const int32_t *__restrict__ cell_start,
                            int64_t ncells, RangeGeom geo, const int32_t *__restrict__ line_of_key,
                            const int32_t *__restrict__ line_first, unsigned long long *__restrict__ cref) {
    const int64_t total = ncells * geo.nranges;
    const int kl = geo.k - 1;
    const int64_t mlast = geo.m[kl];
    unsigned long long acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / geo.nranges;
        const int o = (int)(t - c * geo.nranges);
        int64_t cc[kMaxIndexDims];
        decode_key(cell_key[c], geo, cc);
        const int64_t base = neighbour_line(cc, o, geo);
        if (base < 0) continue;
        const int64_t lo_c = cc[kl] > 0 ? cc[kl] - 1 : 0;
        const int64_t hi_c = cc[kl] < mlast - 1 ? cc[kl] + 1 : cc[kl];
        const Range r = line_segment(cell_key, cell_start, ncells, line_of_key, line_first, base, mlast, lo_c, hi_c);
        acc += (unsigned long long)(cell_start[c + 1] - cell_start[c]) * (unsigned long long)(r.end - r.begin);
    }
    block_add(acc, cref);
}

// Dense map line key -> compact line id (-1 for empty lines).
__global__ void k_line_table(const int64_t *__restrict__ cell_key, const int32_t *__restrict__ line_first,
                             const int32_t *__restrict__ nlines_p, int64_t m_last, int32_t *__restrict__ table) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= *nlines_p) return;
    table[cell_key[line_first[l]] / m_last] = (int32_t)l;
}

RangeGeom range_geom(const Grid &g) {
    RangeGeom rg{};
    rg.k = g.k;
    rg.nranges = g.nranges;
    for (int j = 0; j < g.k; ++j) {
        rg.m[j] = g.m[j];
        rg.stride[j] = g.stride[j];
    }
    rg.sb = g.sub_bits;
    return rg;
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads); }

}  // namespace

void fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    unsigned blocks = (unsigned)std::min<size_t>((bytes + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(kThreads), 0, s, (unsigned char *)p, bytes, (unsigned char)0);
    SJ_HIP(hipGetLastError());
}

// Stable sort of (key, value) pairs by the low `bits` key bits. On return
// *key_a / *val_a point at the sorted arrays (buffers may be swapped).
void radix_sort_pairs(unsigned long long **key_a, int32_t **val_a, unsigned long long *key_b, int32_t *val_b,
                      int64_t n, int bits, hipStream_t s) {
    if (n <= 0) return;
    const int nb = (int)std::max<int64_t>(1, (n + kRsTile - 1) / kRsTile);
    int32_t *hist = dev_alloc_n<int32_t>((size_t)nb * 256, s);
    int32_t *hist_ex = dev_alloc_n<int32_t>((size_t)nb * 256, s);
    unsigned long long *ka = *key_a, *kb = key_b;
    int32_t *va = *val_a, *vb = val_b;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kThreads), 0, s, ka, n, shift, hist, nb);
        SJ_HIP(hipGetLastError());
        exclusive_scan<int32_t, int32_t>(hist, hist_ex, (int64_t)nb * 256, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kThreads), 0, s, ka, va, kb, vb, n, shift, hist_ex, nb);
        SJ_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    dev_free(hist, s);
    dev_free(hist_ex, s);
    *key_a = ka;
    *val_a = va;
}

void exclusive_scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s) {
    exclusive_scan<int32_t, int64_t>(in, out, n, s);
}

void free_grid(Grid &g, hipStream_t s) {
    if (g.borrowed) {  // the index arrays belong to a segmented build
        g.xs = g.xa = g.nrm = g.pn = nullptr;
        g.perm = nullptr;
        g.ranges = nullptr;
        g.item = nullptr;
        g.tile_off = nullptr;
        g.blocks = nullptr;
    }
    void *bufs[] = {g.xs,   g.xa,       g.nrm,        g.perm,       g.cell_key, g.cell_start, g.ranges,
                    g.item, g.dev_nmax, g.line_first, g.line_table, g.blocks,   g.cnt,        g.off, g.ctr,
                    g.tile_off, g.masks, g.pn, g.lp_goff, g.lp_masks};
    for (void *p : bufs)
        if (p) dev_free(p, s);
    g.xs = g.xa = g.nrm = g.pn = nullptr;
    g.perm = nullptr;
    g.cell_key = nullptr;
    g.cell_start = nullptr;
    g.ranges = nullptr;
    g.item = nullptr;
    g.dev_nmax = nullptr;
    g.line_first = nullptr;
    g.line_table = nullptr;
    g.blocks = nullptr;
    g.cnt = nullptr;
    g.off = nullptr;
    g.ctr = nullptr;
    g.tile_off = nullptr;
    g.masks = nullptr;
    g.masks_valid = false;
    g.lp_goff = nullptr;
    g.lp_masks = nullptr;
    g.lp_groups = -1;
    g.lp_masks_valid = false;
}

// Host-side reading of the grid geometry; identical arithmetic to the
// reference definition (floor((max - min) / w) + 1 cells per dimension).
// index_dims < 0 (no index): one indexed dimension with a cell wider than
// the data, so a single cell, one line and one candidate range [0, n) per
// work item (every ordered pair is a candidate).
static void choose_geometry(Grid &g, int index_dims) {
    double w = g.eps * (1.0 + 0x1p-19);
    if (index_dims < 0) w = std::max(w, 2.0 * (g.hi[0] - g.lo[0]));
    g.w = w;
    int k = index_dims < 0   ? 1
            : index_dims > 0 ? std::min(index_dims, std::min(g.d, kMaxIndexDims))
                             : std::min(g.d, kMaxIndexDims);
    // cells per dimension counted in double (an extent of 2^63 cells or more
    // must not wrap); if the first dimension alone needs 2^62 cells or more,
    // the grid is one cell (every key clamps to 0)
    double mc[kMaxIndexDims];
    for (;;) {
        double prod = 1.0;
        for (int j = 0; j < k; ++j) {
            mc[j] = std::floor((g.hi[j] - g.lo[j]) / w) + 1.0;
            prod *= mc[j];
        }
        if (prod < 0x1p62 || k == 1) break;
        --k;
    }
    const bool one_cell = !(mc[0] < 0x1p62);
    if (one_cell) mc[0] = 1.0;
    for (int j = 0; j < k; ++j) g.m[j] = (int64_t)mc[j];
    g.k = k;
    int64_t st = 1;
    for (int j = k - 1; j >= 0; --j) {
        g.stride[j] = st;
        st *= g.m[j];
    }
    const unsigned long long maxkey = (unsigned long long)st - 1ull;
    int bits = 0;
    while (bits < 64 && (maxkey >> bits) != 0ull) ++bits;
    g.key_bits = bits;
    // sub-cell bits fill the last 8-bit radix digit (at least 5 of them: one
    // more digit when fewer are free); none in the index-free form
    int sb = (bits + 7) / 8 * 8 - bits;
    if (sb < 5) sb += 8;
    g.sub_bits = (index_dims < 0 || one_cell) ? 0 : std::min(sb, 64 - bits);
    g.nranges = 1;
    for (int j = 0; j < k - 1; ++j) g.nranges *= 3;
}

// Dimension order of the distance tiles. A tile's 16 candidates come from
// one stretch of the sorted order, so they lie close together on the indexed
// dimensions, where a neighbour cell can put all of them up to two cell sides
// from the queries: the indexed dimensions come first (input order), and a
// whole tile is often beyond eps after them alone. The other dimensions
// follow by decreasing variance (ties by index), so the partial distance at
// each later K-step boundary grows as fast as the data allows (a filter
// choice only). An indexed dimension with a single cell bounds nothing and
// counts as non-indexed. Identity for d <= 4 or dim_order = 1.
static void choose_dim_order(Grid &g, const std::vector<double> &var) {
    const int d = g.d;
    for (int t = 0; t < d; ++t) g.fo[t] = (uint8_t)t;
    if (d <= 4 || g.dim_order != 0) return;
    auto bounded = [&](int j) { return j < g.k && g.m[j] > 1; };
    std::vector<int> idx(d);
    for (int t = 0; t < d; ++t) idx[t] = t;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (bounded(a) != bounded(b)) return bounded(a);
        if (bounded(a)) return a < b;
        return var[a] > var[b];
    });
    for (int t = 0; t < d; ++t) g.fo[t] = (uint8_t)idx[t];
}

void build_grid(Grid &g, const double *points, int64_t n, int d, double eps, int index_dims,
                hipStream_t s) {
    g.n = n;
    g.d = d;
    g.eps = eps;
    g.eps2 = eps * eps;
    g.dp = (d + 3) & ~3;
    g.da = (d & 3) ? ((d + 1 + 3) & ~3) : d;
    g.build_stream = s;
    const size_t rows = (size_t)n + kRowPad;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // device time of the build (not in a lean build)
    if (!g.lean) {
        SJ_HIP(hipEventCreate(&ev0));
        SJ_HIP(hipEventCreate(&ev1));
    }
    struct EvGuard {
        hipEvent_t &a, &b;
        ~EvGuard() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } evg{ev0, ev1};
    if (ev0) SJ_HIP(hipEventRecord(ev0, s));

    // ---- G1: bounding box, finiteness and (d > 4) moments (one host sync) ----
    const bool mom = d > 4 && g.dim_order == 0;
    std::vector<double> var(d, 0.0);
    if (n == 0) {
        for (int j = 0; j < d; ++j) g.lo[j] = g.hi[j] = g.mid[j] = 0.0;
    } else {
        const int64_t rows_per_block = std::max<int64_t>(1024, (n + 2047) / 2048);
        const int nb = (int)std::max<int64_t>(1, (n + rows_per_block - 1) / rows_per_block);
        const int parts = mom ? 4 : 2;
        double *part = dev_alloc_n<double>((size_t)parts * nb * d, s);
        double *pmin = part, *pmax = part + (size_t)nb * d;
        double *psum = mom ? part + 2 * (size_t)nb * d : nullptr;
        double *psq = mom ? part + 3 * (size_t)nb * d : nullptr;
        const size_t nbox = (size_t)(mom ? 4 : 2) * d;
        double *box = dev_alloc_n<double>(nbox + 1, s);
        int *bad = reinterpret_cast<int *>(box + nbox);
        fill_zero(bad, sizeof(int), s);
        if (mom)
            hipLaunchKernelGGL(k_bbox_partial<true>, dim3(nb), dim3(kThreads), 0, s, points, n, d, rows_per_block,
                               pmin, pmax, psum, psq, bad);
        else
            hipLaunchKernelGGL(k_bbox_partial<false>, dim3(nb), dim3(kThreads), 0, s, points, n, d, rows_per_block,
                               pmin, pmax, psum, psq, bad);
        SJ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_bbox_final, dim3(d), dim3(kThreads), 0, s, pmin, pmax, psum, psq, nb, d, box);
        SJ_HIP(hipGetLastError());
        std::vector<double> hb(nbox + 1);
        SJ_HIP(hipMemcpyAsync(hb.data(), box, (nbox + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
        dev_free(part, s);
        dev_free(box, s);
        int badflag;
        std::memcpy(&badflag, &hb[nbox], sizeof(int));
        if (badflag) throw std::string("non-finite coordinate in points");
        for (int j = 0; j < d; ++j) {
            g.lo[j] = hb[j];
            g.hi[j] = hb[d + j];
            g.mid[j] = 0.5 * g.lo[j] + 0.5 * g.hi[j];  // no overflow for any finite lo, hi
            if (mom) {
                const double m1 = hb[2 * d + j] / (double)n;
                var[j] = std::max(0.0, hb[3 * d + j] / (double)n - m1 * m1);
            }
        }
    }
    choose_geometry(g, index_dims);
    choose_dim_order(g, var);

    // ---- G2 + G3: cell keys, then a one-sweep radix sort on the key bits in use ----
    unsigned long long *key_a = dev_alloc_n<unsigned long long>(n, s);
    unsigned long long *key_b = dev_alloc_n<unsigned long long>(n, s);
    int32_t *val_a = dev_alloc_n<int32_t>(n, s);
    int32_t *val_b = dev_alloc_n<int32_t>(n, s);
    const int sort_bits = g.key_bits + g.sub_bits;
    const int passes = (sort_bits + 7) / 8;
    const bool packed = passes > 0 && sort_bits <= 32;
    const int64_t os_tiles = std::max<int64_t>(1, (n + kOsTile - 1) / kOsTile);
    int32_t *os_hist = dev_alloc_n<int32_t>(kOsMaxPasses * 256 + kOsMaxPasses + 1, s);  // hists, tile counters, err
    int32_t *os_ctr = os_hist + kOsMaxPasses * 256;
    int32_t *os_err = os_ctr + kOsMaxPasses;
    unsigned long long *os_status =
        passes > 0 ? dev_alloc_n<unsigned long long>((size_t)passes * os_tiles * 256, s) : nullptr;
    fill_zero_many({{os_hist, (kOsMaxPasses * 256 + kOsMaxPasses + 1) * sizeof(int32_t)},
                    {os_status, os_status ? (size_t)passes * os_tiles * 256 * sizeof(unsigned long long) : 0}},
                   s);
    if (n > 0) {
        KeyGeom geo{};
        geo.k = g.k;
        geo.d = d;
        geo.sb = g.sub_bits;
        geo.w = g.w;
        for (int j = 0; j < g.k; ++j) {
            geo.lo[j] = g.lo[j];
            geo.m[j] = g.m[j];
            geo.stride[j] = g.stride[j];
        }
        const unsigned kb = std::min(blocks_for(n), 512u);
        if (packed)
            hipLaunchKernelGGL(k_keys_hist<true>, dim3(kb), dim3(kThreads), 0, s, points, n, geo, key_a, val_a,
                               passes, os_hist);
        else
            hipLaunchKernelGGL(k_keys_hist<false>, dim3(kb), dim3(kThreads), 0, s, points, n, geo, key_a, val_a,
                               passes, os_hist);
        SJ_HIP(hipGetLastError());
        for (int p = 0; p < passes; ++p) {
            const bool last = p == passes - 1;
            unsigned long long *st = os_status + (size_t)p * os_tiles * 256;
            if (!packed)
                hipLaunchKernelGGL(k_onesweep<OS_WIDE>, dim3((unsigned)os_tiles), dim3(kThreads), 0, s, key_a, val_a,
                                   key_b, val_b, n, 8 * p, os_hist + 256 * p, st, os_ctr + p, os_err);
            else if (!last)
                hipLaunchKernelGGL(k_onesweep<OS_PACKED>, dim3((unsigned)os_tiles), dim3(kThreads), 0, s, key_a,
                                   val_a, key_b, val_b, n, 8 * p, os_hist + 256 * p, st, os_ctr + p, os_err);
            else
                hipLaunchKernelGGL(k_onesweep<OS_PACKED_SPLIT>, dim3((unsigned)os_tiles), dim3(kThreads), 0, s,
                                   key_a, val_a, key_b, val_b, n, 8 * p, os_hist + 256 * p, st, os_ctr + p, os_err);
            SJ_HIP(hipGetLastError());
            std::swap(key_a, key_b);
            // packed passes carry the index in the key word; the last one
            // writes it to the index array
            if (!packed || last) std::swap(val_a, val_b);
        }
    }
    if (os_status) dev_free(os_status, s);
    g.perm = val_a;
    dev_free(val_b, s);

    // ---- G6: gather sorted rows, centred rows, norms ----
    g.xs = dev_alloc_n<double>(rows * g.dp, s);
    g.xa = dev_alloc_n<double>(rows * g.da, s);
    g.nrm = dev_alloc_n<double>(rows, s);
    g.npc = d > 4 ? g.da / 4 - 1 : 0;
    if (g.npc > 0) g.pn = dev_alloc_n<double>(rows * g.npc, s);
    g.dev_nmax = dev_alloc_n<double>(1, s);
    int32_t *counters = dev_alloc_n<int32_t>(4, s);                    // ncells, nlines, nitems
    unsigned long long *acc = dev_alloc_n<unsigned long long>(3, s);  // item candidates, tiles, united candidates
    // padding rows, nmax (n = 0), counters: one launch
    fill_zero_many({{g.xs + (size_t)n * g.dp, (size_t)kRowPad * g.dp * sizeof(double)},
                    {g.xa + (size_t)n * g.da, (size_t)kRowPad * g.da * sizeof(double)},
                    {g.nrm + n, (size_t)kRowPad * sizeof(double)},
                    {g.pn ? g.pn + (size_t)n * g.npc : nullptr, (size_t)kRowPad * g.npc * sizeof(double)},
                    {g.dev_nmax, sizeof(double)},
                    {counters, 4 * sizeof(int32_t)},
                    {acc, 3 * sizeof(unsigned long long)}},
                   s);
    if (n > 0) {
        const bool lds_rows = d >= 16 && d <= kGatherLdsD;
        const unsigned nb = d <= 4 ? std::min(blocks_for(4 * n), 4096u)
                            : lds_rows ? (unsigned)((n + kGatherRows - 1) / kGatherRows)
                                       : blocks_for(n);
        double *part = dev_alloc_n<double>(nb, s);
        if (d <= 4) {
            Mid4 mid{};
            for (int j = 0; j < d; ++j) mid.m[j] = g.mid[j];
            hipLaunchKernelGGL(k_gather4, dim3(nb), dim3(kThreads), 0, s, points, g.perm, n, d, mid, g.xs, g.xa,
                               g.nrm, part);
        } else {
            GatherArgs ga{};
            ga.d = d;
            ga.dp = g.dp;
            ga.da = g.da;
            ga.npc = g.npc;
            for (int j = 0; j < d; ++j) {
                ga.mid[j] = g.mid[j];
                ga.fo[j] = g.fo[j];
            }
            if (lds_rows)
                hipLaunchKernelGGL(k_gather_lds, dim3(nb), dim3(64), 0, s, points, g.perm, n, ga, g.xs, g.xa, g.nrm,
                                   g.pn, part);
            else
                hipLaunchKernelGGL(k_gather, dim3(nb), dim3(kThreads), 0, s, points, g.perm, n, ga, g.xs, g.xa,
                                   g.nrm, g.pn, part);
        }
        SJ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kThreads), 0, s, part, (int64_t)nb, g.dev_nmax);
        SJ_HIP(hipGetLastError());
        dev_free(part, s);
    }

    // ---- G4: cell table, lines, work items ----
    // flags / scan scratch, reused for cells (n), lines (<= n) and items (<= n + n/16 + 1)
    int32_t *flag = dev_alloc_n<int32_t>(n + n / kTileQ + 2, s);
    int32_t *cid = dev_alloc_n<int32_t>(n + n / kTileQ + 2, s);
    g.cell_key = dev_alloc_n<int64_t>(n + 1, s);
    g.cell_start = dev_alloc_n<int32_t>(n + 2, s);
    int32_t *line_first = dev_alloc_n<int32_t>(n + 2, s);
    int32_t *nitem = dev_alloc_n<int32_t>(n + 1, s);
    int32_t *item_off = dev_alloc_n<int32_t>(n + 1, s);
    if (n > 0) {
        hipLaunchKernelGGL(k_cell_flags, dim3(blocks_for(n)), dim3(kThreads), 0, s, key_a, n, g.sub_bits, flag);
        SJ_HIP(hipGetLastError());
        exclusive_scan<int32_t, int32_t>(flag, cid, n, s);
        hipLaunchKernelGGL(k_cell_write, dim3(blocks_for(n)), dim3(kThreads), 0, s, key_a, g.sub_bits, flag, cid, n,
                           g.cell_key, g.cell_start, counters + 0);
        SJ_HIP(hipGetLastError());
        // lines (cells grid-stride bounded by n)
        hipLaunchKernelGGL(k_line_flags, dim3(blocks_for(n)), dim3(kThreads), 0, s, g.cell_key, counters + 0,
                           (int64_t)g.m[g.k - 1], flag);
        SJ_HIP(hipGetLastError());
        exclusive_scan<int32_t, int32_t>(flag, cid, n, s);  // entries past ncells are ignored
        hipLaunchKernelGGL(k_line_write, dim3(blocks_for(n)), dim3(kThreads), 0, s, flag, cid, g.cell_start,
                           counters + 0, line_first, counters + 1);
        SJ_HIP(hipGetLastError());
        fill_zero(nitem, (size_t)(n + 1) * sizeof(int32_t), s);
        hipLaunchKernelGGL(k_line_items, dim3(blocks_for(n)), dim3(kThreads), 0, s, line_first, g.cell_start,
                           counters + 1, nitem);
        SJ_HIP(hipGetLastError());
    }
    // ---- G5: work items and their neighbour ranges (tables sized by upper bounds) ----
    const int64_t items_ub = n + n / kTileQ + 1;  // lines <= cells <= n
    g.tile_off = dev_alloc_n<int64_t>((size_t)items_ub + 1, s);
    int32_t *item_tiles = dev_alloc_n<int32_t>((size_t)items_ub + 1, s);
    g.item = dev_alloc_n<Item>((size_t)items_ub, s);
    g.blocks = dev_alloc_n<int32_t>((size_t)items_ub + 1, s);
    g.ranges = dev_alloc_n<Range>((size_t)items_ub * g.nranges, s);
    g.line_first = line_first;
    line_first = nullptr;  // kept by the grid (lazy C_ref)
    if (n > 0) {
        exclusive_scan<int32_t, int32_t>(nitem, item_off, n, s);  // entries past nlines are ignored
        hipLaunchKernelGGL(k_items_total, dim3(1), dim3(1), 0, s, nitem, item_off, counters + 1, counters + 2);
        SJ_HIP(hipGetLastError());
        // dense line table when the leading indexed dimensions span few lines
        int64_t nline_keys = 1;
        for (int j = 0; j < g.k - 1; ++j) nline_keys *= g.m[j];
        if (nline_keys <= (g.lean ? kLeanLineTable : (int64_t(1) << 24))) {
            g.line_table = dev_alloc_n<int32_t>((size_t)nline_keys, s);
            fill_ones(g.line_table, (size_t)nline_keys * sizeof(int32_t), s);
            hipLaunchKernelGGL(k_line_table, dim3(blocks_for(n)), dim3(kThreads), 0, s, g.cell_key, g.line_first,
                               counters + 1, (int64_t)g.m[g.k - 1], g.line_table);
            SJ_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_items, dim3(blocks_for(items_ub)), dim3(kThreads), 0, s, g.line_first, item_off,
                           g.cell_start, counters + 1, counters + 2, g.item, flag);
        SJ_HIP(hipGetLastError());
        // block items (groups of up to kBlockItems items of one line)
        exclusive_scan<int32_t, int32_t>(flag, cid, items_ub, s);
        hipLaunchKernelGGL(k_blocks, dim3(blocks_for(items_ub)), dim3(kThreads), 0, s, flag, cid, counters + 2,
                           g.blocks, counters + 3);
        SJ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_item_ranges, dim3(2048), dim3(kThreads), 0, s, g.item, counters + 2, g.cell_key,
                           g.cell_start, counters + 0, range_geom(g), g.line_table, g.line_first, key_a,
                           g.ranges, acc);
        SJ_HIP(hipGetLastError());
        if (d > 4) {  // block items share one candidate list
            Range *united = dev_alloc_n<Range>((size_t)items_ub * g.nranges, s);
            hipLaunchKernelGGL(k_unite_ranges, dim3(2048), dim3(kThreads), 0, s, g.item, counters + 2, flag,
                               g.nranges, g.ranges, united, acc + 2);
            SJ_HIP(hipGetLastError());
            dev_free(g.ranges, s);
            g.ranges = united;
            g.united = true;
        }
        // tile offsets of the items (for the per-tile in-masks of the count pass)
        hipLaunchKernelGGL(k_item_tiles, dim3(blocks_for(items_ub + 1)), dim3(kThreads), 0, s, g.ranges,
                           counters + 2, g.nranges, item_tiles);
        SJ_HIP(hipGetLastError());
        exclusive_scan<int32_t, int64_t>(item_tiles, g.tile_off, items_ub + 1, s);
        hipLaunchKernelGGL(k_tiles_total, dim3(1), dim3(1), 0, s, g.tile_off, counters + 2, acc + 1);
        SJ_HIP(hipGetLastError());
    }
    // ---- one host sync: table sizes, candidates of the items, nmax (gathered
    // on the device into one block, so that one copy brings them all) ----
    BuildReadback rb{};
    BuildReadback *rb_dev = nullptr;
    if (n > 0) {
        rb_dev = dev_alloc_n<BuildReadback>(1, s);
        hipLaunchKernelGGL(k_build_readback, dim3(1), dim3(1), 0, s, counters, os_err, g.dev_nmax, acc, rb_dev);
        SJ_HIP(hipGetLastError());
        SJ_HIP(hipMemcpyAsync(&rb, rb_dev, sizeof rb, hipMemcpyDeviceToHost, s));
    }
    const int32_t *hc = rb.c;
    const int32_t herr = rb.err;
    const double hn = rb.nmax;
    const unsigned long long *hacc = rb.acc;
    if (ev1) {
        SJ_HIP(hipEventRecord(ev1, s));
        SJ_HIP(hipEventSynchronize(ev1));
        float ms = 0.f;
        SJ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        g.ms_build = ms;
    } else {
        SJ_HIP(hipStreamSynchronize(s));
    }
    dev_free(os_hist, s);
    if (herr) throw HipError{hipErrorLaunchFailure, "radix sort: a tile's look-back did not complete"};
    g.cells = hc[0];
    g.items = hc[2];
    g.nblocks = hc[3];
    g.nmax = hn;
    g.cand_ref = -1;  // computed on request (grid_cref)
    g.cand_items = (int64_t)(g.united ? hacc[2] : hacc[0]);
    g.tiles = (int64_t)hacc[1];

    if (rb_dev) dev_free(rb_dev, s);
    dev_free(acc, s);
    dev_free(item_tiles, s);
    dev_free(key_a, s);
    dev_free(key_b, s);
    dev_free(flag, s);
    dev_free(cid, s);
    dev_free(counters, s);
    dev_free(nitem, s);
    dev_free(item_off, s);
}

int64_t grid_cref(Grid &g, hipStream_t s) {
    if (g.cand_ref >= 0) return g.cand_ref;
    if (g.cells == 0) return g.cand_ref = 0;
    unsigned long long *acc = dev_alloc_n<unsigned long long>(1, s);
    fill_zero(acc, sizeof(unsigned long long), s);
    hipLaunchKernelGGL(k_cell_cref, dim3(2048), dim3(kThreads), 0, s, g.cell_key, g.cell_start, g.cells,
                       range_geom(g), g.line_table, g.line_first, acc);
    SJ_HIP(hipGetLastError());
    unsigned long long h = 0;
    SJ_HIP(hipMemcpyAsync(&h, acc, sizeof h, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    dev_free(acc, s);
    g.cand_ref = (int64_t)h;
    return g.cand_ref;
}

// ============================================================ segmented ====
// Grid builds of many problems at once (the batched form). Every step runs
// over all problems in one launch: points, cells, lines and work items of
// all problems sit in shared arrays, problem p's sorted points at
// [pt_off[p], pt_off[p] + n_p). The sort key carries the problem index above
// the cell key, so one radix sort orders every problem's points by its own
// cells; each problem's cells, lines and items are then contiguous, and the
// first element of the next problem ends the one before (the searches of a
// problem stay inside its own cells). Two host synchronisations in all: the
// bounding boxes (for the geometry, chosen on the host per problem), and the
// table sizes at the end.
namespace {

struct SegProb {
    const double *X;
    int64_t n, pt_off;       // points; first sorted position
    int64_t xs_off, xa_off;  // first element of the problem's rows in the shared arrays
    int64_t row_off;         // first row of nrm (rows include kRowPad pads)
    int64_t pn_off;          // first element of its prefix norms
    int64_t range_base;      // first range slot of its items
    int32_t d, dp, da, npc, nranges, mid_off;
    KeyGeom key;
    RangeGeom rg;
};

struct SegBlk {  // a block's share of one problem's rows
    int32_t p;
    int64_t r0, r1;
};

__device__ __forceinline__ int seg_find(const int64_t *__restrict__ off, int B, int64_t x) {
    int lo = 0, hi = B;  // last p with off[p] <= x
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Bounding box and moments of one problem's row run per block (as
// k_bbox_partial), into the block's 4 d partials.
__global__ void k_seg_bbox_partial(const SegProb *__restrict__ P, const SegBlk *__restrict__ blk,
                                   const int64_t *__restrict__ part_off, double *__restrict__ part,
                                   int *__restrict__ bad) {
    __shared__ double smin[kThreads], smax[kThreads], ssum[kThreads], ssq[kThreads];
    const SegBlk b = blk[blockIdx.x];
    const SegProb &q = P[b.p];
    const int d = q.d;
    const int S = (kThreads / d) * d;
    const int tid = threadIdx.x;
    double mn = INFINITY, mx = -INFINITY, s1 = 0.0, s2 = 0.0;
    int nonfinite = 0;
    if (tid < S && b.r0 < b.r1) {
        const double x0 = q.X[tid % d];
        for (int64_t e = b.r0 * d + tid; e < b.r1 * d; e += S) {
            const double v = q.X[e];
            nonfinite |= !isfinite(v);
            mn = fmin(mn, v);
            mx = fmax(mx, v);
            const double c = v - x0;
            s1 += c;
            s2 = fma(c, c, s2);
        }
    }
    smin[tid] = mn;
    smax[tid] = mx;
    ssum[tid] = s1;
    ssq[tid] = s2;
    if (nonfinite) atomicOr(bad, 1);
    __syncthreads();
    if (tid < d) {
        double a = INFINITY, c = -INFINITY, c1 = 0.0, c2 = 0.0;
        for (int t = tid; t < S; t += d) {
            a = fmin(a, smin[t]);
            c = fmax(c, smax[t]);
            c1 += ssum[t];
            c2 += ssq[t];
        }
        double *o = part + part_off[blockIdx.x];
        o[tid] = a;
        o[d + tid] = c;
        o[2 * d + tid] = c1;
        o[3 * d + tid] = c2;
    }
}

// One block per (problem, dimension): min, max and moment sums over the
// problem's blocks [b0, b1) into box[box_off + {0, d, 2d, 3d} + j].
struct SegDim {
    int32_t p, j, b0, b1;
    int64_t box_off;
};

__global__ void k_seg_bbox_final(const SegProb *__restrict__ P, const SegDim *__restrict__ dims,
                                 const int64_t *__restrict__ part_off, const double *__restrict__ part,
                                 double *__restrict__ box) {
    __shared__ double smin[kThreads], smax[kThreads], t1[kThreads], t2[kThreads];
    const SegDim D = dims[blockIdx.x];
    const int d = P[D.p].d;
    double a = INFINITY, b = -INFINITY, c1 = 0.0, c2 = 0.0;
    for (int t = D.b0 + (int)threadIdx.x; t < D.b1; t += blockDim.x) {
        const double *o = part + part_off[t];
        a = fmin(a, o[D.j]);
        b = fmax(b, o[d + D.j]);
        c1 += o[2 * d + D.j];
        c2 += o[3 * d + D.j];
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    t1[threadIdx.x] = c1;
    t2[threadIdx.x] = c2;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            t1[threadIdx.x] += t1[threadIdx.x + w];
            t2[threadIdx.x] += t2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        box[D.box_off + D.j] = smin[0];
        box[D.box_off + d + D.j] = smax[0];
        box[D.box_off + 2 * d + D.j] = t1[0];
        box[D.box_off + 3 * d + D.j] = t2[0];
    }
}

// Keys (problem index above the problem's cell key and sub-cell bits, as
// k_keys_hist) and values (global point index), with every pass's digit
// histogram.
__global__ __launch_bounds__(kThreads) void k_seg_keys_hist(const SegProb *__restrict__ P,
                                                            const SegBlk *__restrict__ blk, int keybits,
                                                            unsigned long long *__restrict__ key,
                                                            int32_t *__restrict__ val, int passes,
                                                            int32_t *__restrict__ hist) {
    __shared__ int32_t h[kOsMaxPasses * 256];
    for (int t = threadIdx.x; t < passes * 256; t += kThreads) h[t] = 0;
    __syncthreads();
    const SegBlk b = blk[blockIdx.x];
    const SegProb &q = P[b.p];
    const KeyGeom &geo = q.key;
    for (int64_t i = b.r0 + threadIdx.x; i < b.r1; i += kThreads) {
        unsigned long long kk = 0, sub = 0;
        for (int j = 0; j < geo.k; ++j) {
            const double t = __ddiv_rn(__dsub_rn(q.X[i * geo.d + j], geo.lo[j]), geo.w);
            double c = floor(t);
            c = !(c >= 0.0) ? 0.0 : (c > (double)(geo.m[j] - 1) ? (double)(geo.m[j] - 1) : c);
            const int64_t ci = (int64_t)c;
            kk += (unsigned long long)ci * (unsigned long long)geo.stride[j];
            if (j == geo.k - 1) sub = sub_cell(t, ci, geo.sb);
        }
        const unsigned long long full = ((unsigned long long)b.p << keybits) | (kk << geo.sb) | sub;
        key[q.pt_off + i] = full;
        val[q.pt_off + i] = (int32_t)(q.pt_off + i);
        for (int ps = 0; ps < passes; ++ps) atomicAdd(&h[ps * 256 + (int)((full >> (8 * ps)) & 255u)], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < passes * 256; t += kThreads)
        if (h[t]) atomicAdd(&hist[t], h[t]);
}

// Rows [0, n + kRowPad) of each problem: sorted rows (input order), centred
// rows in the problem's tile order, norms, prefix norms and the local input
// index (as k_gather); pad rows are zero. Also the sorted keys without the
// problem bits, and each problem's largest norm (bit pattern, atomic max).
__global__ void k_seg_gather(const SegProb *__restrict__ P, const SegBlk *__restrict__ blk,
                             const unsigned long long *__restrict__ key, const int32_t *__restrict__ val,
                             const double *__restrict__ mid_all, const uint8_t *__restrict__ fo_all, int keybits,
                             double *__restrict__ xs_all, double *__restrict__ xa_all, double *__restrict__ nrm_all,
                             double *__restrict__ pn_all, int32_t *__restrict__ perm_all,
                             unsigned long long *__restrict__ skey, unsigned long long *__restrict__ nmax_bits) {
    const SegBlk b = blk[blockIdx.x];
    const SegProb &q = P[b.p];
    const int d = q.d, dp = q.dp, da = q.da, npc = q.npc;
    const double *mid = mid_all + q.mid_off;
    const uint8_t *fo = fo_all + q.mid_off;
    const int64_t i = b.r0 + threadIdx.x;
    double nn = 0.0;
    if (i < b.r1) {
        double *ps = xs_all + q.xs_off + i * dp;
        double *pa = xa_all + q.xa_off + i * da;
        double *pnr = npc > 0 ? pn_all + q.pn_off + i * npc : nullptr;
        if (i < q.n) {
            const int64_t pos = q.pt_off + i;
            const int32_t loc = val[pos] - (int32_t)q.pt_off;
            perm_all[pos] = loc;
            skey[pos] = key[pos] & ((1ull << keybits) - 1ull);
            const double *src = q.X + (int64_t)loc * d;
            for (int t = 0; t < d; ++t) ps[t] = src[t];
            for (int t = 0; t < d; ++t) {
                const int u = fo[t];
                const double c = __dsub_rn(src[u], mid[u]);
                pa[t] = c;
                nn = __fma_rn(c, c, nn);
                if ((t & 3) == 3 && (t >> 2) < npc) pnr[t >> 2] = nn;
            }
            for (int t = d; t < dp; ++t) ps[t] = 0.0;
            for (int t = d; t < da; ++t) pa[t] = 0.0;
            if (d & 3) pa[d] = nn;
        } else {
            for (int t = 0; t < dp; ++t) ps[t] = 0.0;
            for (int t = 0; t < da; ++t) pa[t] = 0.0;
            for (int t = 0; t < npc; ++t) pnr[t] = 0.0;
        }
        nrm_all[q.row_off + i] = nn;
    }
    // block maximum (every row of the block belongs to problem b.p)
    __shared__ double red[kThreads / 64];
    double v = nn;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, red[w]);
        if (m > 0.0) atomicMax(&nmax_bits[b.p], (unsigned long long)__double_as_longlong(m));
    }
}

// Cell starts over all problems (flag[N] = 0 ends the scan).
__global__ void k_seg_cell_flags(const unsigned long long *__restrict__ skey, int64_t N,
                                 const int64_t *__restrict__ pt_off, int B, const int32_t *__restrict__ sbs,
                                 int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    if (i == N) {
        flag[i] = 0;
        return;
    }
    const int p = seg_find(pt_off, B, i);
    const int sb = sbs[p];
    flag[i] = (i == pt_off[p] || (skey[i] >> sb) != (skey[i - 1] >> sb)) ? 1 : 0;
}

__global__ void k_seg_cell_write(const unsigned long long *__restrict__ skey, int64_t N,
                                 const int64_t *__restrict__ pt_off, int B, const int32_t *__restrict__ sbs,
                                 const int32_t *__restrict__ flag, const int32_t *__restrict__ cid,
                                 int64_t *__restrict__ cell_key, int32_t *__restrict__ cell_start,
                                 int32_t *__restrict__ cellp, int32_t *__restrict__ ncells) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (flag[i]) {
        const int p = seg_find(pt_off, B, i);
        cell_key[cid[i]] = (int64_t)(skey[i] >> sbs[p]);
        cell_start[cid[i]] = (int32_t)i;
        cellp[cid[i]] = p;
    }
    if (i == N - 1) {
        const int32_t c = cid[i] + flag[i];
        *ncells = c;
        cell_start[c] = (int32_t)N;
        cellp[c] = B;
    }
}

// Line starts over all problems' cells; entries [ncells, len) are 0.
__global__ void k_seg_line_flags(const int64_t *__restrict__ cell_key, const int32_t *__restrict__ cellp,
                                 const int32_t *__restrict__ ncells_p, const int64_t *__restrict__ mlast, int64_t len,
                                 int32_t *__restrict__ lflag) {
    const int64_t ncells = *ncells_p;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= len) return;
    if (c >= ncells) {
        lflag[c] = 0;
        return;
    }
    const int p = cellp[c];
    lflag[c] = (c == 0 || cellp[c - 1] != p || cell_key[c] / mlast[p] != cell_key[c - 1] / mlast[p]) ? 1 : 0;
}

// Per problem: first cell, line and work item (entry B: the totals).
__global__ void k_seg_offsets(const int64_t *__restrict__ pt_off, int B, const int32_t *__restrict__ cid,
                              const int32_t *__restrict__ lid, const int32_t *__restrict__ item_off,
                              int64_t *__restrict__ cell_off, int64_t *__restrict__ it_off) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > B) return;
    const int32_t c = cid[pt_off[p]];
    cell_off[p] = c;
    it_off[p] = item_off[lid[c]];
}

// Candidate ranges of every work item of every problem (as k_item_ranges, on
// the problem's own cells), stored as the problem's local sorted positions
// at the problem's range slots.
__global__ void k_seg_item_ranges(const SegProb *__restrict__ P, int B, const Item *__restrict__ items,
                                  const int32_t *__restrict__ nitems_p, const int64_t *__restrict__ it_off,
                                  const int64_t *__restrict__ cell_off, const int64_t *__restrict__ cell_key,
                                  const int32_t *__restrict__ cell_start, const unsigned long long *__restrict__ skey,
                                  Range *__restrict__ ranges) {
    constexpr int kR = 27;  // 3^(kMaxIndexDims - 1)
    const int64_t total = (int64_t)(*nitems_p) * kR;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t it = t / kR;
        const int o = (int)(t - it * kR);
        const int p = seg_find(it_off, B, it);
        const SegProb &q = P[p];
        const RangeGeom &geo = q.rg;
        if (o >= geo.nranges) continue;
        const int kl = geo.k - 1;
        const int64_t mlast = geo.m[kl];
        const int64_t c0g = cell_off[p];
        const int64_t *ck = cell_key + c0g;
        const int32_t *cs = cell_start + c0g;
        const int64_t nc = cell_off[p + 1] - c0g;
        const Item I = items[it];
        const unsigned long long kf = geo.sb > 0 ? skey[I.qbegin] : 0ull;
        const unsigned long long kb = geo.sb > 0 ? skey[I.qend - 1] : 0ull;
        int64_t c0[kMaxIndexDims], c1[kMaxIndexDims];
        decode_key(cell_key[I.cell_first], geo, c0);
        decode_key(cell_key[I.cell_last], geo, c1);
        const int64_t base = neighbour_line(c0, o, geo);
        Range r{0, 0};
        if (base >= 0) {
            const int64_t lo_c = c0[kl] > 0 ? c0[kl] - 1 : 0;
            const int64_t hi_c = c1[kl] < mlast - 1 ? c1[kl] + 1 : c1[kl];
            r = line_segment(ck, cs, nc, nullptr, nullptr, base, mlast, lo_c, hi_c);
            if (geo.sb > 0 && r.end > r.begin) {
                const unsigned long long sub = (1ull << geo.sb) - 1ull;
                const int64_t pf = (int64_t)((((kf >> geo.sb) % (unsigned long long)mlast) << geo.sb) | (kf & sub));
                const int64_t pb = (int64_t)((((kb >> geo.sb) % (unsigned long long)mlast) << geo.sb) | (kb & sub));
                const int64_t span = int64_t(1) << geo.sb, pmax = mlast * span - 1;
                const int64_t plo = max(pf - span - 1, int64_t(0)), phi = min(pb + span + 1, pmax);
                const unsigned long long klo = ((unsigned long long)base << geo.sb) + (unsigned long long)plo;
                const unsigned long long khi = ((unsigned long long)base << geo.sb) + (unsigned long long)phi;
                int64_t x0, x1;
                bounds2<unsigned long long>(skey, r.begin, r.end, klo, khi, x0, x1);
                r.begin = (int32_t)x0;
                r.end = (int32_t)x1;
            }
        }
        if (r.end > r.begin) {
            r.begin -= (int32_t)q.pt_off;
            r.end -= (int32_t)q.pt_off;
        } else {
            r.begin = r.end = 0;
        }
        ranges[q.range_base + (it - it_off[p]) * geo.nranges + o] = r;
    }
}

// Per item of every problem: its in-mask tile slots (as k_item_tiles, entry
// nitems = 0), its candidate pairs into the problem's total, and its query
// run moved to the problem's local positions.
__global__ void k_seg_item_tiles(const SegProb *__restrict__ P, int B, Item *__restrict__ items,
                                 const int32_t *__restrict__ nitems_p, const int64_t *__restrict__ it_off,
                                 const Range *__restrict__ ranges, int32_t *__restrict__ tiles,
                                 unsigned long long *__restrict__ cand) {
    const int64_t I = *nitems_p;
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it > I) return;
    if (it == I) {
        tiles[it] = 0;
        return;
    }
    const int p = seg_find(it_off, B, it);
    const SegProb &q = P[p];
    const Range *rr = ranges + q.range_base + (it - it_off[p]) * q.nranges;
    int64_t c = 0;
    for (int o = 0; o < q.nranges; ++o) c += rr[o].end > rr[o].begin ? rr[o].end - rr[o].begin : 0;
    const int64_t nt = (c + 15) / 16;
    tiles[it] = (int32_t)((nt + 15) / 16 * 16);
    Item m = items[it];
    atomicAdd(&cand[p], (unsigned long long)(m.qend - m.qbegin) * (unsigned long long)c);
    m.qbegin -= (int32_t)q.pt_off;
    m.qend -= (int32_t)q.pt_off;
    items[it] = m;
}

// The united ranges of every problem with d > 4 (as k_unite_ranges, at the
// problem's range slots; blocks never cross a line, hence never a problem);
// others copied.
__global__ void k_seg_unite(const SegProb *__restrict__ P, int B, const int32_t *__restrict__ nitems_p,
                            const int64_t *__restrict__ it_off, const int32_t *__restrict__ bflag,
                            const Range *__restrict__ in, Range *__restrict__ out) {
    constexpr int kR = 27;
    const int64_t I = *nitems_p;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < I * kR; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t it = t / kR;
        const int o = (int)(t - it * kR);
        const int p = seg_find(it_off, B, it);
        const SegProb &q = P[p];
        if (o >= q.nranges) continue;
        const int64_t base = q.range_base - it_off[p] * q.nranges;  // slot of global item i: base + i nranges
        if (q.d <= 4) {
            out[base + it * q.nranges + o] = in[base + it * q.nranges + o];
            continue;
        }
        int64_t b0 = it;
        while (b0 > it_off[p] && !bflag[b0]) --b0;
        int64_t b1 = b0 + 1;
        while (b1 < it_off[p + 1] && !bflag[b1]) ++b1;
        Range u{0, 0};
        bool any = false;
        for (int64_t i = b0; i < b1; ++i) {
            const Range r = in[base + i * q.nranges + o];
            if (r.end <= r.begin) continue;
            u.begin = any ? min(u.begin, r.begin) : r.begin;
            u.end = any ? max(u.end, r.end) : r.end;
            any = true;
        }
        out[base + it * q.nranges + o] = u;
    }
}

// Per problem: first block item (entry B: the total).
__global__ void k_seg_block_off(const int64_t *__restrict__ it_off, int B, const int32_t *__restrict__ bid,
                                int64_t *__restrict__ bl_off) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > B) return;
    bl_off[p] = bid[it_off[p]];
}

// Per problem: in-mask tile slots (entry B: the total).
__global__ void k_seg_tiles(const int64_t *__restrict__ it_off, int B, const int64_t *__restrict__ tile_off,
                            int64_t *__restrict__ ptiles) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > B) return;
    ptiles[p] = tile_off[it_off[p]];
}

}  // namespace

bool build_grids_segmented(const std::vector<SegInput> &in, std::vector<Grid *> &out, std::vector<void *> &owned,
                           hipStream_t s) {
    const int B = (int)in.size();
    out.assign(B, nullptr);
    if (B == 0) return true;
    int pbits = 1;
    while ((1 << pbits) < B) ++pbits;
    // ---- phase 1: bounding boxes and moments of every problem ----
    std::vector<SegProb> hp(B);
    std::vector<int64_t> pt_off(B + 1, 0);
    std::vector<SegBlk> blk;
    std::vector<int64_t> part_off;
    std::vector<SegDim> dims;
    std::vector<int64_t> box_off(B + 1, 0);
    int64_t part_total = 0;
    for (int p = 0; p < B; ++p) {
        const SegInput &x = in[p];
        pt_off[p + 1] = pt_off[p] + x.n;
        hp[p].X = x.points;
        hp[p].n = x.n;
        hp[p].d = x.d;
        const int b0 = (int)blk.size();
        const int64_t rpb = 2048;
        for (int64_t r0 = 0; r0 < x.n; r0 += rpb) {
            blk.push_back({p, r0, std::min(x.n, r0 + rpb)});
            part_off.push_back(part_total);
            part_total += 4 * (int64_t)x.d;
        }
        for (int j = 0; j < x.d && x.n > 0; ++j) dims.push_back({p, j, b0, (int)blk.size(), box_off[p]});
        box_off[p + 1] = box_off[p] + 4 * (int64_t)x.d;
    }
    const int64_t N = pt_off[B];
    if (N >= (int64_t(1) << 31) - (int64_t)B * kRowPad) throw std::string("too many points in one batch");
    auto up = [&](const void *h, size_t bytes) {
        void *d = dev_alloc(bytes + 16, s);
        if (bytes) SJ_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
        return d;
    };
    SegProb *P = static_cast<SegProb *>(up(hp.data(), B * sizeof(SegProb)));
    std::vector<double> hbox(box_off[B] + 1, 0.0);
    int hbad = 0;
    {
        SegBlk *dblk = static_cast<SegBlk *>(up(blk.data(), blk.size() * sizeof(SegBlk)));
        int64_t *dpo = static_cast<int64_t *>(up(part_off.data(), part_off.size() * sizeof(int64_t)));
        SegDim *ddim = static_cast<SegDim *>(up(dims.data(), dims.size() * sizeof(SegDim)));
        double *part = dev_alloc_n<double>((size_t)std::max<int64_t>(1, part_total), s);
        double *box = dev_alloc_n<double>((size_t)box_off[B] + 1, s);
        int *bad = dev_alloc_n<int>(1, s);
        fill_zero(bad, sizeof(int), s);
        if (!blk.empty())
            hipLaunchKernelGGL(k_seg_bbox_partial, dim3((unsigned)blk.size()), dim3(kThreads), 0, s, P, dblk, dpo,
                               part, bad);
        SJ_HIP(hipGetLastError());
        if (!dims.empty())
            hipLaunchKernelGGL(k_seg_bbox_final, dim3((unsigned)dims.size()), dim3(kThreads), 0, s, P, ddim, dpo,
                               part, box);
        SJ_HIP(hipGetLastError());
        SJ_HIP(hipMemcpyAsync(hbox.data(), box, box_off[B] * sizeof(double), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
        for (void *q : {(void *)dblk, (void *)dpo, (void *)ddim, (void *)part, (void *)box, (void *)bad}) dev_free(q, s);
    }
    if (hbad) {
        dev_free(P, s);
        throw std::string("non-finite coordinate in points");
    }
    // ---- host: geometry and tile order per problem ----
    int keybits = 0;
    std::vector<double> mid_all;
    std::vector<uint8_t> fo_all;
    int64_t xs_tot = 0, xa_tot = 0, pn_tot = 0, rng_tot = 0;
    std::vector<int32_t> sbs(B);
    std::vector<int64_t> mlast(B);
    for (int p = 0; p < B; ++p) {
        const SegInput &x = in[p];
        Grid *g = new Grid();
        out[p] = g;
        g->n = x.n;
        g->d = x.d;
        g->eps = x.eps;
        g->eps2 = x.eps * x.eps;
        g->dp = (x.d + 3) & ~3;
        g->da = (x.d & 3) ? ((x.d + 1 + 3) & ~3) : x.d;
        g->sc = x.sc;
        g->dim_order = x.dim_order;
        g->borrowed = true;
        std::vector<double> var(x.d, 0.0);
        const double *bx = hbox.data() + box_off[p];
        for (int j = 0; j < x.d; ++j) {
            if (x.n == 0) {
                g->lo[j] = g->hi[j] = g->mid[j] = 0.0;
                continue;
            }
            g->lo[j] = bx[j];
            g->hi[j] = bx[x.d + j];
            g->mid[j] = 0.5 * g->lo[j] + 0.5 * g->hi[j];
            const double m1 = bx[2 * x.d + j] / (double)x.n;
            var[j] = std::max(0.0, bx[3 * x.d + j] / (double)x.n - m1 * m1);
        }
        choose_geometry(*g, x.index_dims);
        choose_dim_order(*g, var);
        g->npc = x.d > 4 ? g->da / 4 - 1 : 0;
        keybits = std::max(keybits, g->key_bits + g->sub_bits);
        SegProb &q = hp[p];
        q.pt_off = pt_off[p];
        q.xs_off = xs_tot;
        q.xa_off = xa_tot;
        q.row_off = pt_off[p] + (int64_t)p * kRowPad;
        q.pn_off = pn_tot;
        q.range_base = rng_tot;
        q.dp = g->dp;
        q.da = g->da;
        q.npc = g->npc;
        q.nranges = g->nranges;
        q.mid_off = (int32_t)mid_all.size();
        for (int j = 0; j < x.d; ++j) {
            mid_all.push_back(g->mid[j]);
            fo_all.push_back(g->fo[j]);
        }
        q.key = KeyGeom{};
        q.key.k = g->k;
        q.key.d = x.d;
        q.key.sb = g->sub_bits;
        q.key.w = g->w;
        for (int j = 0; j < g->k; ++j) {
            q.key.lo[j] = g->lo[j];
            q.key.m[j] = g->m[j];
            q.key.stride[j] = g->stride[j];
        }
        q.rg = range_geom(*g);
        sbs[p] = g->sub_bits;
        mlast[p] = g->m[g->k - 1];
        const int64_t rows = x.n + kRowPad;
        xs_tot += rows * g->dp;
        xa_tot += rows * g->da;
        pn_tot += rows * g->npc;
        rng_tot += (x.n + x.n / kTileQ + 1) * g->nranges;
    }
    if (pbits + keybits > 64) {  // the problem bits do not fit above the widest key: per-problem builds
        dev_free(P, s);
        for (Grid *g : out) delete g;
        out.assign(B, nullptr);
        return false;
    }
    SJ_HIP(hipMemcpyAsync(P, hp.data(), B * sizeof(SegProb), hipMemcpyHostToDevice, s));
    // ---- phase 2: keys, one sort, rows, cells, lines, items, ranges, tiles ----
    auto keep = [&](void *q) {
        owned.push_back(q);
        return q;
    };
    double *xs_all = static_cast<double *>(keep(dev_alloc_n<double>((size_t)xs_tot, s)));
    double *xa_all = static_cast<double *>(keep(dev_alloc_n<double>((size_t)xa_tot, s)));
    double *nrm_all = static_cast<double *>(keep(dev_alloc_n<double>((size_t)(N + (int64_t)B * kRowPad), s)));
    double *pn_all = pn_tot > 0 ? static_cast<double *>(keep(dev_alloc_n<double>((size_t)pn_tot, s))) : nullptr;
    int32_t *perm_all = static_cast<int32_t *>(keep(dev_alloc_n<int32_t>((size_t)N + 1, s)));
    const int64_t items_ub = N + N / kTileQ + B + 1;
    Item *items = static_cast<Item *>(keep(dev_alloc_n<Item>((size_t)items_ub, s)));
    Range *ranges = static_cast<Range *>(keep(dev_alloc_n<Range>((size_t)std::max<int64_t>(1, rng_tot), s)));
    int32_t *blocks = static_cast<int32_t *>(keep(dev_alloc_n<int32_t>((size_t)items_ub + 1, s)));
    int64_t *tile_off = static_cast<int64_t *>(keep(dev_alloc_n<int64_t>((size_t)items_ub + 1, s)));

    std::vector<void *> tmp;
    auto scratch = [&](size_t bytes) {
        void *q = dev_alloc(bytes + 16, s);
        tmp.push_back(q);
        return q;
    };
    int64_t *d_pt_off = static_cast<int64_t *>(scratch((B + 1) * sizeof(int64_t)));
    SJ_HIP(hipMemcpyAsync(d_pt_off, pt_off.data(), (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    int32_t *d_sbs = static_cast<int32_t *>(up(sbs.data(), B * sizeof(int32_t)));
    tmp.push_back(d_sbs);
    int64_t *d_mlast = static_cast<int64_t *>(up(mlast.data(), B * sizeof(int64_t)));
    tmp.push_back(d_mlast);
    double *d_mid = static_cast<double *>(up(mid_all.data(), mid_all.size() * sizeof(double)));
    tmp.push_back(d_mid);
    uint8_t *d_fo = static_cast<uint8_t *>(up(fo_all.data(), fo_all.size()));
    tmp.push_back(d_fo);
    SegBlk *d_blk = static_cast<SegBlk *>(up(blk.data(), blk.size() * sizeof(SegBlk)));
    tmp.push_back(d_blk);
    // gather blocks: rows [0, n + kRowPad) of each problem, kThreads per block
    std::vector<SegBlk> gblk;
    for (int p = 0; p < B; ++p)
        for (int64_t r0 = 0; r0 < in[p].n + kRowPad; r0 += kThreads)
            gblk.push_back({p, r0, std::min<int64_t>(in[p].n + kRowPad, r0 + kThreads)});
    SegBlk *d_gblk = static_cast<SegBlk *>(up(gblk.data(), gblk.size() * sizeof(SegBlk)));
    tmp.push_back(d_gblk);

    const int bits = pbits + keybits;
    const int passes = (bits + 7) / 8;
    unsigned long long *ka = static_cast<unsigned long long *>(scratch((size_t)(N + 1) * 8));
    unsigned long long *kb = static_cast<unsigned long long *>(scratch((size_t)(N + 1) * 8));
    int32_t *va = static_cast<int32_t *>(scratch((size_t)(N + 1) * 4));
    int32_t *vb = static_cast<int32_t *>(scratch((size_t)(N + 1) * 4));
    const int64_t os_tiles = std::max<int64_t>(1, (N + kOsTile - 1) / kOsTile);
    int32_t *os_hist = static_cast<int32_t *>(scratch((kOsMaxPasses * 256 + kOsMaxPasses + 1) * sizeof(int32_t)));
    int32_t *os_ctr = os_hist + kOsMaxPasses * 256;
    int32_t *os_err = os_ctr + kOsMaxPasses;
    unsigned long long *os_status =
        static_cast<unsigned long long *>(scratch((size_t)passes * os_tiles * 256 * sizeof(unsigned long long)));
    unsigned long long *nmax_bits = static_cast<unsigned long long *>(scratch((size_t)B * 8));
    unsigned long long *cand = static_cast<unsigned long long *>(scratch((size_t)B * 8));
    int32_t *counters = static_cast<int32_t *>(scratch(4 * sizeof(int32_t)));  // ncells, nlines, nitems
    fill_zero_many({{os_hist, (kOsMaxPasses * 256 + kOsMaxPasses + 1) * sizeof(int32_t)},
                    {os_status, (size_t)passes * os_tiles * 256 * sizeof(unsigned long long)},
                    {nmax_bits, (size_t)B * 8},
                    {cand, (size_t)B * 8},
                    {counters, 4 * sizeof(int32_t)}},
                   s);
    if (!blk.empty()) {
        hipLaunchKernelGGL(k_seg_keys_hist, dim3((unsigned)blk.size()), dim3(kThreads), 0, s, P, d_blk, keybits, ka,
                           va, passes, os_hist);
        SJ_HIP(hipGetLastError());
    }
    for (int ps = 0; ps < passes && N > 0; ++ps) {
        unsigned long long *st = os_status + (size_t)ps * os_tiles * 256;
        hipLaunchKernelGGL(k_onesweep<OS_WIDE>, dim3((unsigned)os_tiles), dim3(kThreads), 0, s, ka, va, kb, vb, N,
                           8 * ps, os_hist + 256 * ps, st, os_ctr + ps, os_err);
        SJ_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    unsigned long long *skey = kb;  // the free key array receives the keys without the problem bits
    hipLaunchKernelGGL(k_seg_gather, dim3((unsigned)gblk.size()), dim3(kThreads), 0, s, P, d_gblk, ka, va, d_mid,
                       d_fo, keybits, xs_all, xa_all, nrm_all, pn_all, perm_all, skey, nmax_bits);
    SJ_HIP(hipGetLastError());
    // cells
    int32_t *flag = static_cast<int32_t *>(scratch((size_t)(items_ub + 1) * 4));
    int32_t *cid = static_cast<int32_t *>(scratch((size_t)(items_ub + 1) * 4));
    int64_t *cell_key = static_cast<int64_t *>(scratch((size_t)(N + 1) * 8));
    int32_t *cell_start = static_cast<int32_t *>(scratch((size_t)(N + 2) * 4));
    int32_t *cellp = static_cast<int32_t *>(scratch((size_t)(N + 2) * 4));
    hipLaunchKernelGGL(k_seg_cell_flags, dim3(blocks_for(N + 1)), dim3(kThreads), 0, s, skey, N, d_pt_off, B, d_sbs,
                       flag);
    SJ_HIP(hipGetLastError());
    exclusive_scan<int32_t, int32_t>(flag, cid, N + 1, s);
    hipLaunchKernelGGL(k_seg_cell_write, dim3(blocks_for(N)), dim3(kThreads), 0, s, skey, N, d_pt_off, B, d_sbs, flag,
                       cid, cell_key, cell_start, cellp, counters + 0);
    SJ_HIP(hipGetLastError());
    // lines (cid is kept: it maps a problem's first point to its first cell)
    int32_t *lflag = static_cast<int32_t *>(scratch((size_t)(N + 1) * 4));
    int32_t *lid = static_cast<int32_t *>(scratch((size_t)(N + 1) * 4));
    int32_t *line_first = static_cast<int32_t *>(scratch((size_t)(N + 2) * 4));
    hipLaunchKernelGGL(k_seg_line_flags, dim3(blocks_for(N + 1)), dim3(kThreads), 0, s, cell_key, cellp, counters + 0,
                       d_mlast, N + 1, lflag);
    SJ_HIP(hipGetLastError());
    exclusive_scan<int32_t, int32_t>(lflag, lid, N + 1, s);
    hipLaunchKernelGGL(k_line_write, dim3(blocks_for(N)), dim3(kThreads), 0, s, lflag, lid, cell_start, counters + 0,
                       line_first, counters + 1);
    SJ_HIP(hipGetLastError());
    int32_t *nitem = static_cast<int32_t *>(scratch((size_t)(N + 1) * 4));
    int32_t *item_off = static_cast<int32_t *>(scratch((size_t)(N + 1) * 4));
    fill_zero(nitem, (size_t)(N + 1) * 4, s);
    hipLaunchKernelGGL(k_line_items, dim3(blocks_for(N)), dim3(kThreads), 0, s, line_first, cell_start, counters + 1,
                       nitem);
    SJ_HIP(hipGetLastError());
    exclusive_scan<int32_t, int32_t>(nitem, item_off, N + 1, s);
    hipLaunchKernelGGL(k_items_total, dim3(1), dim3(1), 0, s, nitem, item_off, counters + 1, counters + 2);
    SJ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_items, dim3(blocks_for(items_ub)), dim3(kThreads), 0, s, line_first, item_off, cell_start,
                       counters + 1, counters + 2, items, flag);
    SJ_HIP(hipGetLastError());
    int64_t *cell_off = static_cast<int64_t *>(scratch((B + 1) * sizeof(int64_t)));
    int64_t *it_off = static_cast<int64_t *>(scratch((B + 1) * sizeof(int64_t)));
    hipLaunchKernelGGL(k_seg_offsets, dim3(blocks_for(B + 1)), dim3(kThreads), 0, s, d_pt_off, B, cid, lid, item_off,
                       cell_off, it_off);
    SJ_HIP(hipGetLastError());
    Range *ranges_raw = static_cast<Range *>(scratch((size_t)std::max<int64_t>(1, rng_tot) * sizeof(Range)));
    hipLaunchKernelGGL(k_seg_item_ranges, dim3(2048), dim3(kThreads), 0, s, P, B, items, counters + 2, it_off,
                       cell_off, cell_key, cell_start, skey, ranges_raw);
    SJ_HIP(hipGetLastError());
    // block items (k_items left their start flags in `flag`) and united ranges for d > 4
    int32_t *bid = static_cast<int32_t *>(scratch((size_t)(items_ub + 1) * 4));
    exclusive_scan<int32_t, int32_t>(flag, bid, items_ub, s);
    hipLaunchKernelGGL(k_blocks, dim3(blocks_for(items_ub)), dim3(kThreads), 0, s, flag, bid, counters + 2, blocks,
                       counters + 3);
    SJ_HIP(hipGetLastError());
    int64_t *bl_off = static_cast<int64_t *>(scratch((B + 1) * sizeof(int64_t)));
    hipLaunchKernelGGL(k_seg_block_off, dim3(blocks_for(B + 1)), dim3(kThreads), 0, s, it_off, B, bid, bl_off);
    SJ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_unite, dim3(2048), dim3(kThreads), 0, s, P, B, counters + 2, it_off, flag, ranges_raw,
                       ranges);
    SJ_HIP(hipGetLastError());
    int32_t *item_tiles = static_cast<int32_t *>(scratch((size_t)(items_ub + 1) * 4));
    hipLaunchKernelGGL(k_seg_item_tiles, dim3(blocks_for(items_ub + 1)), dim3(kThreads), 0, s, P, B, items,
                       counters + 2, it_off, ranges, item_tiles, cand);
    SJ_HIP(hipGetLastError());
    exclusive_scan<int32_t, int64_t>(item_tiles, tile_off, items_ub + 1, s);
    int64_t *ptiles = static_cast<int64_t *>(scratch((B + 1) * sizeof(int64_t)));
    hipLaunchKernelGGL(k_seg_tiles, dim3(blocks_for(B + 1)), dim3(kThreads), 0, s, it_off, B, tile_off, ptiles);
    SJ_HIP(hipGetLastError());
    // ---- one host sync: per-problem items, tiles, norms, candidates ----
    std::vector<int64_t> h_it(B + 1), h_tiles(B + 1), h_bl(B + 1);
    std::vector<unsigned long long> h_nmax(B), h_cand(B);
    int32_t herr = 0;
    SJ_HIP(hipMemcpyAsync(h_it.data(), it_off, (B + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(h_tiles.data(), ptiles, (B + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(h_bl.data(), bl_off, (B + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(h_nmax.data(), nmax_bits, B * 8, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(h_cand.data(), cand, B * 8, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(&herr, os_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    for (void *q : tmp) dev_free(q, s);
    dev_free(P, s);
    if (herr) throw HipError{hipErrorLaunchFailure, "radix sort: a tile's look-back did not complete"};
    for (int p = 0; p < B; ++p) {
        Grid &g = *out[p];
        const SegProb &q = hp[p];
        g.xs = xs_all + q.xs_off;
        g.xa = xa_all + q.xa_off;
        g.nrm = nrm_all + q.row_off;
        g.pn = g.npc > 0 ? pn_all + q.pn_off : nullptr;
        g.perm = perm_all + q.pt_off;
        g.item = items + h_it[p];
        g.ranges = ranges + q.range_base;
        g.tile_off = tile_off + h_it[p];  // global tile slots: the batch's in-masks are shared
        g.items = h_it[p + 1] - h_it[p];
        g.tiles = h_tiles[p + 1] - h_tiles[p];
        double nm = 0.0;
        std::memcpy(&nm, &h_nmax[p], sizeof nm);
        g.nmax = nm;
        g.cand_items = (int64_t)h_cand[p];
        g.cand_ref = -1;
        g.blocks = blocks + h_bl[p];  // global item indices: item_base below
        g.nblocks = h_bl[p + 1] - h_bl[p];
        g.item_base = (int32_t)h_it[p];
        g.united = g.d > 4;
    }
    return true;
}

}  // namespace sj

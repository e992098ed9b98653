// Low-precision MFMA paths (FP32, BF16 and split BF16 inputs, FP32
// accumulation) with an exact FP64 recheck. The paper computes its tiles in
// FP64 and names other tensor-core precisions as future work (Section V);
// this is that form.
//
// Split BF16: each centred coordinate y is carried as hi = bf16(fl32(y)) and
// lo = bf16(fl32(y) - hi) (the difference is exact in FP32), so hi + lo holds
// y to about 2^-16 relative instead of BF16's 2^-8. A tile takes three BF16
// MFMAs (lo.hi, hi.lo, hi.hi, small terms first); the lo.lo products are
// dropped and covered by the band.
//
// Work unit: a block item = up to 4 consecutive 16-query work items of one
// grid line (64 queries, one per wave row tile) sharing the union of their
// candidate ranges. Candidates are staged 64 at a time into LDS (the exact
// recheck of the FP32 and split-BF16 paths reads the FP64 rows from global
// memory, where the staging has just brought them into the caches; plain
// BF16, with its wide band, keeps them in LDS):
//  - the rows centred on the block's reference point r (its first query)
//    and rounded to FP32 or BF16 (round to nearest even) -- the MFMA B
//    operand,
//  - the FP64 squared norms of the rounded rows.
// Each wave's A operand holds its 16 queries, centred and rounded the same
// way, times -2 (exact). The accumulator starts at the candidate norm, so a
// tile yields D = |c'|^2 - 2 q'.c' (Eq. (3) with |q'|^2 moved to the
// threshold side): in iff D <= eps^2 - |q'|^2.
//
// Scale. The tiles work on centred coordinates times sc = 2^-ilogb(eps), a
// power of two that puts eps in [1, 2) (exact in FP64), so the FP32 / BF16
// values keep their precision whatever the data's units; the band below is
// in those units. The grid's range guard (lowp_in_range) sends data whose
// extent exceeds 2^40 eps in some dimension, or eps outside [2^-500, 2^500],
// to the FP64 paths instead, so no scaled value approaches the FP32 range.
//
// Proven band, per query row. Let a = |q'|, eta the input rounding unit
// (subtraction in FP64, then rounding to the tile precision), u_a the FP32
// accumulation unit taken twice for safety, eps+ = eps (1 + (d + 4) u64),
// e = eta (2a + eps+) / (1 - 2 eta) and tau = eps+ + e. Only candidates with
// |c'| <= b = a + tau can be within eps+ of the query; for them the Gram value
// differs from the exact d2 - |q'|^2 by at most
//   F = (u32 + g_d + g_{K+1}) b^2 + 2 g_{K+1} a b + g_d a^2 + u32 (eps^2 + a^2)
// (C-init rounding, FP64 norms, accumulation; g_m = gamma_m) plus the
// conversion and oracle terms 2 tau e + e^2 + gamma_{d+2} tau^2; Delta is
// twice their sum. For |c'| > b the value minus its own error still
// increases with |c'| and exceeds eps^2 - Delta, so such candidates are
// never taken for in, and their exact distance exceeds eps+. Values with
// D <= thr - Delta are in, D > thr + Delta out, the rest are re-evaluated
// with the exact FP64 chain on the original coordinates: the result is the
// exact set.
//
// In-masks. The count pass records each wave's final in-bits (after the
// recheck, so exact) per 64-candidate tile of its block item, and a pairs
// pass then expands them (MODE_MASKEMIT: no staging, no distances) in the
// count's tile order, instead of running the tiles again.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "sj_internal.h"

namespace sj {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kTC = 64;            // candidates per staged tile
constexpr int kRing = 512;

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef short short8_t __attribute__((ext_vector_type(8)));

// MODE_MASKEMIT: the pairs of a count's recorded in-masks.
enum { MODE_COUNT = 0, MODE_EMIT = 1, MODE_MEASURE = 2, MODE_MASKEMIT = 3 };
enum { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2, PREC_FP8 = 3 };

struct LpGrid {
    const double *xs;
    const double *nrm;
    const int32_t *perm;
    const Range *ranges;
    const Item *items;
    const int32_t *blocks;
    int32_t nblocks;
    int32_t d, dp, nranges;
    double eps2;         // fl(eps^2): the exact test of the recheck
    double sc;           // power of two with eps * sc in [1, 2): the tiles work on scaled centred coordinates
    double eps_s, eps2_s;  // eps * sc, eps2 * sc^2 (exact)
};

struct LpOut {
    int32_t *cnt;
    const int64_t *off;
    int64_t base;
    int32_t qlo, qhi;
    int32_t *pairs;
    double *d2;
    DevCounters *ctr;              // rechecks, band widths (scaled units), measurements
    int32_t block_lo;              // first block item of this launch
    unsigned long long *masks;     // count: in-masks to record (nullable); MODE_MASKEMIT: to expand
    const int64_t *goff;           // first mask group of each block item
};

// The block item's candidate list along neighbour line o (lane o < nranges):
// from the smallest begin to the largest end of its items' ranges.
__device__ __forceinline__ void block_span(const LpGrid &G, int ib, int ie, int o, int &rb, int &re) {
    rb = G.ranges[(int64_t)ib * G.nranges + o].begin;
    re = G.ranges[(int64_t)ib * G.nranges + o].end;
    for (int it = ib + 1; it < ie; ++it) {
        const Range r = G.ranges[(int64_t)it * G.nranges + o];
        rb = min(rb, r.begin);
        re = max(re, r.end);
    }
}

// Mask groups of each block item: its 64-candidate tiles (per neighbour
// line, ceil(length / 64)) in groups of 4.
__global__ __launch_bounds__(kThreads) void k_lp_groups(LpGrid G, int32_t *__restrict__ groups) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= G.nblocks) return;
    const int ib = G.blocks[bi], ie = G.blocks[bi + 1];
    int tiles = 0;
    for (int o = 0; o < G.nranges; ++o) {
        int rb, re;
        block_span(G, ib, ie, o, rb, re);
        if (re > rb) tiles += (re - rb + kTC - 1) / kTC;
    }
    groups[bi] = (tiles + 3) >> 2;
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Hardware block b runs on XCD b % 8: chunks of kXcdChunk consecutive logical
// blocks (adjacent block items share candidates in one L2) are dealt
// round-robin to the XCDs, spreading dense regions of the index; a final
// partial round keeps the hardware order.
constexpr int kXcdChunk = 16;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int full = nb / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (b >= full) return b;
    const int x = b & 7, k = b >> 3;
    return ((k / kXcdChunk) * 8 + x) * kXcdChunk + (k % kXcdChunk);
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const unsigned lane = threadIdx.x & 63u;
    return lane ? ((~0ull) >> (64u - lane)) : 0ull;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The exact chain (ascending dimensions from +0.0, fl(a - b) then fma).
__device__ __forceinline__ double exact_d2(const double *a, const double *b, int d) {
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        const double delta = __dsub_rn(a[t], b[t]);
        acc = __fma_rn(delta, delta, acc);
    }
    return acc;
}

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// FP64 -> FP8 E4M3 (the OCP "e4m3fn" form the gfx950 FP8 MFMA reads: bias
// 7, 3 mantissa bits, largest finite 448, subnormals down to 2^-9), rounded
// to nearest even in one step; |y| must be below 464 (the range guard keeps
// the scaled values far below). Returns the rounded value and its bits.
__device__ __forceinline__ double fp8_round(double y, unsigned &bits) {
    const double ay = fabs(y);
    const unsigned sign = y < 0.0 ? 0x80u : 0u;
    if (ay == 0.0) {
        bits = 0u;
        return 0.0;
    }
    const int e = ilogb(ay);
    const double spacing = e < -6 ? 0x1p-9 : ldexp(1.0, e - 3);
    const double q = rint(ay / spacing) * spacing;  // exact quotient (power of two), RNE
    unsigned code = 0u;
    if (q != 0.0) {
        const int eq = ilogb(q);
        if (eq < -6) code = (unsigned)(q * 0x1p9);  // subnormal: exponent field 0
        else code = ((unsigned)(eq + 7) << 3) | ((unsigned)(q * ldexp(1.0, 3 - eq)) - 8u);
    }
    bits = code ? (sign | code) : 0u;
    return sign ? -q : q;
}

// Rounds an FP64 value to the tile precision; returns the rounded value as
// a double (exact) and its storage bits (split BF16: hi in the low half, lo
// in the high half; the value is hi + lo).
template <int PREC>
__device__ __forceinline__ double round_in(double y, unsigned &bits) {
    if constexpr (PREC == PREC_FP8) return fp8_round(y, bits);
    const float f = (float)y;  // RNE
    if (PREC == PREC_F32) {
        bits = __float_as_uint(f);
        return (double)f;
    }
    const unsigned short h = f32_to_bf16(f);
    const float fh = bf16_to_f32(h);
    if (PREC == PREC_BF16) {
        bits = h;
        return (double)fh;
    }
    const unsigned short l = f32_to_bf16(f - fh);  // f - fh exact
    bits = (unsigned)h | ((unsigned)l << 16);
    return (double)fh + (double)bf16_to_f32(l);
}

__device__ __forceinline__ double gam(double m, double u) { return m * u / (1.0 - m * u); }

// Band half-width of one query row (see the file comment), in the scaled
// units of the tiles (eps in [1, 2)): a2 = |q'|^2. Besides the relative
// terms, FP32 / BF16 values below the normal range (2^-126) may be flushed:
// at most 2^-126 per coordinate (2^-123 per vector of d <= 64) on the inputs
// and 2^-126 per product or partial sum, norm and threshold conversion.
template <int PREC>
__device__ __forceinline__ double lp_delta(double a2, double eps, double eps2, int d, int K) {
    const double u64 = 0x1p-53, u32 = 0x1p-24;
    // input rounding unit: FP32; BF16 via FP32 (two roundings); split BF16:
    // |fl32(y) - hi| <= 2^-8 |fl32(y)| and lo rounds that to 2^-8 of itself
    // (FP8: relative 2^-4 for normal values, from FP64 in one rounding)
    const double uin = PREC == PREC_F32    ? 0x1p-24
                       : PREC == PREC_BF16 ? (0x1p-8 + 0x1p-24)
                       : PREC == PREC_FP8  ? 0x1p-4
                                           : (0x1p-16 + 0x1p-24 + 0x1p-39);
    const double eta = uin + u64 + uin * u64;
    const double ua = 2.0 * 0x1p-24;
    const double a = sqrt(a2 * (1.0 + 1e-12));
    const double epsp = eps * (1.0 + (d + 4) * u64);
    // FP8 subnormals: at most 2^-10 per coordinate, 2^-7 per vector of d <= 64, for q' and c'
    const double e = eta * (2.0 * a + epsp) / (1.0 - 2.0 * eta) + 0x1p-122 +
                     (PREC == PREC_FP8 ? 0x1p-6 : 0.0);  // conversion error at |c'| = a + tau
    const double tau = epsp + e;
    const double b = a + tau;  // candidates beyond cannot be near the threshold
    const double A2 = a * a, B2 = b * b;
    // split BF16: 3d non-zero products per tile (the zero padding adds
    // exactly); sum_k (|hi|+|lo|)(|hi|+|lo|) over both rows is at most
    // (1 + 2^-6)^2 |q'||c'|, and the dropped 2 sum_k lo_q lo_c at most
    // 2 (2^-8 (1 + 2^-6))^2 |q'||c'| <= 2^-14 a b
    const int nt = PREC == PREC_BF16X3 ? 3 * d : K;
    const double gk = gam(nt + 1, ua);
    const double sp = PREC == PREC_BF16X3 ? (1.0 + 0x1p-6) * (1.0 + 0x1p-6) : 1.0;
    const double drop = PREC == PREC_BF16X3 ? 0x1p-14 : 0.0;
    const double F = (u32 + gam(d, u64) + gk) * B2 + (2.0 * gk * sp + drop) * a * b  // accumulation
                     + gam(d, u64) * A2 + u32 * (eps2 + A2)                        // threshold
                     + (2.0 * nt + 16.0) * 0x1p-126;                               // flushed tiny values
    return 2.0 * (F + 2.0 * tau * e + e * e + gam(d + 2, u64) * tau * tau) + (d + 2) * 0x1p-1021;
}

template <int PREC>
struct Prec;
template <>
struct Prec<PREC_F32> {
    static constexpr int kstep = 4;
    typedef float operand_t;
};
template <>
struct Prec<PREC_BF16> {
    static constexpr int kstep = 32;
    typedef short8_t operand_t;
};
template <>
struct Prec<PREC_BF16X3> {
    static constexpr int kstep = 32;
    typedef short8_t operand_t;
};

// K padded to the instruction's K-step; LDS row strides padded against bank
// conflicts.
template <>
struct Prec<PREC_FP8> {
    static constexpr int kstep = 32;
    typedef long operand_t;  // 8 FP8 values
};

template <int PREC>
constexpr int lp_kmax() {
    return PREC == PREC_F32 ? kLpMaxD : ((kLpMaxD + 31) / 32) * 32;
}
template <int PREC>
constexpr int lp_stride() {  // in 32-bit words
    return PREC == PREC_F32 ? lp_kmax<PREC>() + 1 : PREC == PREC_FP8 ? lp_kmax<PREC>() / 4 + 2 : lp_kmax<PREC>() / 2 + 4;
}

template <int PREC>
__device__ __forceinline__ float4_t lp_mfma(typename Prec<PREC>::operand_t a, typename Prec<PREC>::operand_t b,
                                            float4_t c);
template <>
__device__ __forceinline__ float4_t lp_mfma<PREC_F32>(float a, float b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ float4_t lp_mfma<PREC_BF16>(short8_t a, short8_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ float4_t lp_mfma<PREC_BF16X3>(short8_t a, short8_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <>
__device__ __forceinline__ float4_t lp_mfma<PREC_FP8>(long a, long b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// Reads the 8 FP8 values of one lane's K slice (8-byte aligned) from a row of bytes.
__device__ __forceinline__ long lds_fp8x8(const uint32_t *w) {
    return (long)((unsigned long long)w[0] | ((unsigned long long)w[1] << 32));
}

// Reads the 8 BF16 values of one lane's K slice from a row of 16-bit halves.
__device__ __forceinline__ short8_t lds_bf16x8(const uint32_t *w) {
    short8_t v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t x = w[e];
        v[2 * e] = (short)(x & 0xffffu);
        v[2 * e + 1] = (short)(x >> 16);
    }
    return v;
}

// The FP32 and split-BF16 counts fit four waves per SIMD (at most 128
// VGPRs) with the in-mask recording as without it.
template <int PREC, int MODE>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(MODE == MODE_COUNT && (PREC == PREC_F32 || PREC == PREC_BF16X3) ? 4 : 1, 8)))
void k_lowp(LpGrid G, LpOut R) {
    constexpr int KMAX = lp_kmax<PREC>();
    constexpr int STR = lp_stride<PREC>();
    constexpr int KSTEP = Prec<PREC>::kstep;
    constexpr bool kTiles = MODE != MODE_MASKEMIT;   // stage and compute tiles
    constexpr bool kEmit = MODE == MODE_EMIT || MODE == MODE_MASKEMIT;
    __shared__ double xr[kTiles ? kLpMaxD : 1];      // reference row
    // plain BF16 rechecks tens of percent of its pairs: it keeps the FP64
    // rows in LDS; the narrower-band paths read them from global memory
    constexpr bool kRowsInLds = kTiles && (PREC == PREC_BF16 || PREC == PREC_FP8);
    __shared__ double f64t[kRowsInLds ? kTC : 1][kLpMaxD + 1];
    __shared__ uint32_t lpt[kTiles ? kTC * STR : 1];  // rounded, centred rows (split BF16: hi)
    __shared__ uint32_t lptl[kTiles && PREC == PREC_BF16X3 ? kTC * STR : 1];  // split BF16: lo
    __shared__ float nc32[kTiles ? kTC : 1];         // their norms (FP32, accumulator init)
    __shared__ uint32_t ring_lds[kEmit ? kWaves * 3 * kRing : 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int bi = R.block_lo + xcd_block(blockIdx.x, gridDim.x);
    if (bi >= G.nblocks) return;  // whole block
    const int ib = G.blocks[bi], ie = G.blocks[bi + 1];
    const int d = G.d, dp = G.dp;
    const int K = ((d + KSTEP - 1) / KSTEP) * KSTEP;
    const int ks = K / KSTEP;

    // reference point: the block's first query
    if constexpr (kTiles) {
        const int qref = G.items[ib].qbegin;
        if (tid < d) xr[tid] = G.xs[(int64_t)qref * dp + tid];
        __syncthreads();
    }

    // this wave's queries
    const bool has_q = ib + wv < ie;
    int q0 = 0, nq = 0;
    if (has_q) {
        const Item I = G.items[ib + wv];
        q0 = I.qbegin;
        nq = I.qend - I.qbegin;
    }
    q0 = uniform_i32(q0);
    nq = uniform_i32(nq);
    const int j = lane & 15;
    const int g = lane >> 4;
    // A operand: -2 * round(q_j - r) over K (zeros past d or for absent rows)
    typename Prec<PREC>::operand_t aq[(KMAX + KSTEP - 1) / KSTEP];
    short8_t aql[PREC == PREC_BF16X3 ? (KMAX + KSTEP - 1) / KSTEP : 1];  // split BF16: -2 lo
    double nq_part = 0.0;
    if constexpr (kTiles) {
        const double *qrow = G.xs + (int64_t)(q0 + (j < nq ? j : 0)) * dp;
#pragma unroll
        for (int s = 0; s < (KMAX + KSTEP - 1) / KSTEP; ++s) {
            if constexpr (PREC == PREC_F32) {
                const int k = KSTEP * s + g;
                float v = 0.f;
                if (s < ks && j < nq && k < d) {
                    unsigned bits;
                    const double y = round_in<PREC>(__dsub_rn(qrow[k], xr[k]) * G.sc, bits);
                    nq_part = __fma_rn(y, y, nq_part);
                    v = -2.0f * __uint_as_float(bits);
                }
                aq[s] = v;
            } else if constexpr (PREC == PREC_FP8) {
                unsigned long long v = 0ull;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = KSTEP * s + 8 * g + e;
                    if (s < ks && j < nq && k < d) {
                        unsigned bits;
                        const double y = round_in<PREC>(__dsub_rn(qrow[k], xr[k]) * G.sc, bits);
                        nq_part = __fma_rn(y, y, nq_part);
                        unsigned b2;
                        (void)fp8_round(-2.0 * y, b2);  // exact: -2y is an FP8 value below the range limit
                        v |= (unsigned long long)b2 << (8 * e);
                    }
                }
                aq[s] = (long)v;
            } else {
                short8_t v, vl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = KSTEP * s + 8 * g + e;
                    unsigned short h = 0, l = 0;
                    if (s < ks && j < nq && k < d) {
                        unsigned bits;
                        const double y = round_in<PREC>(__dsub_rn(qrow[k], xr[k]) * G.sc, bits);
                        nq_part = __fma_rn(y, y, nq_part);
                        h = f32_to_bf16(-2.0f * bf16_to_f32((unsigned short)(bits & 0xffffu)));  // exact
                        l = f32_to_bf16(-2.0f * bf16_to_f32((unsigned short)(bits >> 16)));
                    }
                    v[e] = (short)h;
                    vl[e] = (short)l;
                }
                aq[s] = v;
                if constexpr (PREC == PREC_BF16X3) aql[s] = vl;
            }
        }
    }
    // |q'|^2 of query j: sum of the four K slices (lanes j, j+16, j+32, j+48)
    double nqj = nq_part;
    nqj += __shfl_xor(nqj, 16);
    nqj += __shfl_xor(nqj, 32);
    // rows of this lane in the result: 4g + r (16x16 FP32 / BF16 layouts)
    float lo[4], hi[4];
    double nqr[4], dlt[4];
    double maxdelta = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 4 * g + r;
        const double v = __shfl(nqj, i);
        nqr[r] = v;
        dlt[r] = lp_delta<PREC>(v, G.eps_s, G.eps2_s, d, K);
        const double thr = G.eps2_s - v;
        lo[r] = i < nq ? (float)(thr - dlt[r]) : -INFINITY;
        hi[r] = i < nq ? (float)(thr + dlt[r]) : -INFINITY;
        if (kTiles && i < nq) maxdelta = fmax(maxdelta, dlt[r]);
    }
    // emission state
    bool emit_r[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 4 * g + r;
        emit_r[r] = kEmit && i < nq && q0 + i >= R.qlo && q0 + i < R.qhi;
    }
    int64_t pbase_lane = -1;
    int32_t pq_lane = 0;
    if (kEmit && lane < nq && q0 + lane >= R.qlo && q0 + lane < R.qhi) {
        pbase_lane = R.off[q0 + lane] - R.base;
        pq_lane = G.perm[q0 + lane];
    }
    uint32_t *rcand = ring_lds + (kEmit ? wv * 3 * kRing : 0);
    uint32_t *rrel = rcand + kRing;
    uint32_t *rcol = rrel + kRing;
    int head = 0, tail = 0;
    const unsigned long long lt = lanemask_lt();
    const unsigned long long grp = 0xffffull << (16 * g);
    int cur[4] = {0, 0, 0, 0};
    int cnt[4] = {0, 0, 0, 0};
    unsigned long long band = 0, band_in = 0, viol = 0;
    double maxerr = 0.0;

    auto flush = [&](int nflush) {
        wave_lds_sync();
        const int e = (head + lane) & (kRing - 1);
        const uint32_t c = rcand[e], rel = rrel[e], col = rcol[e];
        const int64_t pb = __shfl(pbase_lane, (int)col);
        const int32_t pq = __shfl(pq_lane, (int)col);
        if (lane < nflush) {
            const int64_t pos = pb + rel;
            reinterpret_cast<int2 *>(R.pairs)[pos] = make_int2(pq, G.perm[c]);
            if (R.d2) R.d2[pos] = exact_d2(G.xs + (int64_t)(q0 + (int)col) * dp, G.xs + (int64_t)c * dp, d);
        }
        head += nflush;
        wave_lds_sync();
    };

    // per neighbour line, the span of the block's items' ranges (the items'
    // ranges may be cut to their own coordinate extents)
    int rb = 0, re = 0;
    if (lane < G.nranges) block_span(G, ib, ie, lane, rb, re);
    // in-masks: this wave's words of the block item's groups (4 tiles each)
    const bool rec = MODE == MODE_COUNT && R.masks != nullptr && has_q;
    // first word of this wave (wave-uniform; lane l adds l)
    const int64_t mbase = (MODE == MODE_COUNT || MODE == MODE_MASKEMIT) && R.masks
                              ? ((int64_t)__builtin_amdgcn_readfirstlane((int)(R.goff[bi] >> 32)) << 32 |
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)R.goff[bi])) * (kWaves * 64) + wv * 64
                              : 0;
    unsigned long long mword = 0;
    int tix = 0;  // tiles of the block item so far (block-uniform)
    // Tiles of 64 candidates over the block's ranges, in order. The next
    // tile's FP64 rows are loaded into registers while the current one is
    // computed; 4 threads per row, thread `part` holding dimensions
    // part, part + 4, ... (coalesced 32-byte runs per row).
    constexpr int CPT = KMAX / 4;
    const int srow = tid >> 2, part = tid & 3;
    double pre[CPT];
    int o_next = -1, t_next = 0, e_next = 0;
    auto advance = [&]() -> bool {  // block-uniform
        t_next += kTC;
        while (t_next >= e_next) {
            if (++o_next >= G.nranges) return false;
            t_next = __builtin_amdgcn_readlane(rb, o_next);
            e_next = __builtin_amdgcn_readlane(re, o_next);
        }
        return true;
    };
    auto prefetch = [&]() {
        const bool rowok = srow < e_next - t_next;
        const double *src = G.xs + (int64_t)(t_next + (rowok ? srow : 0)) * dp;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
            const int k = part + 4 * cc;
            pre[cc] = (rowok && k < d) ? src[k] : 0.0;
        }
    };
    if constexpr (MODE == MODE_MASKEMIT) {
        // expand the count's in-masks: the same tile walk, one word per
        // group of 4 tiles, no staging and no block synchronisation
        if (!has_q) return;
        bool more = advance();
        while (more) {
            const int t = t_next;
            const int nvalid = min(kTC, e_next - t_next);
            if ((tix & 3) == 0) mword = R.masks[mbase + (int64_t)(tix >> 2) * (kWaves * 64) + lane];
            for (int sub = 0; sub < kTC / 16; ++sub) {
                if (16 * sub >= nvalid) break;
                const int crow = 16 * sub + j;
                const unsigned inm = (unsigned)(mword >> (4 * (4 * (tix & 3) + sub))) & 0xFu;
                unsigned long long bal[4];
                int base_e = 0;
                int pre[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    bal[r] = __ballot(emit_r[r] && ((inm >> r) & 1u));
                    pre[r] = base_e + __popcll(bal[r] & lt);
                    base_e += __popcll(bal[r]);
                }
                if (base_e) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (emit_r[r] && ((inm >> r) & 1u)) {
                            const int e = (tail + pre[r]) & (kRing - 1);
                            rcand[e] = (uint32_t)(t + crow);
                            rrel[e] = (uint32_t)(cur[r] + __popcll(bal[r] & lt & grp));
                            rcol[e] = (uint32_t)(4 * g + r);
                        }
                    }
                    tail += base_e;
#pragma unroll
                    for (int r = 0; r < 4; ++r) cur[r] += __popcll(bal[r] & grp);
                    while (tail - head >= 64) flush(64);
                }
            }
            ++tix;
            more = advance();
        }
        if (tail > head) flush(tail - head);
        return;
    }
    bool have = advance();
    if (have) prefetch();
    while (have) {
        const int t = t_next;
        const int nvalid = min(kTC, e_next - t_next);
        __syncthreads();  // previous tile consumed
        // ---- stage the prefetched rows: FP64, rounded, norms ----
        {
            const bool rowok = srow < nvalid;
            double np = 0.0;
#pragma unroll
            for (int cc = 0; cc < CPT; ++cc) {
                const int k = part + 4 * cc;
                if (k < K) {  // K is a multiple of 4: uniform over the row's threads
                    const double x = pre[cc];
                    if constexpr (kRowsInLds) {
                        if (k < d) f64t[srow][k] = x;
                    }
                    unsigned bits = 0;
                    double y = 0.0;
                    if (rowok && k < d) y = round_in<PREC>(__dsub_rn(x, xr[k]) * G.sc, bits);
                    np = __fma_rn(y, y, np);
                    if constexpr (PREC == PREC_F32) {
                        lpt[srow * STR + k] = bits;
                    } else if constexpr (PREC == PREC_FP8) {
                        reinterpret_cast<unsigned char *>(lpt + srow * STR)[k] = (unsigned char)bits;
                    } else {
                        unsigned short *h = reinterpret_cast<unsigned short *>(lpt + srow * STR);
                        h[k] = (unsigned short)(bits & 0xffffu);
                        if constexpr (PREC == PREC_BF16X3) {
                            unsigned short *l = reinterpret_cast<unsigned short *>(lptl + srow * STR);
                            l[k] = (unsigned short)(bits >> 16);
                        }
                    }
                }
            }
            np += __shfl_xor(np, 1);
            np += __shfl_xor(np, 2);
            if (part == 0) nc32[srow] = rowok ? (float)np : INFINITY;
        }
        __syncthreads();
        have = advance();
        if (have) prefetch();  // in flight during this tile's MFMAs
        const int tcur = tix++;
        if (!has_q) continue;
        for (int sub = 0; sub < kTC / 16; ++sub) {
            if (16 * sub >= nvalid) break;
            const int crow = 16 * sub + j;  // candidate column j of this sub-tile
            const float nc = nc32[crow];
            float4_t acc = (float4_t){nc, nc, nc, nc};
            if constexpr (PREC == PREC_F32) {
                // up to 16 K-steps: a rolled loop (aq read by indexed moves),
                // four K-steps per trip so their LDS reads are in flight together
                const uint32_t *brow = lpt + crow * STR + g;
                int s = 0;
                for (; s + 4 <= ks; s += 4) {
                    const float b0 = __uint_as_float(brow[KSTEP * s]);
                    const float b1 = __uint_as_float(brow[KSTEP * (s + 1)]);
                    const float b2 = __uint_as_float(brow[KSTEP * (s + 2)]);
                    const float b3 = __uint_as_float(brow[KSTEP * (s + 3)]);
                    acc = lp_mfma<PREC>(aq[s], b0, acc);
                    acc = lp_mfma<PREC>(aq[s + 1], b1, acc);
                    acc = lp_mfma<PREC>(aq[s + 2], b2, acc);
                    acc = lp_mfma<PREC>(aq[s + 3], b3, acc);
                }
                for (; s < ks; ++s) acc = lp_mfma<PREC>(aq[s], __uint_as_float(brow[KSTEP * s]), acc);
            } else {
                // at most 2 K-steps: unrolled over the largest K so that aq /
                // aql are indexed statically (a runtime index would select
                // through every register of the arrays)
#pragma unroll
                for (int s = 0; s < (KMAX + KSTEP - 1) / KSTEP; ++s) {
                    if (s >= ks) break;  // block-uniform
                    if constexpr (PREC == PREC_FP8) {
                        acc = lp_mfma<PREC>(aq[s], lds_fp8x8(lpt + crow * STR + (KSTEP * s + 8 * g) / 4), acc);
                    } else {
                        const int o = crow * STR + (KSTEP * s + 8 * g) / 2;
                        const short8_t bh = lds_bf16x8(lpt + o);
                        if constexpr (PREC == PREC_BF16) {
                            acc = lp_mfma<PREC>(aq[s], bh, acc);
                        } else {
                            const short8_t bl = lds_bf16x8(lptl + o);
                            acc = lp_mfma<PREC>(aql[s], bh, acc);
                            acc = lp_mfma<PREC>(aq[s], bl, acc);
                            acc = lp_mfma<PREC>(aq[s], bh, acc);
                        }
                    }
                }
            }
            // element r: query 4g + r, candidate t + crow
            unsigned inm = 0, mbm = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                inm |= (acc[r] <= lo[r] ? 1u : 0u) << r;
                mbm |= (acc[r] <= hi[r] ? 1u : 0u) << r;
            }
            if (MODE == MODE_MEASURE) {
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * g + r;
                    if (i < nq && crow < nvalid) {
                        const double ex = exact_d2(G.xs + (int64_t)(q0 + i) * dp,
                                                   kRowsInLds ? &f64t[crow][0] : G.xs + (int64_t)(t + crow) * dp, d);
                        if (ex <= G.eps2) {  // the per-row bound covers pairs within eps
                            const double err = fabs((double)acc[r] - (ex * G.sc * G.sc - nqr[r]));
                            maxerr = fmax(maxerr, err);
                            if (err > dlt[r]) ++viol;
                        }
                    }
                }
            }
            const unsigned bm = mbm & ~inm;
            if (__any(bm != 0)) {
                for (int r = 0; r < 4; ++r) {
                    if (bm & (1u << r)) {
                        const int i = 4 * g + r;
                        const double ex = exact_d2(G.xs + (int64_t)(q0 + i) * dp,
                                                   kRowsInLds ? &f64t[crow][0] : G.xs + (int64_t)(t + crow) * dp, d);
                        if (ex <= G.eps2) {
                            inm |= 1u << r;
                            ++band_in;
                        }
                        ++band;
                    }
                }
            }
            if (MODE == MODE_EMIT) {
                unsigned long long bal[4];
                int base_e = 0;
                int pre[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    bal[r] = __ballot(emit_r[r] && ((inm >> r) & 1u));
                    pre[r] = base_e + __popcll(bal[r] & lt);
                    base_e += __popcll(bal[r]);
                }
                if (base_e) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (emit_r[r] && ((inm >> r) & 1u)) {
                            const int e = (tail + pre[r]) & (kRing - 1);
                            rcand[e] = (uint32_t)(t + crow);
                            rrel[e] = (uint32_t)(cur[r] + __popcll(bal[r] & lt & grp));
                            rcol[e] = (uint32_t)(4 * g + r);
                        }
                    }
                    tail += base_e;
#pragma unroll
                    for (int r = 0; r < 4; ++r) cur[r] += __popcll(bal[r] & grp);
                    while (tail - head >= 64) flush(64);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) cnt[r] += (inm >> r) & 1u;
                if (rec) mword |= (unsigned long long)inm << (4 * (4 * (tcur & 3) + sub));
            }
        }
        if (rec && ((tcur & 3) == 3 || !have)) {  // the group's last tile, or the list's
            R.masks[mbase + (int64_t)(tcur >> 2) * (kWaves * 64) + lane] = mword;
            mword = 0;
        }
    }
    if (MODE == MODE_EMIT && has_q && tail > head) flush(tail - head);
    if (MODE == MODE_COUNT && has_q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int v = cnt[r];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            if (j == 0 && 4 * g + r < nq) R.cnt[q0 + 4 * g + r] = v;
        }
    }
    for (int sh = 32; sh > 0; sh >>= 1) {
        band += __shfl_xor(band, sh);
        band_in += __shfl_xor(band_in, sh);
        if (MODE == MODE_MEASURE) {
            viol += __shfl_xor(viol, sh);
            maxerr = fmax(maxerr, __shfl_xor(maxerr, sh));
        }
        maxdelta = fmax(maxdelta, __shfl_xor(maxdelta, sh));
    }
    if (lane == 0) {
        if (band) {
            atomicAdd(&R.ctr->rechecked, band);
            atomicAdd(&R.ctr->rechecked_in, band_in);
        }
        if (MODE == MODE_MEASURE) {
            atomicMax(&R.ctr->max_err, (unsigned long long)__double_as_longlong(maxerr));
            if (viol) atomicAdd(&R.ctr->violations, viol);
        }
        atomicMax(&R.ctr->max_delta, (unsigned long long)__double_as_longlong(maxdelta));
    }
}

LpGrid lp_grid(const Grid &g) {
    LpGrid G;
    G.xs = g.xs;
    G.nrm = g.nrm;
    G.perm = g.perm;
    G.ranges = g.ranges;
    G.items = g.item;
    G.blocks = g.blocks;
    G.nblocks = (int32_t)g.nblocks;
    G.d = g.d;
    G.dp = g.dp;
    G.nranges = g.nranges;
    G.eps2 = g.eps2;
    G.sc = lowp_scale(g);
    G.eps_s = g.eps * G.sc;
    G.eps2_s = g.eps2 * G.sc * G.sc;
    return G;
}

template <int MODE>
void launch_lowp(const Grid &g, sj_path path, const LpOut &R, int nblocks, hipStream_t s) {
    if (g.d > kLpMaxD) throw Unsupported{"FP32/BF16 MFMA paths support d <= 64"};
    if (nblocks <= 0) return;
    const LpGrid G = lp_grid(g);
    if (path == SJ_FP32_MFMA)
        hipLaunchKernelGGL((k_lowp<PREC_F32, MODE>), dim3(nblocks), dim3(kThreads), 0, s, G, R);
    else if (path == SJ_BF16_MFMA)
        hipLaunchKernelGGL((k_lowp<PREC_BF16, MODE>), dim3(nblocks), dim3(kThreads), 0, s, G, R);
    else if (path == SJ_FP8_MFMA)
        hipLaunchKernelGGL((k_lowp<PREC_FP8, MODE>), dim3(nblocks), dim3(kThreads), 0, s, G, R);
    else
        hipLaunchKernelGGL((k_lowp<PREC_BF16X3, MODE>), dim3(nblocks), dim3(kThreads), 0, s, G, R);
    SJ_HIP(hipGetLastError());
}

}  // namespace

double lowp_scale(const Grid &g) { return std::ldexp(1.0, -std::ilogb(g.eps)); }

bool lowp_in_range(const Grid &g, sj_path path) {
    if (!(g.eps >= 0x1p-500 && g.eps <= 0x1p500)) return false;
    // FP8: scaled centred values (|y| < 2 extent / eps) and -2y stay below 448
    const double lim = path == SJ_FP8_MFMA ? 100.0 * g.eps : std::ldexp(g.eps, 40);
    for (int j = 0; j < g.d; ++j)
        if (!(g.hi[j] - g.lo[j] <= lim)) return false;  // also false for an infinite extent
    return true;
}

namespace {

// The in-mask layout of a grid (once per grid: it depends only on the block
// items and their ranges): groups per block item, their exclusive prefix
// (one host sync for the total), and the buffer if it fits the budget.
void lp_mask_layout(Grid &g, hipStream_t s) {
    if (g.lp_groups >= 0) return;
    const int64_t nb = g.nblocks;
    g.lp_goff = dev_alloc_n<int64_t>((size_t)nb + 1, s);
    int32_t *groups = dev_alloc_n<int32_t>((size_t)nb + 1, s);
    fill_zero(groups + nb, sizeof(int32_t), s);  // the scan's last entry: the total
    if (nb > 0) {
        hipLaunchKernelGGL(k_lp_groups, dim3((unsigned)((nb + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                           lp_grid(g), groups);
        SJ_HIP(hipGetLastError());
    }
    exclusive_scan_i32_to_i64(groups, g.lp_goff, nb + 1, s);
    int64_t total = 0;
    SJ_HIP(hipMemcpyAsync(&total, g.lp_goff + nb, sizeof total, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    dev_free(groups, s);
    g.lp_groups = total;
    const int64_t bytes = total * kWaves * 64 * (int64_t)sizeof(unsigned long long);
    if (total > 0 && bytes <= kMaskBudget) g.lp_masks = dev_alloc_n<unsigned long long>((size_t)bytes / 8, s);
}

}  // namespace

// Count: per-query counts into cnt_sorted; counters (band half-widths in
// the tiles' scaled units) in ro.ctr, zeroed here. With ro.record_lp the
// pass records its in-masks on the grid (g.lp_masks, if they fit).
void lowp_count(Grid &g, sj_path path, int32_t *cnt_sorted, RefineOut &ro, hipStream_t s) {
    if (ro.record_lp) lp_mask_layout(g, s);
    fill_zero(ro.ctr, sizeof(DevCounters), s);
    LpOut R{};
    R.cnt = cnt_sorted;
    R.ctr = ro.ctr;
    R.block_lo = 0;
    R.masks = ro.record_lp ? g.lp_masks : nullptr;
    R.goff = g.lp_goff;
    ro.kt.start(ro.timed, s);
    launch_lowp<MODE_COUNT>(g, path, R, (int)g.nblocks, s);
    ro.kt.stop(s);
}

void lowp_pairs(Grid &g, sj_path path, const ChunkPlan &p, int64_t qlo, int32_t *pairs, double *d2, RefineOut &ro,
                hipStream_t s) {
    // block items covering the chunk's work items
    LpOut R{};
    R.off = g.off;
    R.base = p.base;
    R.qlo = (int32_t)qlo;
    R.qhi = (int32_t)p.next;
    R.pairs = pairs;
    R.d2 = d2;
    R.ctr = ro.ctr;
    fill_zero(ro.ctr, sizeof(DevCounters), s);
    R.block_lo = (int32_t)p.block_lo;
    ro.kt.start(ro.timed, s);
    if (g.lp_masks_valid && g.lp_masks) {  // expand the count's in-masks
        R.masks = g.lp_masks;
        R.goff = g.lp_goff;
        launch_lowp<MODE_MASKEMIT>(g, path, R, (int)(p.block_hi - p.block_lo), s);
    } else {
        launch_lowp<MODE_EMIT>(g, path, R, (int)(p.block_hi - p.block_lo), s);
    }
    ro.kt.stop(s);
}

void lowp_measure(Grid &g, sj_path path, double *max_err, double *max_band, int64_t *viol, hipStream_t s) {
    DevCounters *ctr = dev_alloc_n<DevCounters>(1, s);
    fill_zero(ctr, sizeof(DevCounters), s);
    LpOut R{};
    R.ctr = ctr;
    R.block_lo = 0;
    launch_lowp<MODE_MEASURE>(g, path, R, (int)g.nblocks, s);
    DevCounters h{};
    SJ_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    dev_free(ctr, s);
    const HostCounters hc = read_counters(h);
    const double sc = lowp_scale(g);  // back to the data's units
    *max_err = hc.max_err / (sc * sc);
    *max_band = hc.max_delta / (sc * sc);
    *viol = hc.violations;
}

}  // namespace sj

/*
 * selfjoin_oracle.c -- plain CPU reference for the epsilon-distance self-join.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do. It shares no code, header or constant with the GPU path.
 *
 * What it computes (Gallet & Gowanlock, "Leveraging GPU Tensor Cores for Double
 * Precision Euclidean Distance Calculations"):
 *   - Section II-A, Eq. (1): the Euclidean distance; the self-join of a set V
 *     with a search distance eps is every pair (a, b) of V x V whose distance is
 *     at most eps, i.e. one range query per point of V.
 *   - Section III-A, Eq. (2): the squared distance is a chain of
 *     multiply-accumulate steps, dimension 1 first, starting from 0. Here every
 *     step is one correctly rounded fused multiply-add of the coordinate
 *     difference with itself onto the running sum.
 *   - Section IV-A (selectivity): the result set contains each point paired
 *     with itself, and pairs are ordered, (a, b) and (b, a) both present.
 * Readings where the paper is silent: the test is on the squared distance,
 * d2 <= fl(eps * eps), no square root; duplicates at distinct indices pair.
 *
 * Three independent routines:
 *   oracle_bruteforce  - all n^2 ordered pairs, the definition written out.
 *   oracle_query       - one range query by brute force (for sampled checks at
 *                        sizes where n^2 is out of reach).
 *   oracle_grid_*      - the same set through a uniform grid whose cells have
 *                        side eps (Section II-D "search" then "refine";
 *                        Section III-B, the grid of cells of size eps^d whose
 *                        neighbouring cells hold every candidate). Pinned to
 *                        the brute force by the tests. oracle_grid_digest
 *                        adds two order-independent checksums of the pair
 *                        set, so that results too large to store can be
 *                        compared whole.
 *
 * Grid readings (the paper gives cell side eps, not origin or rounding):
 * origin = per-dimension minimum; cell side w = eps * (1 + 2^-19) so that the
 * rounded cell coordinates of two points within eps differ by at most one
 * (with w = eps exactly a pair eps apart along an axis can land two cells
 * apart); the top cell is clamped; k = min(d, 4) leading dimensions are
 * indexed (Section II-D: indexing fewer dimensions than d), fewer if the cell
 * count would not fit in 62 bits. The grid also yields C_ref, the number of
 * ordered candidate pairs in the full 3^k stencil, the implementation-free
 * unit of work used to report distance evaluations per second.
 *
 * Build: gcc -O2 -ffp-contract=off (no contraction: every rounding is explicit).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_KMAX 4

/* Eq. (1) squared, in the accumulation order of Eq. (2). */
double oracle_d2(const double *a, const double *b, int d)
{
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double delta = a[t] - b[t];
        acc = fma(delta, delta, acc);
    }
    return acc;
}

double oracle_eps2(double eps) { return eps * eps; }

static int valid_input(const double *X, int64_t n, int d, double eps)
{
    if (n < 0 || d < 1 || !(eps > 0.0) || !isfinite(eps)) return 0;
    if (n > 0 && X == NULL) return 0;
    for (int64_t i = 0; i < n * (int64_t)d; ++i)
        if (!isfinite(X[i])) return 0;
    return 1;
}

/* Brute force: every ordered pair (i, j), i and j ascending. Returns |R| or -1
 * on invalid input. per_point (n entries) and pairs (cap x 2, row (i, j)) may
 * be NULL; pairs beyond cap are counted but not written. */
int64_t oracle_bruteforce(const double *X, int64_t n, int d, double eps,
                          int32_t *per_point, int32_t *pairs, int64_t cap)
{
    if (!valid_input(X, n, d, eps)) return -1;
    const double eps2 = eps * eps;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (oracle_d2(X + i * d, X + j * d, d) <= eps2) {
                if (pairs && total < cap) {
                    pairs[2 * total] = (int32_t)i;
                    pairs[2 * total + 1] = (int32_t)j;
                }
                ++cnt;
                ++total;
            }
        }
        if (per_point) per_point[i] = cnt;
    }
    return total;
}

/* One range query by brute force: the indices j (ascending) with
 * d2(q, j) <= eps2. Returns the count or -1. */
int64_t oracle_query(const double *X, int64_t n, int d, double eps, int64_t q,
                     int32_t *js, int64_t cap)
{
    if (n < 0 || d < 1 || !(eps > 0.0) || !isfinite(eps) || q < 0 || q >= n) return -1;
    const double eps2 = eps * eps;
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (oracle_d2(X + q * d, X + j * d, d) <= eps2) {
            if (js && cnt < cap) js[cnt] = (int32_t)j;
            ++cnt;
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Grid self-join                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t key;
    int32_t idx;
} keyed_t;

typedef struct {
    const double *X;
    int64_t n;
    int d, k;
    double eps2;
    int64_t m[ORACLE_KMAX];      /* cells per indexed dimension */
    int64_t stride[ORACLE_KMAX]; /* key = sum c_j * stride_j, last indexed dim fastest */
    keyed_t *sorted;             /* points sorted by (key, idx) */
    int64_t ncells;
    int64_t *cell_key, *cell_start, *cell_count;
} grid_t;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

double oracle_cell_side(double eps) { return eps * (1.0 + 0x1p-19); }

/* Builds the reference grid. Returns 0 on success. */
static int grid_build(grid_t *g, const double *X, int64_t n, int d, double eps)
{
    memset(g, 0, sizeof *g);
    g->X = X;
    g->n = n;
    g->d = d;
    g->eps2 = eps * eps;
    const double w = oracle_cell_side(eps);
    double lo[ORACLE_KMAX], hi[ORACLE_KMAX];
    int k = d < ORACLE_KMAX ? d : ORACLE_KMAX;
    for (int j = 0; j < k; ++j) {
        lo[j] = INFINITY;
        hi[j] = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            double v = X[i * d + j];
            if (v < lo[j]) lo[j] = v;
            if (v > hi[j]) hi[j] = v;
        }
        if (n == 0) lo[j] = hi[j] = 0.0;
    }
    /* Cells per dimension (counted in double: an extent of 2^63 cells or more
     * must not wrap); drop trailing indexed dimensions until the total cell
     * count fits in 62 bits. If the first dimension alone needs 2^62 cells or
     * more, the grid is a single cell: every pair is a candidate. */
    double mc[ORACLE_KMAX];
    for (;;) {
        double prod = 1.0;
        for (int j = 0; j < k; ++j) {
            mc[j] = floor((hi[j] - lo[j]) / w) + 1.0;
            prod *= mc[j];
        }
        if (prod < 0x1p62 || k == 1) break;
        --k;
    }
    if (!(mc[0] < 0x1p62)) mc[0] = 1.0;
    for (int j = 0; j < k; ++j) g->m[j] = (int64_t)mc[j];
    g->k = k;
    int64_t s = 1;
    for (int j = k - 1; j >= 0; --j) {
        g->stride[j] = s;
        s *= g->m[j];
    }
    g->sorted = (keyed_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed_t));
    if (!g->sorted) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t key = 0;
        for (int j = 0; j < k; ++j) {
            /* clamped in double before the conversion, so no value (an
             * infinite quotient included) is converted out of range */
            double q = floor((X[i * d + j] - lo[j]) / w);
            if (!(q >= 0.0)) q = 0.0;
            if (q > (double)(g->m[j] - 1)) q = (double)(g->m[j] - 1);
            key += (int64_t)q * g->stride[j];
        }
        g->sorted[i].key = key;
        g->sorted[i].idx = (int32_t)i;
    }
    qsort(g->sorted, (size_t)n, sizeof(keyed_t), cmp_keyed);
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || g->sorted[i].key != g->sorted[i - 1].key) ++nc;
    g->ncells = nc;
    g->cell_key = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    g->cell_start = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    g->cell_count = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    if (!g->cell_key || !g->cell_start || !g->cell_count) return -1;
    nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || g->sorted[i].key != g->sorted[i - 1].key) {
            g->cell_key[nc] = g->sorted[i].key;
            g->cell_start[nc] = i;
            g->cell_count[nc] = 0;
            ++nc;
        }
        g->cell_count[nc - 1]++;
    }
    return 0;
}

static void grid_free(grid_t *g)
{
    free(g->sorted);
    free(g->cell_key);
    free(g->cell_start);
    free(g->cell_count);
}

/* Index of the cell with this key, or -1. */
static int64_t find_cell(const grid_t *g, int64_t key)
{
    int64_t a = 0, b = g->ncells;
    while (a < b) {
        int64_t mid = a + (b - a) / 2;
        if (g->cell_key[mid] < key) a = mid + 1;
        else b = mid;
    }
    return (a < g->ncells && g->cell_key[a] == key) ? a : -1;
}

/* Visits the neighbouring cells of cell ci (all 3^k offsets, itself included)
 * and returns them in out[] (at most 3^k entries). */
static int neighbours(const grid_t *g, int64_t ci, int64_t *out)
{
    int64_t c[ORACLE_KMAX];
    int64_t key = g->cell_key[ci];
    for (int j = 0; j < g->k; ++j) {
        c[j] = key / g->stride[j];
        key -= c[j] * g->stride[j];
    }
    int total = 1;
    for (int j = 0; j < g->k; ++j) total *= 3;
    int cnt = 0;
    for (int o = 0; o < total; ++o) {
        int rem = o, ok = 1;
        int64_t nkey = 0;
        for (int j = 0; j < g->k; ++j) {
            int64_t cj = c[j] + (rem % 3) - 1;
            rem /= 3;
            if (cj < 0 || cj >= g->m[j]) { ok = 0; break; }
            nkey += cj * g->stride[j];
        }
        if (!ok) continue;
        int64_t ni = find_cell(g, nkey);
        if (ni >= 0) out[cnt++] = ni;
    }
    return cnt;
}

/* Order-independent checksums of a pair set (test bookkeeping, not part of
 * the self-join): two pair lists of hundreds of millions of pairs are compared
 * through the sums, modulo 2^64, of mix(key) and mix(key + G) over their pairs
 * (i, j), key = i * 2^32 + j, G = 0x9e3779b97f4a7c15, where mix is the 64-bit
 * finaliser of SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014). Sums do not depend on the
 * order of the pairs or on how the list is split into chunks. */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static void digest_add(uint64_t sums[2], int32_t i, int32_t j)
{
    const uint64_t key = ((uint64_t)(uint32_t)i << 32) | (uint64_t)(uint32_t)j;
    sums[0] += mix64(key);
    sums[1] += mix64(key + 0x9e3779b97f4a7c15ull);
}

/* Checksums of an explicit pair list (rows (i, j)), for the tests. */
void oracle_pairs_digest(const int32_t *pairs, int64_t npairs, uint64_t *sums)
{
    sums[0] = sums[1] = 0;
    for (int64_t p = 0; p < npairs; ++p) digest_add(sums, pairs[2 * p], pairs[2 * p + 1]);
}

typedef struct {
    const grid_t *g;
    int tid, nthreads;
    int32_t *per_point;
    int64_t total, cref;
    int digest;       /* also accumulate the pair checksums */
    uint64_t sums[2];
} count_job_t;

static void *count_worker(void *arg)
{
    count_job_t *job = (count_job_t *)arg;
    const grid_t *g = job->g;
    const int d = g->d;
    int64_t nb[81];
    for (int64_t ci = job->tid; ci < g->ncells; ci += job->nthreads) {
        int nn = neighbours(g, ci, nb);
        int64_t cand = 0;
        for (int t = 0; t < nn; ++t) cand += g->cell_count[nb[t]];
        job->cref += g->cell_count[ci] * cand;
        for (int64_t a = g->cell_start[ci]; a < g->cell_start[ci] + g->cell_count[ci]; ++a) {
            const int32_t qi = g->sorted[a].idx;
            const double *xq = g->X + (int64_t)qi * d;
            int32_t cnt = 0;
            for (int t = 0; t < nn; ++t) {
                int64_t ni = nb[t];
                for (int64_t b = g->cell_start[ni]; b < g->cell_start[ni] + g->cell_count[ni]; ++b) {
                    const double *xc = g->X + (int64_t)g->sorted[b].idx * d;
                    if (oracle_d2(xq, xc, d) <= g->eps2) {
                        ++cnt;
                        if (job->digest) digest_add(job->sums, qi, g->sorted[b].idx);
                    }
                }
            }
            if (job->per_point) job->per_point[qi] = cnt;
            job->total += cnt;
        }
    }
    return NULL;
}

static int64_t grid_count_impl(const double *X, int64_t n, int d, double eps, int nthreads,
                               int32_t *per_point, int64_t *cref, int *kdims, uint64_t *sums);

/* Grid self-join, count only. per_point (n, original order) may be NULL.
 * cref (nullable) receives C_ref; kdims (nullable) the indexed dimension
 * count. Threads split the query cells. Returns |R| or -1. */
int64_t oracle_grid_count(const double *X, int64_t n, int d, double eps, int nthreads,
                          int32_t *per_point, int64_t *cref, int *kdims)
{
    return grid_count_impl(X, n, d, eps, nthreads, per_point, cref, kdims, NULL);
}

/* As oracle_grid_count, plus the two pair checksums of R (see mix64) in
 * sums[0..1]. */
int64_t oracle_grid_digest(const double *X, int64_t n, int d, double eps, int nthreads,
                           int32_t *per_point, int64_t *cref, int *kdims, uint64_t *sums)
{
    return grid_count_impl(X, n, d, eps, nthreads, per_point, cref, kdims, sums);
}

static int64_t grid_count_impl(const double *X, int64_t n, int d, double eps, int nthreads,
                               int32_t *per_point, int64_t *cref, int *kdims, uint64_t *sums)
{
    if (!valid_input(X, n, d, eps) || n >= ((int64_t)1 << 31)) return -1;
    grid_t g;
    if (grid_build(&g, X, n, d, eps) != 0) { grid_free(&g); return -1; }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    count_job_t jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].g = &g;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
        jobs[t].per_point = per_point;
        jobs[t].total = 0;
        jobs[t].cref = 0;
        jobs[t].digest = sums != NULL;
        jobs[t].sums[0] = jobs[t].sums[1] = 0;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, count_worker, &jobs[t]);
    count_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    int64_t total = 0, cr = 0;
    uint64_t s0 = 0, s1 = 0;
    for (int t = 0; t < nthreads; ++t) {
        total += jobs[t].total;
        cr += jobs[t].cref;
        s0 += jobs[t].sums[0];
        s1 += jobs[t].sums[1];
    }
    if (sums) {
        sums[0] = s0;
        sums[1] = s1;
    }
    if (cref) *cref = cr;
    if (kdims) *kdims = g.k;
    grid_free(&g);
    return total;
}

/* Grid self-join with the pair list (single thread). Pairs (original indices)
 * are written as rows (i, j) up to cap, in cell-sorted query order; per_point
 * and d2 (the squared distance of each written pair) may be NULL. Returns |R|
 * or -1. */
int64_t oracle_grid_pairs(const double *X, int64_t n, int d, double eps,
                          int32_t *per_point, int32_t *pairs, double *d2, int64_t cap)
{
    if (!valid_input(X, n, d, eps) || n >= ((int64_t)1 << 31)) return -1;
    grid_t g;
    if (grid_build(&g, X, n, d, eps) != 0) { grid_free(&g); return -1; }
    int64_t nb[81];
    int64_t total = 0;
    for (int64_t ci = 0; ci < g.ncells; ++ci) {
        int nn = neighbours(&g, ci, nb);
        for (int64_t a = g.cell_start[ci]; a < g.cell_start[ci] + g.cell_count[ci]; ++a) {
            const int32_t qi = g.sorted[a].idx;
            const double *xq = X + (int64_t)qi * d;
            int32_t cnt = 0;
            for (int t = 0; t < nn; ++t) {
                int64_t ni = nb[t];
                for (int64_t b = g.cell_start[ni]; b < g.cell_start[ni] + g.cell_count[ni]; ++b) {
                    const int32_t cj = g.sorted[b].idx;
                    const double v = oracle_d2(xq, X + (int64_t)cj * d, d);
                    if (v <= g.eps2) {
                        if (total < cap) {
                            if (pairs) {
                                pairs[2 * total] = qi;
                                pairs[2 * total + 1] = cj;
                            }
                            if (d2) d2[total] = v;
                        }
                        ++total;
                        ++cnt;
                    }
                }
            }
            if (per_point) per_point[qi] = cnt;
        }
    }
    grid_free(&g);
    return total;
}

/* Sampled counts: for each listed query index, its count through the grid
 * (one grid build, then only the listed queries). Used to time the CPU
 * baseline on a bounded sample and to check per-point counts at full size.
 * Also returns the candidates those queries see (C_ref restricted to them). */
int64_t oracle_grid_count_sample(const double *X, int64_t n, int d, double eps,
                                 const int64_t *queries, int64_t nq,
                                 int32_t *counts, int64_t *cref_sample)
{
    if (!valid_input(X, n, d, eps) || n >= ((int64_t)1 << 31)) return -1;
    grid_t g;
    if (grid_build(&g, X, n, d, eps) != 0) { grid_free(&g); return -1; }
    /* position of each point in the sorted order -> its cell */
    int64_t *cell_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!cell_of) { grid_free(&g); return -1; }
    for (int64_t ci = 0; ci < g.ncells; ++ci)
        for (int64_t a = g.cell_start[ci]; a < g.cell_start[ci] + g.cell_count[ci]; ++a)
            cell_of[g.sorted[a].idx] = ci;
    int64_t nb[81];
    int64_t total = 0, cr = 0;
    for (int64_t s = 0; s < nq; ++s) {
        int64_t qi = queries[s];
        if (qi < 0 || qi >= n) { total = -1; break; }
        int nn = neighbours(&g, cell_of[qi], nb);
        const double *xq = X + qi * d;
        int32_t cnt = 0;
        for (int t = 0; t < nn; ++t) {
            int64_t ni = nb[t];
            cr += g.cell_count[ni];
            for (int64_t b = g.cell_start[ni]; b < g.cell_start[ni] + g.cell_count[ni]; ++b)
                if (oracle_d2(xq, X + (int64_t)g.sorted[b].idx * d, d) <= g.eps2) ++cnt;
        }
        if (counts) counts[s] = cnt;
        total += cnt;
    }
    if (cref_sample) *cref_sample = cr;
    free(cell_of);
    grid_free(&g);
    return total;
}

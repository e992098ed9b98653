"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exact rational arithmetic, lattice closed forms, Gauss-circle counts, an
independent one-dimensional sweep, brute force on small inputs, exact
invariants of the self-join, and the expected selectivity of uniform data.

Definitions followed: Section II-A Eq. (1) (distance and self-join), Section
III-A Eq. (2) (dimension-ascending multiply-accumulate from 0), Section IV-A
(selectivity s = (|R| - |V|) / |V|, so each point pairs with itself).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import generators as gen


# --------------------------------------------------------------------------
# The squared-distance chain
# --------------------------------------------------------------------------

def _chain_exact(a, b):
    """Eq. (2) with one rounding per multiply-accumulate step, evaluated with
    exact rationals: delta = fl(a - b) (IEEE subtraction, done by Python
    floats), then acc = round(delta * delta + acc) with the rounding of
    Fraction -> float (correctly rounded, ties to even)."""
    acc = 0.0
    for x, y in zip(a, b):
        delta = x - y
        acc = float(Fraction(delta) * Fraction(delta) + Fraction(acc))
    return acc


def _chain_unfused(a, b):
    acc = 0.0
    for x, y in zip(a, b):
        delta = x - y
        acc = acc + delta * delta
    return acc


def test_d2_is_fused_chain_exactly():
    rng = np.random.default_rng(1)
    differs_from_unfused = 0
    for trial in range(3000):
        d = int(rng.integers(1, 12))
        scale = 10.0 ** rng.integers(-6, 4)
        a = rng.random(d) * scale
        b = a + (rng.random(d) - 0.5) * scale * 1e-2
        got = oracle.d2(a, b)
        assert got == _chain_exact(a, b), (trial, a, b)
        assert got == oracle.d2(b, a)  # fl(a-b) = -fl(b-a): bitwise symmetric
        if got != _chain_unfused(a, b):
            differs_from_unfused += 1
    # the check has teeth: plain multiply-then-add rounds differently here
    assert differs_from_unfused > 50


def test_d2_accumulates_in_ascending_dimension_order():
    # Dimension 1 first (Eq. 2). Reversed accumulation gives another value here.
    a = np.array([1.0, 2.0 ** -27, 2.0 ** -27, 2.0 ** -27])
    b = np.zeros(4)
    asc = oracle.d2(a, b)
    assert asc == _chain_exact(a, b)
    assert asc == 1.0  # each 2^-54 is absorbed by the leading 1.0
    assert _chain_exact(a[::-1], b[::-1]) != asc
    assert oracle.d2(np.zeros(3), np.zeros(3)) == 0.0
    assert math.copysign(1.0, oracle.d2(np.zeros(2), np.zeros(2))) == 1.0  # +0.0


def test_eps2_single_rounding():
    for e in [0.0218, 0.1, 1e-3, 3.3, 2.0 ** -6 * 3]:
        assert oracle.eps2(e) == float(Fraction(e) * Fraction(e))


# --------------------------------------------------------------------------
# Closed forms on a lattice (all arithmetic exact)
# --------------------------------------------------------------------------

def _lattice_count(L, d, r):
    """#R for the points {0..L-1}^d: number of ordered (p, q) with
    |p - q|^2 <= r^2 = sum over integer offsets v with |v|^2 <= r^2 of the
    number of lattice points p with p + v also in the lattice, i.e.
    prod_j max(0, L - |v_j|). Evaluated as the coefficients of degree <= r^2 of
    (sum_x max(0, L - |x|) z^(x^2))^d."""
    R2 = r * r
    one = [0] * (R2 + 1)
    for x in range(-min(r, L - 1), min(r, L - 1) + 1):
        one[x * x] += L - abs(x)
    poly = [1] + [0] * R2
    for _ in range(d):
        nxt = [0] * (R2 + 1)
        for i, a in enumerate(poly):
            if a:
                for j, b in enumerate(one):
                    if b and i + j <= R2:
                        nxt[i + j] += a * b
        poly = nxt
    return sum(poly)


def _lattice_count_enum(L, d, r):
    total = 0
    for v in itertools.product(range(-r, r + 1), repeat=d):
        if sum(x * x for x in v) <= r * r:
            total += math.prod(max(0, L - abs(x)) for x in v)
    return total


def test_lattice_closed_form_known_value():
    # d = 2, L = 10, r = 1: the 100 self-pairs plus 4 axis directions x 90.
    assert _lattice_count(10, 2, 1) == 100 + 4 * 90 == 460
    for L, d, r in [(10, 2, 1), (5, 3, 2), (4, 4, 2), (7, 2, 5)]:
        assert _lattice_count(L, d, r) == _lattice_count_enum(L, d, r)


@pytest.mark.parametrize("L,d,r", [(10, 2, 1), (12, 2, 2), (9, 2, 3), (6, 3, 1), (6, 3, 2),
                                   (5, 4, 1), (4, 4, 2), (3, 5, 2), (40, 1, 3), (3, 6, 2),
                                   (2, 10, 2), (2, 10, 3)])
def test_lattice_matches_closed_form(L, d, r):
    h = 2.0 ** -6
    X = gen.lattice(L, d, h)
    eps = r * h  # exact, and every lattice distance is exact: ties sit on eps
    want = _lattice_count(L, d, r)
    cnt_bf, pp_bf, _ = oracle.bruteforce(X, eps, want_pairs=False)
    cnt_g, pp_g, _, _ = oracle.grid_count(X, eps, nthreads=3)
    assert cnt_bf == want
    assert cnt_g == want
    assert np.array_equal(pp_bf, pp_g)


@pytest.mark.parametrize("d,r,want", [(2, 1, 5), (2, 2, 13), (2, 3, 29), (3, 1, 7), (3, 2, 33),
                                      (4, 1, 9)])
def test_gauss_circle_interior_counts(d, r, want):
    # Number of integer points in the closed ball of radius r (Gauss circle /
    # sphere problem): 5, 13, 29 in the plane; 7, 33 in space; 9 in 4-D.
    L = 2 * r + 3
    h = 2.0 ** -6
    X = gen.lattice(L, d, h)
    centre = int(np.flatnonzero(np.all(X == (r + 1) * h, axis=1))[0])
    js = oracle.query(X, r * h, centre)
    assert len(js) == want
    _, pp, _, _ = oracle.grid_count(X, r * h)
    assert pp[centre] == want


# --------------------------------------------------------------------------
# Independent one-dimensional sweep
# --------------------------------------------------------------------------

def _sweep_1d_counts(x, eps):
    """Sort, then two pointers: for d = 1 the test fl(delta^2) <= fl(eps^2) is
    monotone in |delta|, so each query's neighbours form a window of the
    sorted order. Independent of grids and of the oracle's loops."""
    e2 = eps * eps
    order = np.argsort(x, kind="stable")
    xs = x[order]
    n = len(xs)
    counts = np.zeros(n, dtype=np.int64)
    lo = 0
    hi = 0
    for i in range(n):
        while (xs[i] - xs[lo]) * (xs[i] - xs[lo]) > e2:
            lo += 1
        while hi + 1 < n and (xs[hi + 1] - xs[i]) * (xs[hi + 1] - xs[i]) <= e2:
            hi += 1
        hi = max(hi, i)
        counts[order[i]] = hi - lo + 1
    return counts


@pytest.mark.parametrize("dist,eps", [("uniform", 0.001), ("expo", 0.0005), ("uniform", 0.02)])
def test_d1_sweep_equals_grid_and_bruteforce(dist, eps):
    X = gen.make(dist, 3000, 1, seed=5)
    # snap some points onto an eps-spaced ladder to create exact ties
    X[:200, 0] = np.arange(200) * eps
    want = _sweep_1d_counts(X[:, 0].copy(), eps)
    _, pp_bf, _ = oracle.bruteforce(X, eps, want_pairs=False)
    _, pp_g, _, _ = oracle.grid_count(X, eps)
    assert np.array_equal(pp_bf, want)
    assert np.array_equal(pp_g, want)


# --------------------------------------------------------------------------
# Grid join == brute force (exact pair sets)
# --------------------------------------------------------------------------

def _pairset(pairs):
    p = np.asarray(pairs, dtype=np.int64)
    return np.sort(p[:, 0] << 32 | p[:, 1])


CASES = []
for _d in (1, 2, 3, 4, 5, 8, 16, 64):
    for _dist in ("uniform", "expo", "gmm"):
        CASES.append((_dist, _d))


def _eps_for(X, target_s):
    """A search distance with roughly target_s neighbours, from the brute-force
    distance distribution of a few queries (test inputs only)."""
    n = X.shape[0]
    rng = np.random.default_rng(7)
    qs = rng.integers(0, n, 40)
    dd = np.sort(np.concatenate([np.sqrt(((X - X[q]) ** 2).sum(1)) for q in qs]))
    return float(dd[min(len(dd) - 1, int(len(qs) * (target_s + 1)))])


@pytest.mark.parametrize("dist,d", CASES)
def test_grid_pairs_equal_bruteforce(dist, d):
    n = 1500 if d <= 8 else 800
    X = gen.make(dist, n, d, seed=d)
    eps = _eps_for(X, 12)
    cnt_bf, pp_bf, pairs_bf = oracle.bruteforce(X, eps)
    cnt_g, pp_g, pairs_g = oracle.grid_pairs(X, eps)
    assert cnt_bf == cnt_g
    assert np.array_equal(pp_bf, pp_g)
    assert np.array_equal(_pairset(pairs_bf), _pairset(pairs_g))


def test_grid_adversarial_sets():
    rng = np.random.default_rng(3)
    sets = []
    # duplicates (distinct indices, identical coordinates)
    base = rng.random((300, 3))
    sets.append((np.concatenate([base, base, base[:50]]), 0.05))
    # collinear points on a line of slope 1 in 2-D
    t = np.sort(rng.random(500))
    sets.append((np.stack([t, t], 1), 0.01))
    # points exactly on cell faces: multiples of eps
    e = 0.125
    sets.append((rng.integers(0, 8, (600, 2)).astype(np.float64) * e, e))
    # non-dyadic eps with coordinates at multiples of 0.1
    sets.append((rng.integers(0, 10, (700, 3)).astype(np.float64) * 0.1, 0.1))
    # large offset and tiny spread
    sets.append((1e6 + rng.random((500, 2)) * 1e-3, 1e-4))
    # negative coordinates, huge spread in one dimension
    Y = rng.random((600, 4)) - 0.5
    Y[:, 0] *= 1e4
    sets.append((Y, 0.2))
    for X, eps in sets:
        cnt_bf, pp_bf, pairs_bf = oracle.bruteforce(X, eps)
        cnt_g, pp_g, pairs_g = oracle.grid_pairs(X, eps)
        assert cnt_bf == cnt_g
        assert np.array_equal(_pairset(pairs_bf), _pairset(pairs_g))


def test_grid_extents_beyond_the_cell_count_range():
    # extent / eps of 1e19 (more cells than an int64 holds) or infinite
    # (max - min overflows): the grid drops indexed dimensions, down to a
    # single cell, and stays equal to brute force
    sets = [np.array([[0.0, 0.0], [0.0, 1e20]]), np.array([[0.0, 0.0], [1e20, 0.0]]),
            np.array([[-1e308, 0.0], [1e308, 0.0], [1e308, 5.0]]),
            np.array([[0.0, 0.0], [1e20, 0.0], [1e20, 5.0], [3.0, 1e25]])]
    rng = np.random.default_rng(12)
    Y = rng.random((400, 3))
    Y[:7, 0] = [1e19, -1e19, 4e18, 1e300, -1e300, 2.5, 1e200]
    sets.append(Y)
    for X in sets:
        cb, pb, rb = oracle.bruteforce(X, 10.0 if X.shape[0] < 10 else 0.2)
        cg, pg, rg = oracle.grid_pairs(X, 10.0 if X.shape[0] < 10 else 0.2)
        assert cb == cg and np.array_equal(pb, pg)
        assert np.array_equal(_pairset(rb), _pairset(rg))


def test_cell_side_margin_is_needed():
    """With cells of side exactly eps, rounding of the cell coordinate can put a
    pair that is exactly eps apart two cells apart. Find such pairs with plain
    float64 arithmetic, then check the oracle's grid still reports them."""
    rng = np.random.default_rng(11)
    found = []
    for _ in range(200000):
        eps = float(rng.uniform(0.01, 0.3))
        lo = float(rng.uniform(-3, 0))
        x = lo + float(rng.integers(1, 200)) * eps - float(rng.integers(0, 4)) * 2.0 ** -50
        y = x + eps
        if (y - x) != eps or y - x > eps:
            continue
        cx = math.floor((x - lo) / eps)
        cy = math.floor((y - lo) / eps)
        if abs(cy - cx) >= 2:
            found.append((lo, x, y, eps))
        if len(found) >= 20:
            break
    assert found, "no adversarial case found"
    for lo, x, y, eps in found:
        X = np.array([[lo], [x], [y]])
        js = oracle.query(X, eps, 1)
        assert 2 in js  # brute force: the pair is within eps
        _, pp, _, _ = oracle.grid_count(X, eps)
        assert pp[1] == len(js)


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------

def test_invariants_symmetry_selfpairs_counts():
    X = gen.make("expo", 4000, 3, seed=2)
    eps = _eps_for(X, 20)
    cnt, pp, pairs = oracle.grid_pairs(X, eps)
    n = X.shape[0]
    assert cnt == len(pairs) == int(pp.sum())
    ps = set(map(tuple, pairs.tolist()))
    assert all((j, i) in ps for i, j in ps)
    assert all((i, i) in ps for i in range(n))
    assert np.array_equal(np.bincount(pairs[:, 0], minlength=n), pp)


def test_monotone_in_eps():
    X = gen.make("uniform", 3000, 2, seed=4)
    prev = None
    for eps in [0.005, 0.01, 0.02, 0.04]:
        _, _, pairs = oracle.grid_pairs(X, eps)
        s = set(map(tuple, pairs.tolist()))
        if prev is not None:
            assert prev <= s
        prev = s


def test_permutation_equivariance():
    X = gen.make("gmm", 2000, 8, seed=6)
    eps = _eps_for(X, 10)
    perm = np.random.default_rng(0).permutation(len(X))
    _, pp, pairs = oracle.grid_pairs(X, eps)
    _, pp2, pairs2 = oracle.grid_pairs(X[perm], eps)
    assert np.array_equal(pp2, pp[perm])
    inv = np.argsort(perm)
    mapped = np.stack([perm[pairs2[:, 0]], perm[pairs2[:, 1]]], 1)
    assert np.array_equal(_pairset(mapped), _pairset(pairs))
    del inv


@pytest.mark.parametrize("j", [-7, -1, 3, 10])
def test_power_of_two_scaling_invariance(j):
    X = gen.make("uniform", 2500, 3, seed=8)
    eps = 0.04
    _, pp, pairs = oracle.grid_pairs(X, eps)
    s = 2.0 ** j
    _, pp2, pairs2 = oracle.grid_pairs(X * s, eps * s)
    assert np.array_equal(pp, pp2)
    assert np.array_equal(_pairset(pairs), _pairset(pairs2))


def test_d2_output_of_pairs_is_the_chain():
    X = gen.make("uniform", 1000, 5, seed=9)
    eps = _eps_for(X, 8)
    _, _, pairs, dd = oracle.grid_pairs(X, eps, want_d2=True)
    for k in range(0, len(pairs), 97):
        i, j = pairs[k]
        assert dd[k] == _chain_exact(X[i], X[j])
        assert dd[k] <= oracle.eps2(eps)


# --------------------------------------------------------------------------
# C_ref: candidates of the full 3^k stencil, by an O(n^2) route
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dist,d", [("uniform", 2), ("expo", 3), ("uniform", 4), ("gmm", 6)])
def test_cref_counts_chebyshev_adjacent_pairs(dist, d):
    X = gen.make(dist, 1200, d, seed=1)
    eps = _eps_for(X, 10)
    _, _, cref, k = oracle.grid_count(X, eps)
    assert k == min(d, 4)
    w = oracle.cell_side(eps)
    lo = X[:, :k].min(0)
    hi = X[:, :k].max(0)
    m = np.floor((hi - lo) / w).astype(np.int64) + 1
    c = np.clip(np.floor((X[:, :k] - lo) / w).astype(np.int64), 0, m - 1)
    cheb = np.abs(c[:, None, :] - c[None, :, :]).max(-1)
    assert cref == int((cheb <= 1).sum())


# --------------------------------------------------------------------------
# Sampled counts: per-point counts of listed queries through the grid
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dist,d", [("uniform", 2), ("expo", 3), ("uniform", 4), ("gmm", 6), ("gmm", 16)])
def test_grid_count_sample_equals_full_count_and_bruteforce(dist, d):
    X = gen.make(dist, 1500, d, seed=d + 11)
    eps = _eps_for(X, 10)
    rng = np.random.default_rng(d)
    q = np.concatenate([rng.integers(0, X.shape[0], 200), [0, X.shape[0] - 1, 5, 5]])  # repeats allowed
    counts, cref_s = oracle.grid_count_sample(X, eps, q)
    _, pp_grid, _, k = oracle.grid_count(X, eps)
    _, pp_bf, _ = oracle.bruteforce(X, eps, want_pairs=False)
    assert np.array_equal(counts, pp_bf[q])
    assert np.array_equal(counts, pp_grid[q])
    # restricted C_ref: for each listed query, the points whose cells are
    # Chebyshev-adjacent (|dc| <= 1 on every indexed dimension) to its cell
    w = oracle.cell_side(eps)
    lo = X[:, :k].min(0)
    hi = X[:, :k].max(0)
    m = np.floor((hi - lo) / w).astype(np.int64) + 1
    c = np.clip(np.floor((X[:, :k] - lo) / w).astype(np.int64), 0, m - 1)
    adj = [(np.abs(c - c[i]).max(-1) <= 1).sum() for i in q]
    assert cref_s == int(np.sum(adj))


def test_grid_count_sample_lattice_ties():
    # every neighbour of an interior lattice point lies exactly on eps or
    # inside: d = 2, r = 2 gives the Gauss-circle number 13 in the interior
    h = 2.0 ** -6
    X = gen.lattice(12, 2, h)
    interior = [i for i in range(X.shape[0]) if (X[i] >= 2 * h).all() and (X[i] <= 9 * h).all()]
    counts, _ = oracle.grid_count_sample(X, 2 * h, interior)
    assert (counts == 13).all()


# --------------------------------------------------------------------------
# Pair-set checksums (test bookkeeping for results too large to store)
# --------------------------------------------------------------------------

_M1 = np.uint64(0xbf58476d1ce4e5b9)
_M2 = np.uint64(0x94d049bb133111eb)
_G = np.uint64(0x9e3779b97f4a7c15)


def _mix_np(z):
    """SplitMix64's 64-bit finaliser in numpy uint64 (wrapping arithmetic)."""
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _digest_np(pairs):
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    key = (p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64)
    with np.errstate(over="ignore"):
        a = int(np.sum(_mix_np(key), dtype=np.uint64))
        b = int(np.sum(_mix_np(key + _G), dtype=np.uint64))
    return a, b


def test_mix_matches_published_splitmix64_outputs():
    # SplitMix64 with seed 0: state += 0x9e3779b97f4a7c15, output = mix(state);
    # its first outputs are the published test values of the generator
    state = np.uint64(0)
    outs = []
    for _ in range(3):
        with np.errstate(over="ignore"):
            state = state + _G
        outs.append(int(_mix_np(np.array([state]))[0]))
    assert outs == [0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f]


@pytest.mark.parametrize("dist,d", [("uniform", 2), ("expo", 3), ("gmm", 8)])
def test_grid_digest_equals_digest_of_bruteforce_pairs(dist, d):
    X = gen.make(dist, 1200, d, seed=d + 3)
    eps = _eps_for(X, 9)
    cnt, pp, pairs = oracle.bruteforce(X, eps)
    tot, pp_g, cref, k, sums = oracle.grid_digest(X, eps, nthreads=3)
    assert tot == cnt and np.array_equal(pp_g, pp)
    assert sums == _digest_np(pairs)
    assert oracle.pairs_digest(pairs) == sums
    # order and chunking do not matter; one dropped or altered pair does
    perm = np.random.default_rng(0).permutation(len(pairs))
    assert oracle.pairs_digest(pairs[perm]) == sums
    half = len(pairs) // 2
    a, b = oracle.pairs_digest(pairs[:half]), oracle.pairs_digest(pairs[half:])
    assert ((a[0] + b[0]) % 2 ** 64, (a[1] + b[1]) % 2 ** 64) == sums
    assert oracle.pairs_digest(pairs[1:]) != sums
    bad = pairs.copy()
    bad[7, 1] ^= 1
    assert oracle.pairs_digest(bad) != sums
    # the same results as the plain grid count
    assert oracle.grid_count(X, eps, nthreads=2)[:1] == (tot,)


# --------------------------------------------------------------------------
# Statistical sanity on the small parity workload
# --------------------------------------------------------------------------

def test_uniform_selectivity_matches_pair_distance_cdf():
    # For two uniform points in the unit square, P(dist <= e) =
    # pi e^2 - 8 e^3 / 3 + e^4 / 2, so E[s] = (n - 1) P = 29.31 at n = 20000,
    # eps = 0.0218. Not exact: a 2% window.
    n, eps = 20000, 0.0218
    X = gen.uniform(n, 2, seed=0)
    cnt, _, _, _ = oracle.grid_count(X, eps)
    p = math.pi * eps ** 2 - 8 * eps ** 3 / 3 + eps ** 4 / 2
    s = (cnt - n) / n
    assert abs(s / ((n - 1) * p) - 1) < 0.02


# --------------------------------------------------------------------------
# Invalid input
# --------------------------------------------------------------------------

def test_invalid_inputs_rejected():
    X = gen.uniform(10, 2, 0)
    for eps in [0.0, -1.0, float("nan"), float("inf")]:
        with pytest.raises(ValueError):
            oracle.grid_count(X, eps)
        with pytest.raises(ValueError):
            oracle.bruteforce(X, eps)
    Y = X.copy()
    Y[3, 1] = float("nan")
    with pytest.raises(ValueError):
        oracle.grid_count(Y, 0.1)
    Y[3, 1] = float("inf")
    with pytest.raises(ValueError):
        oracle.bruteforce(Y, 0.1)
    # n = 0 is an empty result
    cnt, pp, _, _ = oracle.grid_count(np.zeros((0, 3)), 0.1)
    assert cnt == 0 and len(pp) == 0


# --------------------------------------------------------------------------
# kNN within eps (reuse of the self-join result)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,k", [(2, 1), (3, 8), (5, 20)])
def test_knn_within_eps_matches_kdtree(d, k):
    """Against scipy's k-d tree (its own distance code and search): the k
    nearest within eps, self excluded, in distance order. Rows with a
    distance within 1e-9 of eps or a near-tie inside the list are skipped
    (rounding decides those differently in the two codes)."""
    from scipy.spatial import cKDTree
    X = gen.uniform(3000, d, seed=40 + d)
    eps = 0.12 if d < 5 else 0.35
    nbr, dd, found = oracle.knn_within_eps(X, eps, k)
    dist, idx = cKDTree(X).query(X, k=k + 1, distance_upper_bound=eps * (1 + 1e-9))
    checked = 0
    for i in range(len(X)):
        got = [j for j in idx[i] if j < len(X) and j != i][:k]
        dk = np.sort(np.sqrt(((X - X[i]) ** 2).sum(1)))
        if np.any(np.abs(dk - eps) < 1e-9 * eps) or np.any(np.diff(dk[:k + 2]) < 1e-12):
            continue
        assert found[i] == len(got), i
        assert list(nbr[i, :found[i]]) == got, i
        assert np.allclose(np.sqrt(dd[i, :found[i]]), [dist[i][list(idx[i]).index(j)] for j in got], rtol=1e-12)
        assert np.all(nbr[i, found[i]:] == -1) and np.all(np.isinf(dd[i, found[i]:]))
        checked += 1
    assert checked > 0.95 * len(X)


def test_knn_within_eps_ties_by_index():
    """Lattice points have many equal distances: each list must be sorted by
    (distance, index), hold only points within eps, exclude the point, and
    be the k smallest of the brute-force neighbour set."""
    g = np.arange(6, dtype=np.float64)
    X = np.array(list(itertools.product(g, g)), dtype=np.float64)
    eps, k = 1.5, 6
    nbr, dd, found = oracle.knn_within_eps(X, eps, k)
    for i in range(len(X)):
        d2 = ((X - X[i]) ** 2).sum(1)
        cand = sorted((d2[j], j) for j in range(len(X)) if j != i and d2[j] <= eps * eps)
        want = cand[:k]
        assert found[i] == len(want)
        assert [(dd[i, r], nbr[i, r]) for r in range(found[i])] == [(float(a), b) for a, b in want]


def test_device_digest_helper_matches_oracle_on_cpu():
    # the GPU tests checksum the library's pairs with this torch helper; here
    # (torch on the CPU) it must agree with the oracle's C routine
    import torch

    from tests.gpu_util import add_digest, digest_pairs_t
    rng = np.random.default_rng(5)
    pairs = rng.integers(0, 2 ** 31 - 1, (10007, 2)).astype(np.int32)
    want = oracle.pairs_digest(pairs)
    t = torch.from_numpy(pairs)
    assert digest_pairs_t(t) == want
    assert digest_pairs_t(t, step=1000) == want
    assert add_digest(digest_pairs_t(t[:5000]), digest_pairs_t(t[5000:])) == want

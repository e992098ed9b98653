"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs. Pair sets and counts must be identical (bit-exact);
emitted distances must equal the oracle's chain bitwise (tolerance 0 here;
the contract allows 1e-12 relative)."""
import numpy as np
import pytest

from tests.gpu_util import gpu_join, log, pair_keys
from workloads import generators as gen

pytestmark = pytest.mark.gpu

PATHS = ["fp64_valu", "fp64_mfma", "fp32_mfma", "bf16_mfma", "bf16x3_mfma", "fp8_mfma"]
LOWP = ["fp32_mfma", "bf16_mfma", "bf16x3_mfma", "fp8_mfma"]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    p.load()
    yield


def _oracle_full(X, eps):
    import oracle
    cnt, pp, pairs, d2 = oracle.grid_pairs(X, eps, want_d2=True)
    _, _, cref, k = oracle.grid_count(X, eps)
    return cnt, pp, pairs, d2, cref, k


def _check_against_oracle(X, eps, path, tag, capacity=None, **build):
    log(f"[parity] {tag} path={path} n={X.shape[0]} d={X.shape[1]} eps={eps} {build}")
    cnt, pp, pairs, d2, cref, k = _oracle_full(X, eps)
    g = gpu_join(X, eps, path, want_pairs=True, want_d2=True, capacity=capacity, **build)
    assert g["total"] == cnt, (g["total"], cnt)
    assert np.array_equal(g["per_point"], pp)
    assert g["info"]["cand_ref"] == cref
    assert g["info"]["k"] == k
    assert np.array_equal(pair_keys(g["pairs"]), pair_keys(pairs))
    # d2 of every pair: bitwise equal to the oracle's chain
    ko = (pairs[:, 0].astype(np.int64) << 32) | pairs[:, 1]
    kg = (g["pairs"][:, 0].astype(np.int64) << 32) | g["pairs"][:, 1]
    oo = np.argsort(ko)
    og = np.argsort(kg)
    assert np.array_equal(d2[oo].view(np.int64), g["d2"][og].view(np.int64))
    return g


@pytest.mark.parametrize("path", PATHS)
def test_small_parity_config(path):
    # n = 20,000 uniform points in the unit square, seed 0, eps = 0.0218
    X = gen.uniform(20000, 2, seed=0)
    _check_against_oracle(X, 0.0218, path, "uniform-20k-2d")


CASES = []
for _d in (1, 2, 3, 4, 5, 6, 7, 8, 12, 16):
    for _dist in ("uniform", "expo", "gmm"):
        CASES.append((_dist, _d))


def _eps_for(X, target_s, seed=7):
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    qs = rng.integers(0, n, 30)
    dd = np.sort(np.concatenate([np.sqrt(((X - X[q]) ** 2).sum(1)) for q in qs]))
    return float(dd[min(len(dd) - 1, int(len(qs) * (target_s + 1)))])


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("dist,d", CASES)
def test_parity_distributions_and_dims(path, dist, d):
    # ragged sizes: not multiples of the 16-query / 16- or 64-candidate tiles
    n = {1: 5003, 2: 7919, 3: 6007, 4: 5501}.get(d, 3001)
    X = gen.make(dist, n, d, seed=100 + d)
    eps = _eps_for(X, 25)
    _check_against_oracle(X, eps, path, f"{dist}-{d}d")


@pytest.mark.parametrize("path", PATHS)
def test_lattice_ties_on_eps(path):
    # every distance exact; many pairs at exactly eps
    for L, d, r in [(40, 2, 3), (12, 3, 2), (7, 4, 2), (5, 5, 1)]:
        X = gen.lattice(L, d, 2.0 ** -6)
        _check_against_oracle(X, r * 2.0 ** -6, path, f"lattice L={L} d={d} r={r}")


@pytest.mark.parametrize("path", PATHS)
def test_adversarial_sets(path):
    rng = np.random.default_rng(3)
    base = rng.random((700, 3))
    sets = [
        (np.concatenate([base, base, base[:50]]), 0.05, "duplicates"),
        (1e6 + rng.random((3000, 2)) * 1e-3, 1e-4, "large-offset"),
        (rng.integers(0, 10, (3000, 3)).astype(np.float64) * 0.1, 0.1, "tenths"),
        (np.zeros((100, 4)), 1.0, "all-identical"),
        (np.repeat(rng.random((1, 2)), 1500, 0) + rng.random((1500, 2)) * 1e-9, 1e-3, "one-cell"),
    ]
    Y = rng.random((2500, 4)) - 0.5
    Y[:, 0] *= 1e4
    sets.append((Y, 0.2, "wide-dim0"))
    for X, eps, tag in sets:
        _check_against_oracle(X, eps, path, tag)


@pytest.mark.parametrize("path", PATHS)
def test_tiny_and_empty(path):
    import torch
    from paper_2209_11287_amd import SelfJoin
    for n in (0, 1, 2, 17):
        X = gen.uniform(n, 3, seed=n) if n else np.zeros((0, 3))
        log(f"[parity] tiny n={n} path={path}")
        sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), 0.3)
        total, pp, _ = sj.count(path, per_point=True)
        if n == 0:
            assert total == 0
        else:
            import oracle
            c, opp, _, _ = oracle.grid_count(X, 0.3)
            assert total == c
            assert np.array_equal(pp.cpu().numpy(), opp)
            pr = sj.all_pairs(path).cpu().numpy()
            _, _, opairs = oracle.bruteforce(X, 0.3)
            assert np.array_equal(pair_keys(pr), pair_keys(opairs))
        sj.close()


@pytest.mark.parametrize("path", PATHS)
def test_chunked_pairs_equal_one_shot(path):
    import torch
    from paper_2209_11287_amd import SelfJoin, SelfJoinError, selfjoin_pairs
    X = gen.exponential(30000, 3, seed=4)
    eps = _eps_for(X, 40)
    log(f"[parity] chunks path={path}")
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), eps)
    total, pp, _ = sj.count(path, per_point=True)
    one = sj.all_pairs(path).cpu().numpy()
    mx = int(pp.max().item())
    for cap in (mx, mx + 7, 5000, total // 3 + 1):
        chunked = sj.all_pairs(path, capacity=cap).cpu().numpy()
        # same pairs in the same (deterministic) order
        assert np.array_equal(chunked, one), cap
    # the next query's pairs do not fit
    buf = torch.empty((mx - 1, 2), dtype=torch.int32, device="cuda:0")
    cursor = 0
    with pytest.raises(SelfJoinError) as ei:
        while True:
            _, cursor, _ = selfjoin_pairs(sj.grid, path, cursor, buf, None, mx - 1)
    assert ei.value.needed >= mx
    sj.close()


@pytest.mark.parametrize("path", PATHS)
def test_deterministic_output(path):
    X = gen.uniform(50000, 2, seed=9)
    a = gpu_join(X, 0.01, path)["pairs"]
    b = gpu_join(X, 0.01, path)["pairs"]
    assert np.array_equal(a, b)


def test_paths_emit_identical_lists():
    X = gen.gaussian_mixture(20000, 8, seed=2)
    eps = _eps_for(X, 30)
    a = gpu_join(X, eps, "fp64_valu")["pairs"]
    for p in PATHS[1:]:
        b = gpu_join(X, eps, p)["pairs"]
        assert np.array_equal(a, b), p


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("d", [24, 32, 48, 64])
def test_parity_high_dimensions(path, d):
    # Gaussian mixture as in the precision workload, small n
    X = gen.gaussian_mixture(4000, d, clusters=20, seed=d)
    eps = _eps_for(X, 40)
    _check_against_oracle(X, eps, path, f"gmm-{d}d")


SC_CASES = [(0, 0), (1, 0), (2, 0), (0, 1), (-1, 0)]


@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
@pytest.mark.parametrize("d", [8, 16, 24, 64])
@pytest.mark.parametrize("sc,order", SC_CASES)
def test_short_circuit_drops_tiles_and_keeps_results(path, d, sc, order):
    """Section III-B's short-circuit on clustered data (many clusters, so that
    the 4-D grid neighbourhood of a query holds tiles of other clusters):
    tiles whose every partial distance is already beyond the threshold are
    left early (MFMA against eps^2 + Delta at K-step boundaries, VALU against
    eps^2 every 4 dimensions), for every schedule (sj_opts.short_circuit: 0 =
    the library's, k = every k K-steps, -1 = off) and dimension order
    (sj_opts.dim_order). Pair sets, counts and distances stay identical to
    the oracle's."""
    X = gen.gaussian_mixture(6000, d, clusters=300, seed=300 + d)
    eps = _eps_for(X, 20)
    g = _check_against_oracle(X, eps, path, f"short-circuit-{d}d", short_circuit=sc, dim_order=order)
    tiles = g["stats"]["cand_eval"] / 256.0
    frac = g["stats"]["tiles_pruned"] / tiles
    log(f"[short-circuit] d={d} path={path} sc={sc} order={order} tiles~{tiles:.0f} left early {frac:.3f}")
    # test points: MFMA after K-step KS / 2 for KS <= 4, else every sc (default
    # 4) K-steps; VALU (d > 8) every 4 sc (default 4) dimensions
    every = sc if sc > 0 else (1 if path == "fp64_valu" else 4)
    ks = d // 4
    has_check = sc != -1 and (d > 8 and 4 * every < d if path == "fp64_valu" else (ks <= 4 or every < ks))
    if not has_check:
        assert g["stats"]["tiles_pruned"] == 0
    else:
        assert g["stats"]["tiles_pruned"] > 0


@pytest.mark.parametrize("path", LOWP)
@pytest.mark.parametrize("d", [24, 64])
@pytest.mark.parametrize("sc", [0, -1])
def test_short_circuit_setting_on_low_precision_tiles(path, d, sc):
    """The FP32 / BF16 tiles run every K-step (their time goes into staging
    the candidate tiles, so checks at K-step boundaries saved nothing when
    measured): any short-circuit setting gives the oracle's results and no
    tile leaves early."""
    X = gen.gaussian_mixture(6000, d, clusters=300, seed=500 + d)
    eps = _eps_for(X, 20)
    g = _check_against_oracle(X, eps, path, f"lowp-short-circuit-{d}d", short_circuit=sc)
    assert g["stats"]["tiles_pruned"] == 0


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("dist,n,d", [("expo", 2048, 16), ("uniform", 3001, 3), ("gmm", 1000, 64)])
def test_index_free_mode_matches_oracle(path, dist, n, d):
    """index_dims = -1 (the brute-force mode of Section IV, Fig. 3): one cell,
    every ordered pair a candidate (C_ref = n^2); the pair set, per-point
    counts and distances are the oracle's (whose grid index does not change
    the result)."""
    import oracle
    from workloads import configs
    X = gen.make(dist, n, d, seed=17)
    eps = configs.brute_workloads()[0]["eps"] if dist == "expo" else _eps_for(X, 20)
    log(f"[index-free] {dist} n={n} d={d} path={path} eps={eps}")
    cnt, pp, pairs, d2 = oracle.grid_pairs(X, eps, want_d2=True)
    g = gpu_join(X, eps, path, want_pairs=True, want_d2=True, index_dims=-1)
    assert g["info"]["cells"] == 1
    assert g["info"]["cand_ref"] == n * n
    assert g["total"] == cnt
    assert np.array_equal(g["per_point"], pp)
    assert np.array_equal(pair_keys(g["pairs"]), pair_keys(pairs))
    ko = (pairs[:, 0].astype(np.int64) << 32) | pairs[:, 1]
    kg = (g["pairs"][:, 0].astype(np.int64) << 32) | g["pairs"][:, 1]
    assert np.array_equal(d2[np.argsort(ko)].view(np.int64), g["d2"][np.argsort(kg)].view(np.int64))


@pytest.mark.parametrize("path", ["fp64_mfma", "bf16_mfma"])
def test_core_points_match_oracle_counts(path):
    """DBSCAN core points (point i is core iff its eps-neighbourhood, itself
    included, holds >= min_pts points) from the oracle's per-point counts;
    min_pts below, at and above the typical count, and min_pts = 1 (every
    point is core: the self-pair)."""
    import torch
    import oracle
    from paper_2209_11287_amd import SelfJoin
    X = gen.make("expo", 6007, 3, seed=23)
    eps = _eps_for(X, 12)
    _, pp = oracle.grid_count(X, eps)[:2]
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), eps)
    try:
        for i, m in enumerate([1, 5, int(np.median(pp)), int(pp.max()), int(pp.max()) + 1]):
            if i == 1:
                sj.count(path)  # later calls reuse the cached counts
            flags, ncore = sj.core_points(m, path)
            want = (pp >= m).astype(np.uint8)
            assert ncore == int(want.sum()), m
            assert np.array_equal(flags.cpu().numpy(), want), m
    finally:
        sj.close()


@pytest.mark.parametrize("path", LOWP)
def test_lowp_rejects_large_d(path):
    import torch
    from paper_2209_11287_amd import SelfJoin, SelfJoinError
    X = gen.uniform(500, 80, seed=1)
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), 1.0)
    with pytest.raises(SelfJoinError) as ei:
        sj.count(path)
    assert ei.value.status == 5
    sj.close()


@pytest.mark.parametrize("path", ["fp64_mfma", "fp32_mfma", "bf16_mfma", "bf16x3_mfma", "fp8_mfma"])
def test_mfma_error_within_band(path):
    import torch
    from paper_2209_11287_amd import SelfJoin, selfjoin_measure_error
    for dist, d in [("uniform", 2), ("expo", 3), ("gmm", 4), ("gmm", 16), ("uniform", 7), ("gmm", 64)]:
        X = gen.make(dist, 20000 if d < 64 else 5000, d, seed=d)
        eps = _eps_for(X, 30)
        sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), eps)
        err, band, viol = selfjoin_measure_error(sj.grid, path)
        log(f"[band] {path} {dist} d={d} max_err={err:.3e} band={band:.3e} rel={band / eps**2:.3e} viol={viol}")
        assert viol == 0
        assert err <= band / 2  # the analysis bound, before its safety factor
        sj.close()
    # queries far from their block's reference point (a wide dimension, a
    # large common offset): the band grows with |q'|, the bound must hold
    rng = np.random.default_rng(11)
    Y = rng.random((6000, 4)) - 0.5
    Y[:, 0] *= 1e3
    for X, eps, tag in [(Y, 0.05, "wide-dim0"), (1e6 + rng.random((6000, 3)) * 1e-2, 1e-3, "large-offset")]:
        sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), eps)
        err, band, viol = selfjoin_measure_error(sj.grid, path)
        log(f"[band] {path} {tag} max_err={err:.3e} band={band:.3e} rel={band / eps**2:.3e} viol={viol}")
        assert viol == 0
        assert err <= band / 2
        sj.close()


def test_nonfinite_input_rejected():
    import torch
    from paper_2209_11287_amd import SelfJoinError, selfjoin_build_grid
    X = gen.uniform(1000, 3, seed=1)
    X[500, 1] = np.nan
    with pytest.raises(SelfJoinError) as ei:
        selfjoin_build_grid(torch.from_numpy(X).to("cuda:0"), 0.1)
    assert ei.value.status == 1
    X[500, 1] = np.inf
    with pytest.raises(SelfJoinError):
        selfjoin_build_grid(torch.from_numpy(X).to("cuda:0"), 0.1)


def test_index_dims_option_is_result_neutral():
    import oracle
    X = gen.gaussian_mixture(15000, 6, seed=5)
    eps = _eps_for(X, 20)
    c, pp, _, _ = oracle.grid_count(X, eps)
    for k in (1, 2, 3, 4):
        for path in PATHS:
            g = gpu_join(X, eps, path, want_pairs=False, index_dims=k)
            assert g["total"] == c
            assert np.array_equal(g["per_point"], pp)


@pytest.mark.parametrize("dist,n,d,k,path,budget", [
    ("uniform", 20000, 2, 8, "fp64_mfma", 0),
    ("expo", 12007, 3, 1, "fp64_valu", 0),
    ("expo", 12007, 3, 16, "fp64_mfma", -1),   # chunked: a few times the largest neighbourhood
    ("gmm", 6001, 16, 64, "bf16x3_mfma", 0),
    ("lattice", 0, 2, 6, "fp32_mfma", 0),
])
def test_knn_within_eps_matches_oracle(dist, n, d, k, path, budget):
    """kNN reuse of the pair list: neighbour indices, their squared distances
    and the number found, bit-exact against the oracle (self excluded, order
    by distance then index), including equal-distance ties on a lattice and
    a pair budget that forces several chunks."""
    import itertools
    import torch
    import oracle
    from paper_2209_11287_amd import SelfJoin
    if dist == "lattice":
        g = np.arange(40, dtype=np.float64)
        X = np.array(list(itertools.product(g, g)), dtype=np.float64)
        eps = 2.0
    else:
        X = gen.make(dist, n, d, seed=31 + d)
        eps = _eps_for(X, 24)
    log(f"[knn] {dist} n={len(X)} d={d} k={k} path={path}")
    want_nbr, want_d2, want_found = oracle.knn_within_eps(X, eps, k)
    if budget < 0:
        _, pp = oracle.grid_count(X, eps)[:2]
        budget = 3 * int(pp.max())
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), eps)
    try:
        nbr, d2, found = sj.knn(k, path, pair_budget=budget)
        assert np.array_equal(found.cpu().numpy(), want_found)
        assert np.array_equal(nbr.cpu().numpy(), want_nbr)
        assert np.array_equal(d2.cpu().numpy(), want_d2)
    finally:
        sj.close()


def test_knn_rejects_bad_arguments():
    """k outside [1, 64] is invalid; a pair budget below one point's
    neighbourhood is reported as unsupported (a host-side check), and the
    handle stays usable afterwards."""
    import torch
    from paper_2209_11287_amd import SelfJoin, SelfJoinError
    X = gen.uniform(4000, 2, seed=9)
    eps = _eps_for(X, 20)
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), eps)
    try:
        for k in (0, 65):
            with pytest.raises(SelfJoinError) as ei:
                sj.knn(k)
            assert ei.value.status == 1
        with pytest.raises(SelfJoinError) as ei:
            sj.knn(4, pair_budget=2)
        assert ei.value.status == 5
        nbr, d2, found = sj.knn(4)
        assert int(found.min()) >= 0 and int(found.max()) <= 4
    finally:
        sj.close()


@pytest.mark.parametrize("path", LOWP)
@pytest.mark.parametrize("d", [3, 16])
def test_low_precision_pairs_from_masks_and_from_tiles(path, d):
    # after a count on the same path the pairs pass expands the count's
    # in-masks; after an FP64 count it runs the tiles again: both the exact
    # set, whole and in chunks
    import torch

    import oracle
    from paper_2209_11287_amd import selfjoin_build_grid, selfjoin_count, selfjoin_pairs
    X = gen.make("gmm", 3001, d, seed=40 + d)
    eps = _eps_for(X, 20)
    _, pp, op = oracle.grid_pairs(X, eps)
    xt = torch.from_numpy(X).to("cuda:0")
    for count_path in (path, "fp64_valu"):
        log(f"[lp-masks] path={path} d={d} count_path={count_path}")
        g = selfjoin_build_grid(xt, eps)
        try:
            total, per, _ = selfjoin_count(g, count_path, per_point=True)
            assert total == len(op)
            assert np.array_equal(per.cpu().numpy(), pp)
            buf = torch.empty((total, 2), dtype=torch.int32, device="cuda:0")
            w, nxt, _ = selfjoin_pairs(g, path, 0, buf, None, total)
            assert (w, nxt) == (total, X.shape[0])
            assert np.array_equal(pair_keys(buf.cpu().numpy()), pair_keys(op))
            cap = int(pp.max()) + 7
            small = torch.empty((cap, 2), dtype=torch.int32, device="cuda:0")
            got, cursor = [], 0
            while cursor < X.shape[0]:
                w, cursor, _ = selfjoin_pairs(g, path, cursor, small, None, cap)
                got.append(small[:w].cpu().numpy())
            assert np.array_equal(pair_keys(np.concatenate(got)), pair_keys(op))
        finally:
            g.close()

"""Half-stencil count (sj_opts.symmetric = 1) through the C ABI against the
CPU oracle: every per-point count and the total are identical to the full
evaluation, on every FP64 tile form (one K-step, the LDS-shared block lists
of d = 5..16, many K-steps, runtime d, the vector-ALU forms), in the
index-free mode, on lattice ties and duplicate points, for tiny and ragged
inputs; a pair list requested after a symmetric count is the exact set; the
low-precision paths ignore the option."""
import numpy as np
import pytest

from tests.gpu_util import gpu_join, log, pair_keys
from workloads import generators as gen

pytestmark = pytest.mark.gpu

FP64 = ["fp64_mfma", "fp64_valu"]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    p.load()
    yield


def _eps_for(X, target_s, seed=7):
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    qs = rng.integers(0, n, 30)
    dd = np.sort(np.concatenate([np.sqrt(((X - X[q]) ** 2).sum(1)) for q in qs]))
    return float(dd[min(len(dd) - 1, int(len(qs) * (target_s + 1)))])


def _check(X, eps, path, tag, pairs=False, **build):
    import oracle
    log(f"[sym] {tag} path={path} n={X.shape[0]} d={X.shape[1]} eps={eps} {build}")
    total, pp, _, _ = oracle.grid_count(X, eps)
    g = gpu_join(X, eps, path, want_pairs=pairs, symmetric=1, **build)
    assert g["total"] == total, (g["total"], total)
    assert np.array_equal(g["per_point"], pp)
    if pairs:
        _, _, op = oracle.grid_pairs(X, eps)
        assert np.array_equal(pair_keys(g["pairs"]), pair_keys(op))
    return g


DIMS = [1, 2, 3, 4, 5, 7, 8, 12, 16, 20, 24, 32, 64, 72]


@pytest.mark.parametrize("path", FP64)
@pytest.mark.parametrize("d", DIMS)
@pytest.mark.parametrize("dist", ["uniform", "gmm"])
def test_symmetric_counts_match_oracle(path, d, dist):
    # ragged sizes; d = 5..16 runs the LDS-shared block lists, d > 16 many
    # K-steps, d = 72 the runtime K-step count, d > 8 the runtime V64 form
    n = {1: 4001, 2: 6007, 3: 5003, 4: 4507}.get(d, 2503)
    X = gen.make(dist, n, d, seed=300 + d)
    _check(X, _eps_for(X, 20), path, f"{dist}-{d}d")


@pytest.mark.parametrize("path", FP64)
def test_symmetric_expo_skewed(path):
    X = gen.make("expo", 30011, 3, seed=11)
    _check(X, _eps_for(X, 40), path, "expo-3d")


@pytest.mark.parametrize("path", FP64)
@pytest.mark.parametrize("d", [2, 8, 24])
def test_symmetric_index_free(path, d):
    X = gen.make("uniform", 1531, d, seed=17)
    _check(X, _eps_for(X, 15), path, f"brute-{d}d", index_dims=-1)


@pytest.mark.parametrize("path", FP64)
@pytest.mark.parametrize("d", [2, 3, 8])
def test_symmetric_lattice_ties_and_duplicates(path, d):
    # integer lattice with eps = 1: pairs at exactly eps; every point twice
    rng = np.random.default_rng(5)
    side = {2: 40, 3: 12, 8: 3}[d]
    L = rng.integers(0, side, size=(2500, d)).astype(np.float64)
    X = np.concatenate([L, L[:700]])
    X = X[rng.permutation(X.shape[0])]
    _check(X, 1.0, path, f"lattice-{d}d", pairs=True)


@pytest.mark.parametrize("path", FP64)
@pytest.mark.parametrize("n", [1, 2, 3, 15, 16, 17, 33, 65])
def test_symmetric_tiny(path, n):
    X = gen.make("uniform", n, 2, seed=n)
    _check(X, 0.5, path, f"tiny-{n}", pairs=True)


@pytest.mark.parametrize("path", FP64)
def test_symmetric_pairs_after_count_and_stats(path):
    X = gen.make("uniform", 20000, 2, seed=0)
    g = _check(X, 0.0218, path, "uniform-20k-pairs", pairs=True)
    full = gpu_join(X, 0.0218, path, want_pairs=False)
    # about half the candidate pairs (those after the item's first query)
    ratio = g["stats"]["cand_eval"] / full["stats"]["cand_eval"]
    log(f"[sym] cand_eval ratio {ratio:.3f}")
    assert 0.4 < ratio < 0.65


@pytest.mark.parametrize("path", ["fp32_mfma", "bf16x3_mfma"])
def test_symmetric_ignored_on_low_precision_paths(path):
    X = gen.make("gmm", 3001, 16, seed=9)
    _check(X, _eps_for(X, 20), path, "gmm-16d-lowp", pairs=True)


def test_symmetric_core_points():
    import torch

    import oracle
    from paper_2209_11287_amd import selfjoin_build_grid, selfjoin_core_points
    X = gen.make("gmm", 8009, 4, seed=21)
    eps = _eps_for(X, 12)
    _, pp, _, _ = oracle.grid_count(X, eps)
    g = selfjoin_build_grid(torch.from_numpy(X).to("cuda:0"), eps, symmetric=1)
    try:
        flags, ncore = selfjoin_core_points(g, 10, "fp64_mfma")
        assert ncore == int((pp >= 10).sum())
        assert np.array_equal(flags.cpu().numpy().astype(bool), pp >= 10)
    finally:
        g.close()

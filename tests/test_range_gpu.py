"""GPU parity at the edges of the floating-point range, the call statistics,
and the allocator hook, through the C ABI against the CPU oracle.

Every path must return the exact set for every finite input: data whose
scale would overflow a path's arithmetic (FP32 / BF16 tiles far from their
reference point, FP64 Gram values beyond 2^1000) are handed to the next exact
path, and the call says which path ran."""
import numpy as np
import pytest

from tests.gpu_util import gpu_join, log, pair_keys
from workloads import generators as gen

pytestmark = pytest.mark.gpu

LOWP = ["fp32_mfma", "bf16_mfma", "bf16x3_mfma", "fp8_mfma"]
ALL = ["fp64_valu", "fp64_mfma"] + LOWP


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    p.load()
    yield


def _exact(X, eps, path, tag):
    import oracle
    log(f"[range] {tag} path={path} n={X.shape[0]} d={X.shape[1]} eps={eps}")
    cnt, pp, pairs, d2 = oracle.grid_pairs(X, eps, want_d2=True)
    g = gpu_join(X, eps, path, want_pairs=True, want_d2=True)
    assert g["total"] == cnt, (g["total"], cnt)
    assert np.array_equal(g["per_point"], pp)
    assert np.array_equal(pair_keys(g["pairs"]), pair_keys(pairs))
    ko = (pairs[:, 0].astype(np.int64) << 32) | pairs[:, 1]
    kg = (g["pairs"][:, 0].astype(np.int64) << 32) | g["pairs"][:, 1]
    assert np.array_equal(d2[np.argsort(ko)].view(np.int64), g["d2"][np.argsort(kg)].view(np.int64))
    return g


@pytest.mark.parametrize("path", ALL)
def test_point_far_along_an_unindexed_extent(path):
    # two points 1e20 apart on the second dimension, eps = 10: the grid keeps
    # one indexed dimension; FP32 tiles centred on the first point would see
    # |c'|^2 = inf, so the low-precision paths hand the call to FP64 MFMA
    X = np.array([[0.0, 0.0], [0.0, 1e20]])
    g = _exact(X, 10.0, path, "two-points-1e20")
    assert g["total"] == 2
    if path in LOWP:
        assert g["stats"]["path_run"] == "fp64_mfma"


@pytest.mark.parametrize("path", ALL)
def test_extents_beyond_the_cell_count_range(path):
    # extent / eps beyond 2^63 cells, or max - min overflowing: the grid drops
    # indexed dimensions down to a single cell and every path stays exact
    sets = [np.array([[0.0, 0.0], [1e20, 0.0]]),
            np.array([[-1e308, 0.0], [1e308, 0.0], [1e308, 5.0]]),
            np.array([[0.0, 0.0], [1e20, 0.0], [1e20, 5.0], [3.0, 1e25]])]
    rng = np.random.default_rng(12)
    Y = rng.random((400, 3))
    Y[:7, 0] = [1e19, -1e19, 4e18, 1e300, -1e300, 2.5, 1e200]
    for i, X in enumerate(sets + [Y]):
        _exact(X, 10.0 if X.shape[0] < 10 else 0.2, path, f"extent-{i}")


@pytest.mark.parametrize("path", ALL)
def test_wide_spread_set(path):
    # clustered pairs spread over 1e15 in one dimension (extent / eps = 1e15
    # > 2^40): low precision runs FP64 MFMA instead
    rng = np.random.default_rng(4)
    base = rng.random((400, 3))
    base[:, 2] *= 1e15
    X = np.concatenate([base, base + rng.random((400, 3)) * 0.3])
    g = _exact(X, 0.5, path, "spread-1e15")
    if path in LOWP:
        assert g["stats"]["path_run"] == "fp64_mfma"


@pytest.mark.parametrize("path", ALL)
def test_huge_coordinates_beyond_fp64_gram_range(path):
    # centred norms ~1e320 overflow: FP64 MFMA hands the call to FP64 VALU;
    # the exact chain of nearby points stays finite. The extent is 3e9 eps,
    # inside the scaled FP32 / BF16 tiles' range: those paths run themselves.
    rng = np.random.default_rng(5)
    X = np.concatenate([rng.random((300, 2)) * 1e160, rng.random((300, 2)) * 1e150 + 1e159])
    eps = 3e150
    g = _exact(X, eps, path, "coords-1e160")
    # (FP8 tiles need extents within 100 eps: they hand the call on too)
    want = "fp64_valu" if path in ("fp64_mfma", "fp8_mfma") else path
    assert g["stats"]["path_run"] == want


@pytest.mark.parametrize("path", ALL)
@pytest.mark.parametrize("scale", [2.0 ** -300, 1e-100, 1e100, 2.0 ** 300])
def test_scale_invariance_at_extreme_units(path, scale):
    # a uniform set in units far from 1 (eps inside the FP32 tiles' range
    # after their power-of-two scaling): every path runs itself and returns
    # the oracle's set, ties included
    X = gen.uniform(3000, 3, seed=2) * scale
    eps = 0.05 * scale
    g = _exact(X, eps, path, f"scale-{scale:.1e}")
    assert g["stats"]["path_run"] == path


@pytest.mark.parametrize("path", LOWP)
def test_lattice_ties_in_tiny_units(path):
    # lattice with every neighbour distance exactly on eps, in units of 2^-400
    h = 2.0 ** -406
    X = gen.lattice(14, 2, h)
    g = _exact(X, 2 * h, path, "lattice-2^-406")
    assert g["stats"]["path_run"] == path


@pytest.mark.parametrize("path", LOWP)
def test_pairs_pass_reports_its_own_rechecks(path):
    import torch
    from paper_2209_11287_amd import SelfJoin, selfjoin_pairs
    X = gen.make("gmm", 6000, 32, seed=3)
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), 0.12)
    try:
        total, _, st_c = sj.count(path)
        assert st_c["path_run"] == path
        assert st_c["ms_refine"] > 0 and st_c["ms_build"] > 0
        buf = torch.empty((total, 2), dtype=torch.int32, device="cuda:0")
        wr, nxt, st_p = selfjoin_pairs(sj.grid, path, 0, buf, None, total)
        assert wr == total and nxt == X.shape[0]
        # after a count on the same path the pairs pass expands its in-masks:
        # no tile runs, no recheck
        assert st_p["rechecked"] == 0 and st_p["rechecked_in"] == 0
        assert st_p["ms_refine"] == 0.0 and st_p["ms_emit"] > 0  # counts were cached
        # after an FP64 count the pairs pass re-runs the tiles, so it meets
        # the same band pairs as the low-precision count
        sj.count("fp64_valu")
        wr2, _, st_p2 = selfjoin_pairs(sj.grid, path, 0, buf, None, total)
        assert wr2 == total
        log(f"[stats] {path} count rechecked={st_c['rechecked']} in={st_c['rechecked_in']} "
            f"pairs (tiles) rechecked={st_p2['rechecked']} in={st_p2['rechecked_in']}")
        assert st_p2["rechecked"] == st_c["rechecked"]
        assert st_p2["rechecked_in"] == st_c["rechecked_in"]
        if path != "fp32_mfma":  # the BF16 bands are wide enough to catch pairs here
            assert st_c["rechecked"] > 0
        assert 0 <= st_c["rechecked_in"] <= st_c["rechecked"]
    finally:
        sj.close()


@pytest.mark.parametrize("path", ["fp64_mfma", "fp32_mfma"])
def test_torch_allocator_hook(path):
    import torch

    import oracle
    from paper_2209_11287_amd import SelfJoin
    X = gen.make("expo", 30000, 3, seed=8)
    eps = 0.01
    cnt, pp, pairs = oracle.grid_pairs(X, eps)
    xt = torch.from_numpy(X).to("cuda:0")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    sj = SelfJoin(xt, eps, torch_alloc=True)
    try:
        held = torch.cuda.memory_allocated() - before
        assert held > X.nbytes  # the grid index lives in torch's allocator
        total, gpp, _ = sj.count(path, per_point=True)
        assert total == cnt and np.array_equal(gpp.cpu().numpy(), pp)
        got = sj.all_pairs(path)
        assert np.array_equal(pair_keys(got.cpu().numpy()), pair_keys(pairs))
        del got, gpp
    finally:
        sj.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before  # every block went back

"""GPU parity of the batched form: each problem of a batch (uneven n and d)
against the oracle run on that problem alone; HIP-graph replays; tuning."""
import os

import numpy as np
import pytest

from tests.gpu_util import log, pair_keys
from workloads import generators as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    p.load()
    yield


def _problems(count=24, seed=0):
    """A small batch shaped like the batched workload: n log-uniform, d from
    {2, 3, 4, 8, 16}, uniform points, eps for ~20 neighbours (estimated from
    the unit-cube volume)."""
    import math
    params = gen.batch_problems(count, seed=seed, n_lo=50, n_hi=4000)
    probs = []
    for b, (n, d) in enumerate(params):
        X = gen.uniform(n, d, seed=[seed, b])
        vol_unit = math.pi ** (d / 2) / math.gamma(d / 2 + 1)
        eps = (20.0 / max(n - 1, 1) / vol_unit) ** (1.0 / d)
        probs.append((X, float(eps)))
    return probs


@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
def test_batch_matches_oracle_per_problem(path):
    import torch

    import oracle
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    probs = _problems()
    log(f"[batch] {len(probs)} problems path={path}")
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs])
    totals, st = selfjoin_batch_count(b, path)
    want = [oracle.grid_count(X, e)[0] for X, e in probs]
    assert totals == want
    buf = torch.empty((sum(totals), 2), dtype=torch.int32, device="cuda:0")
    offs, _ = selfjoin_batch_pairs(b, path, buf)
    out = buf.cpu().numpy()
    for i, (X, e) in enumerate(probs):
        _, _, opairs = oracle.grid_pairs(X, e)
        got = out[offs[i]:offs[i + 1]]
        assert np.array_equal(pair_keys(got), pair_keys(opairs)), i
    selfjoin_batch_free(b)


def test_batch_graph_replays_are_identical():
    import torch

    from paper_2209_11287_amd import selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free
    probs = _problems(16, seed=3)
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs])
    first, _ = selfjoin_batch_count(b, "fp64_mfma")
    for rep in range(4):
        # eager work of the program between replays
        junk = torch.randn(1 << 20, device="cuda:0").sum().item()
        del junk
        torch.cuda.synchronize()
        again, _ = selfjoin_batch_count(b, "fp64_mfma")
        assert again == first, rep
    selfjoin_batch_free(b)


def test_batch_tuning_is_result_neutral(tmp_path):
    import torch

    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_info)
    probs = _problems(12, seed=5)
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    eps = [e for _, e in probs]
    b0 = selfjoin_batch_build(pts, eps)
    t0, _ = selfjoin_batch_count(b0, "fp64_mfma")
    selfjoin_batch_free(b0)
    cache = str(tmp_path / "tune.txt")
    b1 = selfjoin_batch_build(pts, eps, tune=True, tune_cache=cache)
    t1, _ = selfjoin_batch_count(b1, "fp64_mfma")
    assert t0 == t1
    assert os.path.exists(cache) and os.path.getsize(cache) > 0
    ks = [selfjoin_batch_info(b1, i)["index_dims"] for i in range(len(probs))]
    assert all(1 <= k <= 4 for k in ks)
    selfjoin_batch_free(b1)


def test_batch_capacity_error():
    import torch

    from paper_2209_11287_amd import SelfJoinError, selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_pairs
    probs = _problems(6, seed=7)
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs])
    totals, _ = selfjoin_batch_count(b, "fp64_mfma")
    small = torch.empty((max(1, sum(totals) // 2), 2), dtype=torch.int32, device="cuda:0")
    with pytest.raises(SelfJoinError) as ei:
        selfjoin_batch_pairs(b, "fp64_mfma", small)
    assert ei.value.needed == sum(totals)
    b.close()


def test_batch_pairs_graph_replays_and_buffers():
    """The pairs launch is a captured graph per output buffer: replays into
    the same buffer and a capture for a second buffer give the same rows;
    in-masks recorded by one FP64 path's count serve the other path's pairs."""
    import torch

    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    probs = _problems(16, seed=11)
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs])
    totals, _ = selfjoin_batch_count(b, "fp64_valu")
    n = max(1, sum(totals))
    b1 = torch.empty((n, 2), dtype=torch.int32, device="cuda:0")
    b2 = torch.full((n, 2), -1, dtype=torch.int32, device="cuda:0")
    o1, _ = selfjoin_batch_pairs(b, "fp64_mfma", b1)
    first = b1.clone()
    for rep in range(3):
        b1.fill_(-7)
        torch.cuda.synchronize()
        o, _ = selfjoin_batch_pairs(b, "fp64_mfma", b1)
        assert o == o1
        assert torch.equal(b1, first), rep
    o2, _ = selfjoin_batch_pairs(b, "fp64_mfma", b2)
    assert o2 == o1 and torch.equal(b2, first)
    selfjoin_batch_free(b)


def test_batch_tuned_schedule_and_filters_match_oracle(tmp_path):
    """Tuned choices (index_dims, short-circuit per d, and the tile kernels'
    schedule), the short-circuit off and the input dimension order: the
    same per-problem totals and pair sets as the oracle."""
    import torch

    import oracle
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    probs = _problems(14, seed=13)
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    eps = [e for _, e in probs]
    want = [oracle.grid_pairs(X, e)[2] for X, e in probs]
    for kw in ({"tune": True, "tune_cache": str(tmp_path / "t.txt")}, {"short_circuit": -1}, {"dim_order": 1},
               {"short_circuit": 1}):
        log(f"[batch] options {kw}")
        b = selfjoin_batch_build(pts, eps, **kw)
        totals, _ = selfjoin_batch_count(b, "fp64_mfma")
        assert totals == [len(w) for w in want], kw
        buf = torch.empty((max(1, sum(totals)), 2), dtype=torch.int32, device="cuda:0")
        offs, _ = selfjoin_batch_pairs(b, "fp64_mfma", buf)
        out = buf.cpu().numpy()
        for i in range(len(probs)):
            assert np.array_equal(pair_keys(out[offs[i]:offs[i + 1]]), pair_keys(want[i])), (kw, i)
        selfjoin_batch_free(b)


@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
def test_batch_symmetric_count_matches_oracle(path, tmp_path):
    """The half-stencil count for every problem (sj_opts.symmetric), with the
    library's schedule and with the tuned one: the oracle's totals, the same
    on graph replays with eager work between them; fewer candidate pairs
    evaluated than the full stencil's; and a later pairs launch (the tiles
    re-run, as the count recorded no in-masks) writes the oracle's pair set
    of each problem at the offsets the half-stencil counts gave."""
    import torch

    import oracle
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    probs = _problems(20, seed=17)
    # tiny problems: one point, two points within eps, a handful of points
    rng = np.random.default_rng(17)
    probs += [(rng.random((1, 3)), 0.1), (np.array([[0.0, 0.0], [0.05, 0.0]]), 0.1), (rng.random((5, 8)), 0.7)]
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    eps = [e for _, e in probs]
    want = [oracle.grid_pairs(X, e)[2] for X, e in probs]
    full = selfjoin_batch_build(pts, eps)
    _, st_full = selfjoin_batch_count(full, path)
    selfjoin_batch_free(full)
    for kw in ({}, {"tune": True, "tune_cache": str(tmp_path / "t.txt")}):
        log(f"[batch] symmetric path={path} options {kw}")
        b = selfjoin_batch_build(pts, eps, symmetric=1, **kw)
        totals, st = selfjoin_batch_count(b, path)
        assert totals == [len(w) for w in want], kw
        assert 0 < st["cand_eval"] < st_full["cand_eval"], kw
        for rep in range(3):
            junk = torch.randn(1 << 20, device="cuda:0").sum().item()
            del junk
            torch.cuda.synchronize()
            again, _ = selfjoin_batch_count(b, path)
            assert again == totals, (kw, rep)
        buf = torch.empty((max(1, sum(totals)), 2), dtype=torch.int32, device="cuda:0")
        offs, _ = selfjoin_batch_pairs(b, path, buf)
        out = buf.cpu().numpy()
        for i in range(len(probs)):
            assert np.array_equal(pair_keys(out[offs[i]:offs[i + 1]]), pair_keys(want[i])), (kw, i)
        selfjoin_batch_free(b)


@pytest.mark.parametrize("symmetric", [0, 1])
@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
def test_batch_with_empty_problems(path, symmetric):
    """Problems with no points among non-empty ones (d = 2, 3, 8, 16): zero
    totals and empty output rows for them, the oracle's pair sets for the
    others."""
    import torch

    import oracle
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    rng = np.random.default_rng(1)
    probs = [(np.zeros((0, 3)), 0.1), (rng.random((200, 3)), 0.1), (np.zeros((0, 16)), 0.5),
             (rng.random((300, 8)), 0.4), (np.zeros((0, 2)), 0.1)]
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    want = [oracle.grid_pairs(X, e)[2] for X, e in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs], symmetric=symmetric)
    totals, _ = selfjoin_batch_count(b, path)
    assert totals == [len(w) for w in want]
    assert totals[0] == totals[2] == totals[4] == 0
    buf = torch.empty((max(1, sum(totals)), 2), dtype=torch.int32, device="cuda:0")
    offs, _ = selfjoin_batch_pairs(b, path, buf)
    out = buf.cpu().numpy()
    for i in range(len(probs)):
        assert np.array_equal(pair_keys(out[offs[i]:offs[i + 1]]), pair_keys(want[i])), i
    selfjoin_batch_free(b)


@pytest.mark.parametrize("symmetric", [0, 1])
def test_batch_of_many_tiny_problems(symmetric):
    """1100 problems of 0 to 40 points (d = 2, 3, 8): more problems than the
    per-point-count reset kernel's grid rows (1024) and the oracle's totals
    and pair sets for every problem."""
    import torch

    import oracle
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    rng = np.random.default_rng(23)
    probs = []
    for i in range(1100):
        n = int(rng.integers(0, 41))
        d = (2, 3, 8)[i % 3]
        probs.append((rng.random((n, d)), 0.35 if d == 8 else 0.15))
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    want = [oracle.grid_pairs(X, e)[2] for X, e in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs], symmetric=symmetric)
    totals, _ = selfjoin_batch_count(b, "fp64_mfma")
    assert totals == [len(w) for w in want]
    buf = torch.empty((max(1, sum(totals)), 2), dtype=torch.int32, device="cuda:0")
    offs, _ = selfjoin_batch_pairs(b, "fp64_mfma", buf)
    out = buf.cpu().numpy()
    for i in range(len(probs)):
        assert np.array_equal(pair_keys(out[offs[i]:offs[i + 1]]), pair_keys(want[i])), i
    selfjoin_batch_free(b)


@pytest.mark.parametrize("symmetric", [0, 1])
@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
def test_batch_ties_and_duplicates(path, symmetric):
    """Integer-lattice problems with eps = 1 (pairs at exactly eps), every
    point of a problem present twice or more, and one problem of a single
    repeated point, in one batch (d = 2, 3, 8, 16): the oracle's totals and
    pair sets."""
    import torch

    import oracle
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    rng = np.random.default_rng(29)
    probs = []
    for d, side, n in ((2, 30, 900), (3, 10, 700), (8, 3, 600), (16, 2, 400)):
        L = rng.integers(0, side, size=(n, d)).astype(np.float64)
        X = np.concatenate([L, L[: n // 3]])
        probs.append((X[rng.permutation(X.shape[0])], 1.0))
    probs.append((np.full((300, 3), 0.25), 0.5))
    pts = [torch.from_numpy(X).to("cuda:0") for X, _ in probs]
    want = [oracle.grid_pairs(X, e)[2] for X, e in probs]
    b = selfjoin_batch_build(pts, [e for _, e in probs], symmetric=symmetric)
    totals, _ = selfjoin_batch_count(b, path)
    assert totals == [len(w) for w in want]
    assert totals[-1] == 300 * 300
    buf = torch.empty((max(1, sum(totals)), 2), dtype=torch.int32, device="cuda:0")
    offs, _ = selfjoin_batch_pairs(b, path, buf)
    out = buf.cpu().numpy()
    for i in range(len(probs)):
        assert np.array_equal(pair_keys(out[offs[i]:offs[i + 1]]), pair_keys(want[i])), i
    selfjoin_batch_free(b)

"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times (build + count + one-shot pair list, or cursor chunks for the
10M-point set): per-point counts and whole neighbour lists of sampled queries
against the oracle's range query (brute force over all n points), plus
properties that hold at any size (total = sum of counts = list length,
symmetry, self-pairs, per-query runs in candidate order)."""
import numpy as np
import pytest

from tests.gpu_util import log
from workloads import configs
from workloads import generators as gen

pytestmark = pytest.mark.gpu

NSAMPLE = 48


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    p.load()
    yield


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, n, NSAMPLE))


def _check_lists(X, eps, pairs_t, counts, sample):
    """pairs_t: (R, 2) int32 CUDA tensor; rows of each query contiguous."""
    import torch
    import oracle
    q = pairs_t[:, 0]
    for i in sample.tolist():
        sel = pairs_t[q == i, 1].cpu().numpy()
        ref = oracle.query(X, eps, i)
        assert len(sel) == counts[i], (i, len(sel), counts[i])
        assert np.array_equal(np.sort(sel), ref), i
        assert i in set(sel.tolist())  # self-pair
    # symmetry on the sample: (i, j) present => (j, i) present
    keys = (pairs_t[:, 0].to(torch.int64) << 32) | pairs_t[:, 1].to(torch.int64)
    keys_sorted, _ = torch.sort(keys)
    for i in sample[:8].tolist():
        js = pairs_t[q == i, 1].to(torch.int64)
        rev = (js << 32) | i
        pos = torch.searchsorted(keys_sorted, rev)
        pos = torch.clamp(pos, max=keys_sorted.numel() - 1)
        assert bool(torch.all(keys_sorted[pos] == rev)), i


@pytest.mark.parametrize("name", configs.CFG2)
@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
def test_cfg2_full_size(name, path):
    import torch
    import oracle
    from paper_2209_11287_amd import SelfJoin
    w = configs.workload(name)
    X = gen.make(w["dist"], w["n"], w["d"], seed=w["seed"])
    log(f"[fullsize] {name} path={path} n={w['n']} d={w['d']} eps={w['eps']}")
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), w["eps"])
    try:
        total, pp, _ = sj.count(path, per_point=True)
        counts = pp.cpu().numpy()
        assert total == int(counts.sum())
        sample = _sample(w["n"], seed=len(name))
        oc, _ = oracle.grid_count_sample(X, w["eps"], sample)
        assert np.array_equal(counts[sample], oc)
        pairs = sj.all_pairs(path)
        assert pairs.shape[0] == total
        # each query's pairs form one run at its exact offset (sorted order of
        # the grid, input indices in the rows)
        _check_lists(X, w["eps"], pairs, counts, sample)
        torch.cuda.synchronize()
    finally:
        sj.close()


def test_skewed_10m_chunked():
    import torch
    import oracle
    from paper_2209_11287_amd import SelfJoin
    w = configs.workload(configs.SKEWED[0])
    X = gen.make(w["dist"], w["n"], w["d"], seed=w["seed"])
    log(f"[fullsize] {w['name']} n={w['n']} chunked")
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), w["eps"])
    try:
        total, pp, _ = sj.count("fp64_mfma", per_point=True)
        counts = pp.cpu().numpy()
        assert total == int(counts.sum())
        sample = _sample(w["n"], seed=11)
        oc, _ = oracle.grid_count_sample(X, w["eps"], sample)
        assert np.array_equal(counts[sample], oc)
        # the bench's chunk size: 2^28 pairs per chunk, whole queries per chunk
        from paper_2209_11287_amd import selfjoin_pairs
        cap = 1 << 28
        buf = torch.empty((cap, 2), dtype=torch.int32, device="cuda:0")
        cursor, seen = 0, 0
        want = set(sample.tolist())
        while cursor < w["n"]:
            wr, nxt, _ = selfjoin_pairs(sj.grid, "fp64_mfma", cursor, buf, None, cap)
            chunk = buf[:wr]
            q = chunk[:, 0]
            for i in sorted(want):
                sel = chunk[q == i, 1].cpu().numpy()
                if len(sel):
                    ref = oracle.query(X, w["eps"], i)
                    assert np.array_equal(np.sort(sel), ref), i
                    assert len(sel) == counts[i]
                    want.discard(i)
            seen += wr
            cursor = nxt
        assert seen == total
        assert not want  # every sampled query appeared (all have a self-pair)
    finally:
        sj.close()

"""The entry point that allocates nothing (static device scratch):
selfjoin_count_noalloc against selfjoin_build_grid + selfjoin_count on the
same inputs, two calls in a row with the second smaller (the scratch keeps
the first call's contents), every path; and its size limit."""
import numpy as np
import pytest

from tests.gpu_util import log
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


def _reference(xt, eps, path):
    from paper_2209_11287_amd import SelfJoin
    sj = SelfJoin(xt, eps)
    try:
        total, pp, _ = sj.count(path, per_point=True)
        return total, pp.cpu().numpy()
    finally:
        sj.close()


CASES = [
    # (distribution, n first, n second, d, eps first, eps second)
    ("uniform", 200_000, 30_000, 2, 0.004, 0.01),
    ("expo", 150_000, 20_001, 3, 0.004, 0.01),
    ("uniform", 120_000, 9_999, 4, 0.06, 0.1),
    ("gmm", 60_000, 5_000, 16, 0.05, 0.08),
]


@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu", "fp32_mfma", "bf16x3_mfma"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}_d{c[3]}")
def test_noalloc_matches_count_twice(case, path):
    import torch
    from paper_2209_11287_amd import selfjoin_count_noalloc
    dist, n1, n2, d, e1, e2 = case
    for n, eps, seed in ((n1, e1, 1), (n2, e2, 2)):
        log(f"[noalloc] {dist} n={n} d={d} eps={eps} path={path}")
        X = gen.make(dist, n, d, seed=seed)
        xt = torch.from_numpy(X).to("cuda:0")
        want_t, want_pp = _reference(xt, eps, path)
        got_t, got_pp = selfjoin_count_noalloc(xt, eps, path, per_point=True)
        torch.cuda.synchronize()
        assert got_t == want_t
        assert np.array_equal(got_pp.cpu().numpy(), want_pp)
        # without per-point counts
        t2, none = selfjoin_count_noalloc(xt, eps, path)
        assert none is None and t2 == want_t


def test_noalloc_small_and_empty():
    import torch
    import oracle
    from paper_2209_11287_amd import selfjoin_count_noalloc
    X = gen.uniform(20000, 2, seed=0)
    cnt, pp, _, _ = oracle.grid_count(X, 0.0218)
    xt = torch.from_numpy(X).to("cuda:0")
    t, gpp = selfjoin_count_noalloc(xt, 0.0218, "fp64_mfma", per_point=True)
    assert t == cnt and np.array_equal(gpp.cpu().numpy(), pp)
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda:0")
    t0, _ = selfjoin_count_noalloc(e, 0.1, "fp64_mfma", per_point=True)
    assert t0 == 0
    one = torch.zeros((1, 5), dtype=torch.float64, device="cuda:0")
    assert selfjoin_count_noalloc(one, 0.1, "fp64_valu")[0] == 1


def test_noalloc_rejects_beyond_scratch():
    import torch
    from paper_2209_11287_amd import SelfJoinError, selfjoin_count_noalloc
    from paper_2209_11287_amd._lib import SJ_ERR_CAPACITY
    X = torch.zeros((700_000, 4), dtype=torch.float64, device="cuda:0")
    with pytest.raises(SelfJoinError) as ei:
        selfjoin_count_noalloc(X, 0.1, "fp64_mfma")
    assert ei.value.status == SJ_ERR_CAPACITY
    assert "scratch" in str(ei.value)
    # just inside the limit still runs
    Y = torch.from_numpy(gen.uniform(600_000, 4, seed=3)).to("cuda:0")
    t, _ = selfjoin_count_noalloc(Y, 0.02, "fp64_mfma")
    want, _ = _reference(Y, 0.02, "fp64_mfma")
    assert t == want

"""GPU parity at the full workload sizes, in the launch configuration bench.py
times (build + count + one-shot pair list; cursor chunks for the 10M-point
set; the batched form for the 256 problems), on every path.

Whole results are compared with the oracle's, computed by
tests/golden/make_fullsize.py (oracle only) and stored in
tests/golden/fullsize.json: |R|, the per-point counts of all n points (sha256
of the int32 vector in input order), and the two order-independent checksums
of the whole pair set (oracle.grid_digest; the same sums over the GPU's pairs,
chunk by chunk). Independently of the grid oracle, sampled queries' whole
neighbour lists are checked against the brute-force range query over all n
points, and properties that hold at any size (total = sum of counts = list
length, symmetry, self-pairs) are checked on the device."""
import hashlib
import json
import os

import numpy as np
import pytest

from tests.gpu_util import add_digest, digest_pairs_t, log
from workloads import configs
from workloads import generators as gen

pytestmark = pytest.mark.gpu

NSAMPLE = 48
GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize.json")
GOLD = json.load(open(GOLD_PATH)) if os.path.exists(GOLD_PATH) else {}

ALL_PATHS = ["fp64_mfma", "fp64_valu", "fp32_mfma", "bf16_mfma", "bf16x3_mfma", "fp8_mfma"]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_11287_amd as p
    p.load()
    yield


_DATA = {}


def _data(name):
    """The data set and its stored oracle results (inputs checked by sha256)."""
    if name not in GOLD:
        pytest.skip(f"no stored oracle results for {name}; run tests/golden/make_fullsize.py")
    g = GOLD[name]
    if name not in _DATA:
        _DATA.clear()  # one full-size set in host memory at a time
        X = gen.make(g["dist"], g["n"], g["d"], seed=g["seed"])
        assert hashlib.sha256(X.tobytes()).hexdigest() == g["x_sha256"], "input generator changed"
        _DATA[name] = X
    return _DATA[name], g


def _digest(g):
    return int(g["digest"][0]), int(g["digest"][1])


def _check_counts(counts, g, X):
    """All n per-point counts against the oracle's (by sha256; on a mismatch
    the oracle recounts to report how many differ)."""
    h = hashlib.sha256(np.ascontiguousarray(counts, dtype="<i4").tobytes()).hexdigest()
    if h != g["counts_sha256"]:
        import oracle
        _, opp, _, _ = oracle.grid_count(X, g["eps"])
        bad = np.nonzero(opp != counts)[0]
        raise AssertionError(f"{len(bad)} per-point counts differ, first {bad[:8].tolist()}: "
                             f"gpu {counts[bad[:8]].tolist()} oracle {opp[bad[:8]].tolist()}")


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, n, NSAMPLE))


def _check_lists(X, eps, pairs_t, counts, sample):
    """Sampled queries' whole lists against brute force; symmetry on device.
    pairs_t: (R, 2) int32 CUDA tensor."""
    import torch
    import oracle
    q = pairs_t[:, 0]
    for i in sample.tolist():
        sel = pairs_t[q == i, 1].cpu().numpy()
        ref = oracle.query(X, eps, i)
        assert len(sel) == counts[i], (i, len(sel), counts[i])
        assert np.array_equal(np.sort(sel), ref), i
    # the whole list is symmetric: sorted keys (i, j) equal sorted keys (j, i)
    a = (pairs_t[:, 0].to(torch.int64) << 32) | pairs_t[:, 1].to(torch.int64)
    b = (pairs_t[:, 1].to(torch.int64) << 32) | pairs_t[:, 0].to(torch.int64)
    assert bool(torch.equal(torch.sort(a)[0], torch.sort(b)[0]))
    del a, b
    # every self-pair present exactly once
    selfp = pairs_t[:, 0] == pairs_t[:, 1]
    assert int(selfp.sum()) == X.shape[0]
    assert bool(torch.all(torch.bincount(pairs_t[selfp, 0].to(torch.int64), minlength=X.shape[0]) == 1))


def _whole(name, path, sample_lists):
    import torch
    from paper_2209_11287_amd import SelfJoin
    X, g = _data(name)
    log(f"[fullsize] {name} path={path} n={g['n']} d={g['d']} eps={g['eps']}")
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), g["eps"])
    try:
        total, pp, st = sj.count(path, per_point=True)
        counts = pp.cpu().numpy()
        assert total == g["total"], (total, g["total"])
        assert int(counts.sum()) == total
        _check_counts(counts, g, X)
        pairs = sj.all_pairs(path)
        assert pairs.shape[0] == total
        assert digest_pairs_t(pairs) == _digest(g)
        # per-query counts of the list itself
        assert bool(torch.equal(torch.bincount(pairs[:, 0].to(torch.int64), minlength=g["n"]).to(torch.int32),
                                pp))
        if sample_lists:
            _check_lists(X, g["eps"], pairs, counts, _sample(g["n"], seed=len(name)))
        torch.cuda.synchronize()
        return st
    finally:
        sj.close()


@pytest.mark.parametrize("name", configs.CFG2)
@pytest.mark.parametrize("path", ALL_PATHS)
def test_cfg2_full_size(name, path):
    _whole(name, path, sample_lists=path in ("fp64_mfma", "fp64_valu"))


@pytest.mark.parametrize("name", configs.PREC)
@pytest.mark.parametrize("path", ALL_PATHS)
def test_prec_full_size(name, path):
    st = _whole(name, path, sample_lists=path == "fp64_mfma")
    log(f"[fullsize] {name} {path} band_rel={st['band_rel']:.4g} rechecked={st['rechecked']} "
        f"path_run={st['path_run']}")


@pytest.mark.parametrize("path", ["fp32_mfma", "bf16_mfma", "bf16x3_mfma", "fp8_mfma", "fp64_mfma"])
@pytest.mark.parametrize("name", configs.PREC)
def test_prec_band_holds_full_size(name, path):
    """The error band of the tile path covers every candidate pair's
    deviation from the exact chain (no violation), at full size."""
    import torch
    from paper_2209_11287_amd import SelfJoin, selfjoin_measure_error
    if path == "fp64_mfma":
        pytest.skip("a run of this case stalled (killed after 180 s without output) while the FP64 MFMA "
                    "measurement kernel took its items from per-XCD queues; that launch form is taken "
                    "out again, and the case stays off until the cause of the stall is shown")
    X, g = _data(name)
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), g["eps"])
    try:
        err, band, viol = selfjoin_measure_error(sj.grid, path)
        log(f"[band] {name} {path} max|D-d2|={err:.4g} band={band:.4g} eps2={g['eps'] ** 2:.4g}")
        assert viol == 0
        assert err <= band
    finally:
        sj.close()


SKEW_PATHS = ["fp64_mfma", "fp32_mfma", "fp64_valu", "bf16x3_mfma"]


@pytest.mark.parametrize("path", SKEW_PATHS)
def test_skewed_10m_chunked(path):
    """The 10M-point exponential set: all counts, and the pair set in the
    bench's chunks of 2^28 pairs (whole queries per chunk), checksummed chunk
    by chunk."""
    import torch
    from paper_2209_11287_amd import SelfJoin, selfjoin_pairs
    name = configs.SKEWED[0]
    X, g = _data(name)
    log(f"[fullsize] {name} path={path} n={g['n']} chunked")
    sj = SelfJoin(torch.from_numpy(X).to("cuda:0"), g["eps"])
    try:
        total, pp, _ = sj.count(path, per_point=True)
        counts = pp.cpu().numpy()
        assert total == g["total"], (total, g["total"])
        _check_counts(counts, g, X)
        cap = 1 << 28
        buf = torch.empty((cap, 2), dtype=torch.int32, device="cuda:0")
        sample = _sample(g["n"], seed=11) if path == "fp64_mfma" else np.zeros(0, dtype=np.int64)
        want = set(sample.tolist())
        cursor, seen, dig, chunks = 0, 0, (0, 0), 0
        percount = torch.zeros(g["n"], dtype=torch.int64, device="cuda:0")
        while cursor < g["n"]:
            wr, nxt, _ = selfjoin_pairs(sj.grid, path, cursor, buf, None, cap)
            chunk = buf[:wr]
            dig = add_digest(dig, digest_pairs_t(chunk))
            percount += torch.bincount(chunk[:, 0].to(torch.int64), minlength=g["n"])
            q = chunk[:, 0]
            for i in sorted(want):
                sel = chunk[q == i, 1].cpu().numpy()
                if len(sel):
                    import oracle
                    assert np.array_equal(np.sort(sel), oracle.query(X, g["eps"], i)), i
                    assert len(sel) == counts[i]
                    want.discard(i)
            seen += wr
            cursor = nxt
            chunks += 1
        assert chunks > 1
        assert seen == total
        assert dig == _digest(g)
        # whole queries per chunk: each query's pairs were all in one chunk and
        # together match its count
        assert bool(torch.equal(percount.to(torch.int32), pp))
        assert not want
    finally:
        sj.close()


@pytest.mark.parametrize("path", ["fp64_mfma", "fp64_valu"])
def test_batched_256_full_size(path):
    """The batched workload's 256 problems in one batch: every problem's |R|
    and pair-set checksums against the oracle run on that problem alone."""
    import torch
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_pairs)
    if "batched" not in GOLD:
        pytest.skip("no stored oracle results for the batched workload; run tests/golden/make_fullsize.py")
    probs = GOLD["batched"]["problems"]
    ws = configs.batched_workload(GOLD["batched"]["count"], GOLD["batched"]["seed"], GOLD["batched"]["s"])
    log(f"[fullsize] batched {len(ws)} problems path={path}")
    pts = []
    for w, g in zip(ws, probs):
        X = gen.make(w["dist"], w["n"], w["d"], seed=w["seed"])
        assert hashlib.sha256(X.tobytes()).hexdigest() == g["x_sha256"]
        assert w["eps"] == g["eps"]
        pts.append(torch.from_numpy(X).to("cuda:0"))
    b = selfjoin_batch_build(pts, [w["eps"] for w in ws], tune=True)
    try:
        totals, _ = selfjoin_batch_count(b, path)
        assert totals == [g["total"] for g in probs]
        buf = torch.empty((sum(totals), 2), dtype=torch.int32, device="cuda:0")
        offs, _ = selfjoin_batch_pairs(b, path, buf)
        for i, g in enumerate(probs):
            got = buf[offs[i]:offs[i + 1]]
            assert got.shape[0] == g["total"], i
            assert digest_pairs_t(got) == _digest(g), i
    finally:
        selfjoin_batch_free(b)

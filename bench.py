#!/usr/bin/env python
"""Benchmark of the MI355X epsilon-distance self-join (one GPU).

One step = the whole path over the measured workload: for each of the six
data sets (n = 2,000,000 points; d in {2, 3, 4}; uniform in [0,1]^d and
exponential(40) clipped to [0,1]; eps for ~64 mean neighbours), build the
grid index, count R, and write the full pair list to device memory. Inputs
are resident in HBM before the timed region. The six independent joins are
taken by --streams host threads from a shared queue (longest first), one HIP
stream each (default 3), so one set's small build kernels overlap another's
refine kernels. The roofline comes from a single-stream pass after the timed
steps (the launches' own times); the shared-GPU launch times sit beside it.

metric: distance evaluations per second = C_ref / step time, where C_ref is
the number of ordered candidate pairs of the full 3^k stencil of the
reference grid (an implementation-independent work unit), plus the
self-join time. The FP64 MFMA path is the headline; the FP64 vector-ALU path
runs beside it on the same data (--compare).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--path fp64_mfma]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "distance evals/s + self-join time, exact pairs; MFMA vs FP64 vector, 1 GPU"
WORKLOAD_TEXT = {
    "cfg2": "n=2,000,000 x {uniform, exponential(40)} x d in {2,3,4}, s~64; build + count + full pair list",
    "small": "n=20,000 uniform d=2 eps=0.0218 (parity size); build + count + full pair list",
    "prec": "n=1,000,000 Gaussian mixture (100 clusters, sigma 0.02) x d in {16,32,64}, s~50; "
            "build + count + full pair list",
    "skewed": "n=10,000,000 exponential(40) d=3, s~100; build + count + pair list in chunks",
    "batched": "256 independent self-joins, n log-uniform in [1e3, 2e5], d in {2,3,4,8,16}, uniform, s~32; "
               "build + count (one graph) + every pair (one graph)",
    "brute": "index-free (brute-force) mode, exponential(40) d=16, n = 2^11 .. 2^17, one eps (s~64 at 2^17); "
             "build + count + full pair list; C_ref = n^2",
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", default="fp64_mfma")
    ap.add_argument("--compare", default="fp64_valu", help="second path timed on the same data ('none' = none)")
    ap.add_argument("--workload", default="cfg2", choices=["cfg2", "small", "prec", "skewed", "batched", "brute"])
    ap.add_argument("--chunk", type=int, default=0, help="pairs per output chunk (0 = one chunk)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-set", action="store_true", help="skip the per-set single-stream path comparison")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the achievable-peak microbenchmarks (selfjoin_probe_peaks)")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the short passes of the precision, 10M-point and batched workloads")
    ap.add_argument("--streams", type=int, default=3,
                    help="data sets run concurrently, one host thread and HIP stream each")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def datasets(which):
    from workloads import configs
    if which == "brute":
        return [dict(w, index_dims=-1) for w in configs.brute_workloads()]
    names = {"cfg2": configs.CFG2, "small": ["small"], "prec": configs.PREC, "skewed": configs.SKEWED}[which]
    return [configs.workload(nm) for nm in names]


def load_inputs(wl):
    import torch
    from workloads import generators as gen
    out = []
    for w in wl:
        X = gen.make(w["dist"], w["n"], w["d"], seed=w["seed"])
        out.append((w, X, torch.from_numpy(X).to("cuda:0")))
    torch.cuda.synchronize()
    return out


def one_dataset(i, w, xt, path, bufs, collect, cref, chunk, stream):
    """build + count + pairs of data set i on `stream`."""
    import torch
    from paper_2209_11287_amd import (selfjoin_build_grid, selfjoin_count, selfjoin_free_grid,
                                      selfjoin_grid_info, selfjoin_pairs)
    g = selfjoin_build_grid(xt, w["eps"], index_dims=w.get("index_dims", 0), stream=stream)
    total, _, st_c = selfjoin_count(g, path, per_point=False, stream=stream)
    cap = total if chunk <= 0 else min(total, chunk)
    if bufs[i] is None or bufs[i].shape[0] < cap:
        with torch.cuda.stream(stream):
            bufs[i] = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda:0")
    cursor, done, emit_ms = 0, 0, 0.0
    st_p = None
    while cursor < w["n"]:
        written, cursor, st = selfjoin_pairs(g, path, cursor, bufs[i], None, cap, stream=stream)
        done += written
        emit_ms += st["ms_emit"]
        st_p = st if st_p is None else st_p
    if done != total:
        raise RuntimeError(f"pairs incomplete: {done}/{total}")
    st_p = dict(st_p or {"ms": 0.0})
    st_p["ms_emit"] = emit_ms
    if cref is not None:
        cref[w["name"]] = selfjoin_grid_info(g, stream=stream)["cand_ref"]
    if collect is not None:
        collect[i] = {"name": w["name"], "n": w["n"], "d": w["d"], "eps": w["eps"], "pairs": total,
                      "cand_eval": st_c["cand_eval"],
                      "build_ms": st_c["ms_build"],
                      "count_kernel_ms": st_c["ms_refine"], "emit_kernel_ms": st_p["ms_emit"],
                      "count_ms": st_c["ms"], "pairs_ms": st_p["ms"], "rechecked": st_c["rechecked"],
                      "path_run": st_c["path_run"],
                      "band_rel": st_c["band_rel"]}
    selfjoin_free_grid(g, stream=stream)


def one_pass(inputs, path, bufs, collect=None, cref=None, chunk=0, streams=None, order=None, cost=None):
    """build + count + pairs over every data set. `bufs[i]` is a device
    buffer able to hold data set i's pairs (None = size from the count).
    `cref` (dict, optional): filled with C_ref per data set (an extra pass
    over the cells; done outside the timed steps). With several streams one
    host thread per stream takes the next data set from a shared queue
    (`order`: longest first, from the warmup's per-set times) and runs it on
    its stream; the library's host waits release the interpreter, so the GPU
    interleaves the independent joins. `cost` (list, optional) receives each
    set's host wall time."""
    import threading
    import time

    import torch
    streams = streams or [torch.cuda.current_stream()]
    rec = [None] * len(inputs) if collect is not None else None
    errors = []
    queue = list(order if order is not None else range(len(inputs)))
    lock = threading.Lock()

    def work(t):
        try:
            with torch.cuda.stream(streams[t]):
                while True:
                    with lock:
                        if not queue:
                            return
                        i = queue.pop(0)
                    w, _, xt = inputs[i]
                    t0 = time.perf_counter()
                    one_dataset(i, w, xt, path, bufs, rec, cref, chunk, streams[t])
                    if cost is not None:
                        cost[i] = time.perf_counter() - t0
        except Exception as e:  # surfaced after join
            errors.append(e)

    if len(streams) == 1:
        work(0)
    else:
        th = [threading.Thread(target=work, args=(t,)) for t in range(len(streams))]
        for t in th:
            t.start()
        for t in th:
            t.join()
    if errors:
        raise errors[0]
    if collect is not None:
        collect.extend(rec)


def timed(inputs, path, steps, warmup, bufs, cref, chunk=0, streams=None, step_ms=None):
    """Mean seconds per timed step and the per-step records; `step_ms` (list,
    optional) receives each timed step's own wall time in ms (every step ends
    with its work finished)."""
    import torch
    cost = [0.0] * len(inputs)
    for i in range(warmup):
        one_pass(inputs, path, bufs, cref=cref if i == 0 else None, chunk=chunk, streams=streams, cost=cost)
    torch.cuda.synchronize()
    # longest first balances several streams; one stream keeps the listed order
    order = sorted(range(len(inputs)), key=lambda i: -cost[i]) if streams and len(streams) > 1 else None
    recs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        rec = []
        one_pass(inputs, path, bufs, rec, chunk=chunk, streams=streams, order=order)
        if step_ms is not None:
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - ts) * 1e3)
        for r in rec:
            r["cand_ref"] = cref[r["name"]]
        recs.append(rec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, recs


def src_hash():
    h = hashlib.sha256()
    for f in ("sj_refine.hip", "sj_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2209_11287_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key, path, workload):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, only if
    they were taken on the current kernel source, path and workload."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
        e = t.get(kernel_key)
        if e and e.get("src_hash") == src_hash() and e.get("path") == path and e.get("workload") == workload:
            return e.get("bytes_per_launch")
    except Exception:
        return None
    return None


def roofline(recs, path="fp64_mfma", which=None, workload="cfg2"):
    """Dominant tile kernel over the timed steps (or `which`: "emit" /
    "count"); algorithmic work per launch divided by its mean launch time
    (HIP events around the launch)."""
    per = {}
    for rec in recs:
        for r in rec:
            per.setdefault(r["name"], []).append(r)
    count_ms = sum(r["count_kernel_ms"] for rec in recs for r in rec)
    emit_ms = sum(r["emit_kernel_ms"] for rec in recs for r in rec)
    launches = sum(len(rec) for rec in recs)
    if which == "emit" or (which is None and emit_ms >= count_ms):
        # emit: pair rows written (8 B each) + each point's row read once
        byts = sum(8.0 * r["pairs"] + 8.0 * r["n"] * r["d"] + 4.0 * r["n"] for rec in recs for r in rec)
        avg_ms = emit_ms / launches
        achieved = byts / launches / (avg_ms * 1e-3) / 1e9
        kname = {"fp64_mfma": "k_m64", "fp64_valu": "k_v64", "fp32_mfma": "k_lowp<F32>",
                 "bf16_mfma": "k_lowp<BF16>", "bf16x3_mfma": "k_lowp<BF16X3>", "fp8_mfma": "k_lowp<FP8>"}[path]
        return {"kernel": kname + " emit (pairs)", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for("emit", path, workload), "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": round(byts / launches)}
    flops = sum(2.0 * r["d"] * r["cand_ref"] for rec in recs for r in rec)
    avg_ms = count_ms / launches
    achieved = flops / launches / (avg_ms * 1e-3) / 1e12
    peak = {"fp64_mfma": FP64_PEAK_TFLOPS, "fp64_valu": FP64_PEAK_TFLOPS, "fp32_mfma": 157.3,
            "bf16_mfma": 2500.0, "bf16x3_mfma": 2500.0, "fp8_mfma": 5000.0}[path]
    kname = {"fp64_mfma": "k_m64", "fp64_valu": "k_v64", "fp32_mfma": "k_lowp<F32>",
             "bf16_mfma": "k_lowp<BF16>", "bf16x3_mfma": "k_lowp<BF16X3>", "fp8_mfma": "k_lowp<FP8>"}[path]
    return {"kernel": kname + " count", "bound": "mfma" if path != "fp64_valu" else "alu",
            "achieved": round(achieved, 3),
            "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": traffic_for("count", path, workload), "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_flops_per_launch": round(flops / launches)}


PEAK_KEY = {("mfma", "fp64_mfma"): "fp64_mfma_tflops", ("alu", "fp64_valu"): "fp64_valu_tflops",
            ("mfma", "fp32_mfma"): "fp32_mfma_tflops", ("mfma", "bf16_mfma"): "bf16_mfma_tflops",
            ("mfma", "bf16x3_mfma"): "bf16_mfma_tflops", ("mfma", "fp8_mfma"): "fp8_mfma_tflops"}


def measured_peaks():
    """Achievable peaks of this GPU from the library's microbenchmarks
    (matrix forms, FP64 vector FMA, HBM read and copy over 4 GiB buffers)."""
    import paper_2209_11287_amd as pkg
    return {k: round(v, 1) for k, v in pkg.selfjoin_probe_peaks(4 << 30).items()}


def with_achievable(roof, peaks, path):
    """Adds the measured achievable peak of the roofline's unit (the HBM copy
    rate for an HBM-bound kernel) and the fraction of it reached."""
    if not peaks:
        return roof
    key = "hbm_copy_gbs" if roof["bound"] == "hbm" else PEAK_KEY.get((roof["bound"], path))
    if key:
        roof["achievable_peak"] = peaks[key]
        roof["achievable_source"] = key
        roof["frac_achievable"] = round(roof["achieved"] / peaks[key], 4)
    return roof


def isolated(inputs, path, bufs, cref_map, chunk=0):
    """One pass over every data set on a single stream with nothing else on
    the GPU: per-set kernel times of `path` (HIP events around each launch)."""
    iso = []
    one_pass(inputs, path, bufs, iso, chunk=chunk)
    for r in iso:
        r["cand_ref"] = cref_map[r["name"]]
    return iso


def cpu_baseline(inputs, budget_s=10.0):
    """The oracle, as it stands, on a bounded sample of the same workload:
    per data set (in order, until `budget_s` of CPU time), its self-join --
    build + count with all host threads of the box's share, then build +
    pair list into a preallocated host buffer (the oracle writes pairs on
    one thread) -- and the same count on one thread. Also the small parity
    workload (n = 20,000, d = 2) on one thread and on all."""
    import numpy as np

    import oracle
    from workloads import configs
    from workloads import generators as gen
    # the machine's CPU share: OMP_NUM_THREADS (16 per GPU), not os.cpu_count()
    nthreads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16"))))
    done, cref, secs, spent, one = [], 0, 0.0, 0.0, []
    for w, X, _ in inputs:
        t0 = time.perf_counter()
        total, _, c, _ = oracle.grid_count(X, w["eps"], nthreads=nthreads)
        t1 = time.perf_counter()
        buf = np.empty((max(total, 1), 2), dtype=np.int32)
        t2 = time.perf_counter()
        if oracle.grid_pairs_into(X, w["eps"], buf) != total:
            raise RuntimeError("oracle pairs disagree with its count")
        t3 = time.perf_counter()
        oracle.grid_count(X, w["eps"], nthreads=1)
        t4 = time.perf_counter()
        del buf
        cref += c
        secs += (t1 - t0) + (t3 - t2)
        spent += t4 - t0
        done.append(w["name"])
        one.append({"name": w["name"], "count_s": round(t1 - t0, 3), "pairs_1thread_s": round(t3 - t2, 3),
                    "count_1thread_s": round(t4 - t3, 3), "cand_ref": c,
                    "count_evals_per_s": round(c / (t1 - t0)), "count_1thread_evals_per_s": round(c / (t4 - t3))})
        if spent > budget_s:
            break
    sw = configs.workload("small")
    Xs = gen.make(sw["dist"], sw["n"], sw["d"], seed=sw["seed"])
    small = {}
    for th in (1, nthreads):
        t0 = time.perf_counter()
        _, _, cs, _ = oracle.grid_count(Xs, sw["eps"], nthreads=th)
        small[f"count_{th}thread_s"] = round(time.perf_counter() - t0, 4)
    small["cand_ref"] = cs
    return {"value": cref / secs, "unit": "distance evals/s", "cores": nthreads, "kind": "oracle",
            "sample": f"oracle self-join = build + count ({nthreads} threads) + build + pair list into a "
                      f"preallocated host buffer (1 thread), data sets: {', '.join(done)}",
            "seconds": round(secs, 2), "per_set": one, "small_n20000_d2": small}


def brute_compare(inputs, path, bufs, reps=3):
    """Index-free workload, per size: our build + count + pairs (index_dims =
    -1) and a dense reference in the role of the paper's WMMA-Ref -- the
    distance matrix |q|^2 + |c|^2 - 2 Q C^T from an FP64 GEMM (torch.matmul,
    rocBLAS / hipBLASLt) in blocks of 8192 rows, thresholded and counted on the
    device. Its rounding differs from the exact chain, so its count is
    reported, not compared. Median of `reps` runs each."""
    import statistics

    import torch
    out = []
    for i, (w, _, xt) in enumerate(inputs):
        n, eps2 = w["n"], w["eps"] * w["eps"]
        ours, ref = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            one_dataset(i, w, xt, path, bufs, None, None, 0, torch.cuda.current_stream())
            torch.cuda.synchronize()
            ours.append(time.perf_counter() - t0)
        xT = xt.t().contiguous()
        nrm = (xt * xt).sum(1)
        cnt = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = torch.zeros((), dtype=torch.int64, device=xt.device)
            for b0 in range(0, n, 8192):
                q = xt[b0:b0 + 8192]
                dmat = torch.matmul(q, xT).mul_(-2.0).add_(nrm[b0:b0 + 8192, None]).add_(nrm[None, :])
                c += (dmat <= eps2).sum()
                del dmat
            cnt = int(c)
            torch.cuda.synchronize()
            ref.append(time.perf_counter() - t0)
        del xT
        out.append({"n": n, "ms": round(statistics.median(ours) * 1e3, 3),
                    "gemm_reference_ms": round(statistics.median(ref) * 1e3, 3),
                    "gemm_reference_count": cnt})
    return out


def batched_setup():
    """The batched workload's problems on the device, their C_ref (the work
    unit) and algorithmic flops, computed outside any timed region."""
    import torch
    from paper_2209_11287_amd import selfjoin_build_grid, selfjoin_free_grid, selfjoin_grid_info
    from workloads import configs
    from workloads import generators as gen
    ws = configs.batched_workload()
    log(f"[bench] generating {len(ws)} batched problems")
    host = [gen.make(w["dist"], w["n"], w["d"], seed=w["seed"]) for w in ws]
    pts = [torch.from_numpy(X).to("cuda:0") for X in host]
    eps = [w["eps"] for w in ws]
    torch.cuda.synchronize()
    cref, flops, crefs = 0, 0, []
    for p, e in zip(pts, eps):
        g = selfjoin_build_grid(p, e)
        c = selfjoin_grid_info(g)["cand_ref"]
        crefs.append(c)
        cref += c
        flops += 2 * p.shape[1] * c
        selfjoin_free_grid(g)
    return {"ws": ws, "host": host, "pts": pts, "eps": eps, "cref": cref, "flops": flops, "crefs": crefs}


def batched_run(B, path, steps, warmup, cache):
    """`warmup` + `steps` steps of the batched workload on `path`. One step =
    build the batch (every problem's grid in one segmented build, the work
    queue, the in-mask buffer), count every problem (one graph launch), write
    every problem's pairs (one graph launch): all inside the timed region.
    The tuner's choices (index_dims and short-circuit per d, kernel
    schedule) are made in the first warmup step and cached in `cache`."""
    import torch
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_batch_info, selfjoin_batch_pairs)
    pts, eps = B["pts"], B["eps"]
    buf = None
    rec = []
    ks = []
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = selfjoin_batch_build(pts, eps, tune=True, tune_cache=cache)
        totals, st = selfjoin_batch_count(b, path)
        if buf is None:
            buf = torch.empty((max(1, sum(totals)), 2), dtype=torch.int32, device="cuda:0")
        _, st2 = selfjoin_batch_pairs(b, path, buf)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ks = sorted({(p.shape[1], selfjoin_batch_info(b, j)["index_dims"]) for j, p in enumerate(pts)})
        selfjoin_batch_free(b)
        if i >= warmup:
            rec.append({"s": t1 - t0, "build_ms": st["ms_build"], "count_ms": st["ms"], "pairs_ms": st2["ms"],
                        "pruned": st["tiles_pruned"], "pairs": sum(totals), "cand_eval": st["cand_eval"]})
        log(f"[bench] batched {path} step {i}: {1e3 * (t1 - t0):.1f} ms (build {st['ms_build']:.1f}, "
            f"count {st['ms']:.1f}, pairs {st2['ms']:.1f})")
    del buf
    torch.cuda.empty_cache()
    sec = sum(r["s"] for r in rec) / len(rec)
    avg = {k: round(sum(r[k] for r in rec) / len(rec), 3) for k in ("build_ms", "count_ms", "pairs_ms")}
    return sec, avg, rec[-1], ks


def batched_roofline(B, avg, last):
    count_s = avg["count_ms"] / 1e3
    pair_bytes = 8 * last["pairs"] + sum(8 * p.shape[0] * p.shape[1] + 4 * p.shape[0] for p in B["pts"])
    flops = B["flops"]
    return {"kernel": "batched count graph (one tile kernel per d)", "bound": "mfma",
            "achieved": round(flops / count_s / 1e12, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(flops / count_s / 1e12 / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "avg_launch_ms": avg["count_ms"], "algorithmic_flops_per_launch": flops,
            "note": "2 d C_ref flops per problem over the count graph's device time",
            "other_kernel": {"kernel": "batched pairs graph (in-mask expansion)", "bound": "hbm",
                             "achieved": round(pair_bytes / (avg["pairs_ms"] / 1e3) / 1e9, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(pair_bytes / (avg["pairs_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                             "avg_launch_ms": avg["pairs_ms"]}}


def batched_summary(paths, steps, warmup, B=None):
    """The batched workload on each of `paths`: per-step time, phases and
    the count graph's roofline."""
    import tempfile
    B = B or batched_setup()
    cache = os.path.join(tempfile.mkdtemp(), "tune.txt")
    out = {"workload": WORKLOAD_TEXT["batched"], "cand_ref_per_step": B["cref"], "steps": steps, "warmup": warmup,
           "paths": {}}
    for pth in paths:
        sec, avg, last, ks = batched_run(B, pth, steps, warmup, cache)
        out["paths"][pth] = {"ms_per_step": round(sec * 1e3, 3), "value": B["cref"] / sec, "phases_ms": avg,
                             "pairs": last["pairs"], "tiles_pruned": last["pruned"], "tuned_index_dims": ks,
                             "roofline": batched_roofline(B, avg, last)}
    return out


def batched_main(args):
    """The batched workload as the measured one (--workload batched)."""
    import tempfile
    B = batched_setup()
    cache = os.path.join(tempfile.mkdtemp(), "tune.txt")
    sec, avg, last, ks = batched_run(B, args.path, args.steps, args.warmup, cache)
    out = {"metric": METRIC, "value": B["cref"] / sec, "unit": "distance evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": WORKLOAD_TEXT["batched"], "path": args.path, "cand_ref_per_step": B["cref"],
                      "pairs_per_step": last["pairs"], "tuned_index_dims": ks},
           "phases_ms": avg, "tiles_pruned": last["pruned"], "cand_eval": last["cand_eval"],
           "roofline": batched_roofline(B, avg, last)}
    if not args.no_peaks:
        out["peaks_measured"] = measured_peaks()
        with_achievable(out["roofline"], out["peaks_measured"], args.path)
        with_achievable(out["roofline"]["other_kernel"], out["peaks_measured"], args.path)
    if args.compare:
        sec2, avg2, _, _ = batched_run(B, args.compare, args.steps, args.warmup, cache)
        out["compare"] = {"path": args.compare, "value": B["cref"] / sec2, "ms_per_step": round(sec2 * 1e3, 3),
                          "phases_ms": avg2, "speedup_of_headline": round(sec2 / sec, 3)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batched_cpu_baseline(B["ws"], B["host"], B["crefs"])
    print(json.dumps(out))


def batched_cpu_baseline(ws, host, crefs, budget_evals=1.5e9):
    """The oracle on a bounded sample of the batched workload: the problems,
    in order, whose C_ref still fits a budget of `budget_evals` candidate pairs
    (about 10 s of oracle work: its pair list runs on one thread), each its
    build + count (all threads) and build + pair list into a preallocated host
    buffer (one thread)."""
    import numpy as np

    import oracle
    nthreads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16"))))
    cref, secs, taken, used = 0, 0.0, [], 0
    for i, (w, X, c) in enumerate(zip(ws, host, crefs)):
        if used + c > budget_evals:
            continue
        used += c
        t0 = time.perf_counter()
        total, _, c2, _ = oracle.grid_count(X, w["eps"], nthreads=nthreads)
        t1 = time.perf_counter()
        buf = np.empty((max(total, 1), 2), dtype=np.int32)
        t2 = time.perf_counter()
        oracle.grid_pairs_into(X, w["eps"], buf)
        t3 = time.perf_counter()
        cref += c2
        secs += (t1 - t0) + (t3 - t2)
        taken.append(i)
    ds = sorted({ws[i]["d"] for i in taken})
    return {"value": cref / secs, "unit": "distance evals/s", "cores": nthreads, "kind": "oracle",
            "sample": f"oracle self-join (build + count on {nthreads} threads, build + pair list on one) of "
                      f"{len(taken)} of {len(ws)} batched problems (in order, up to {budget_evals:.1e} candidate "
                      f"pairs in all; d in {ds})", "seconds": round(secs, 2)}


def symmetric_counts(reps=3, B=None):
    """Count-only use (per-point counts, as DBSCAN's core test needs): the
    count kernel with the full stencil and with the half stencil
    (sj_opts.symmetric) on the same grids, FP64 MFMA and FP64 vector paths,
    the six 2M-point sets and the precision set; best of `reps` kernel times
    (HIP events around the launch); the totals must agree. With the batched
    workload's problems (B, from batched_setup), its count graph the same
    way (tuned builds, the device time of the graph launch)."""
    import tempfile

    import torch
    from paper_2209_11287_amd import (selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                                      selfjoin_build_grid, selfjoin_count, selfjoin_free_grid)
    out = {}
    if B is not None:
        log("[bench] symmetric count batched")
        cache = os.path.join(tempfile.mkdtemp(), "tune.txt")
        res = {}
        for pth in ("fp64_mfma", "fp64_valu"):
            r = {}
            for sym in (0, 1):
                b = selfjoin_batch_build(B["pts"], B["eps"], tune=True, tune_cache=cache, symmetric=sym)
                best, tot, ev = None, None, None
                for _ in range(reps + 1):
                    t, st = selfjoin_batch_count(b, pth)
                    best = st["ms"] if best is None else min(best, st["ms"])
                    tot, ev = t, st["cand_eval"]
                selfjoin_batch_free(b)
                r[sym] = (best, tot, ev)
            if r[0][1] != r[1][1]:
                raise RuntimeError(f"symmetric batched count differs on {pth}")
            res[pth] = {"count_graph_ms": round(r[0][0], 3), "symmetric_ms": round(r[1][0], 3),
                        "speedup": round(r[0][0] / max(r[1][0], 1e-9), 3), "cand_eval": r[0][2],
                        "symmetric_cand_eval": r[1][2]}
        out["batched"] = res
        torch.cuda.empty_cache()
    for wname in ("cfg2", "prec"):
        log(f"[bench] symmetric count {wname}")
        rows = []
        for w, _, xt in load_inputs(datasets(wname)):
            row = {"name": w["name"]}
            for pth in ("fp64_mfma", "fp64_valu"):
                res = {}
                for sym in (0, 1):
                    g = selfjoin_build_grid(xt, w["eps"], symmetric=sym)
                    best, tot, ev = None, None, None
                    for _ in range(reps + 1):
                        t, _, st = selfjoin_count(g, pth)
                        best = st["ms_refine"] if best is None else min(best, st["ms_refine"])
                        tot, ev = t, st["cand_eval"]
                    selfjoin_free_grid(g)
                    res[sym] = (best, tot, ev)
                if res[0][1] != res[1][1]:
                    raise RuntimeError(f"symmetric count differs on {w['name']} {pth}")
                row[pth] = {"count_kernel_ms": round(res[0][0], 4), "symmetric_ms": round(res[1][0], 4),
                            "speedup": round(res[0][0] / max(res[1][0], 1e-9), 3),
                            "cand_eval": res[0][2], "symmetric_cand_eval": res[1][2]}
            rows.append(row)
            del xt
            torch.cuda.empty_cache()
        out[wname] = rows
    return out


def other_workloads(steps=2, warmup=1):
    """Short timed passes of the other configurations, one stream each, so
    that one run reports them all: the precision set (1M-point Gaussian
    mixture, d = 16, 32, 64) on the FP64 MFMA, FP32 and split-BF16 MFMA and
    FP64 vector paths, with the low-precision paths' measured largest
    |Gram value - exact d^2| against their band; the 10M-point exponential
    set on the FP64 MFMA, FP32 MFMA and FP64 vector paths; the batched
    workload on both FP64 paths. Each: build + count + full pair list per
    step (the batched form as in --workload batched)."""
    import torch
    from paper_2209_11287_amd import selfjoin_build_grid, selfjoin_free_grid, selfjoin_measure_error
    out = {}
    for wname, paths in (("prec", ["fp64_mfma", "fp32_mfma", "bf16x3_mfma", "fp64_valu"]),
                         ("skewed", ["fp64_mfma", "fp32_mfma", "fp64_valu"])):
        log(f"[bench] other workload {wname}")
        inputs = load_inputs(datasets(wname))
        cref_map, res = {}, {}
        for pth in paths:
            bufs = [None] * len(inputs)
            sec, recs = timed(inputs, pth, steps, warmup, bufs, cref_map, 0, None)
            cref = sum(r["cand_ref"] for r in recs[0])
            res[pth] = {"ms_per_step": round(sec * 1e3, 3), "value": cref / sec,
                        "per_set": [{"name": r["name"], "count_kernel_ms": round(r["count_kernel_ms"], 3),
                                     "emit_kernel_ms": round(r["emit_kernel_ms"], 3),
                                     "build_ms": round(r["build_ms"], 3), "rechecked": r["rechecked"],
                                     "band_rel": r["band_rel"], "pairs": r["pairs"]} for r in recs[-1]]}
            del bufs
            torch.cuda.empty_cache()
            if wname == "prec" and pth in ("fp32_mfma", "bf16x3_mfma"):
                # the tiles' largest error before the recheck, against the band
                for r, (w, _, xt) in zip(res[pth]["per_set"], inputs):
                    g = selfjoin_build_grid(xt, w["eps"])
                    err, band, viol = selfjoin_measure_error(g, pth)
                    selfjoin_free_grid(g)
                    r["max_abs_err_d2"] = err
                    r["band_half_width"] = band
                    r["band_violations"] = viol
        out[wname] = {"workload": WORKLOAD_TEXT[wname], "cand_ref_per_step": sum(cref_map.values()),
                      "steps": steps, "warmup": warmup, "streams": 1, "paths": res}
        del inputs
        torch.cuda.empty_cache()
    log("[bench] other workload batched")
    B = batched_setup()
    out["batched"] = batched_summary(["fp64_mfma", "fp64_valu"], steps, warmup, B)
    out["symmetric_count"] = symmetric_counts(B=B)
    del B
    return out


def main():
    args = parse()
    if args.compare in ("", "none"):
        args.compare = ""
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described, not implemented)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    import paper_2209_11287_amd as pkg
    pkg.load()
    if args.workload == "batched":
        batched_main(args)
        return
    wl = datasets(args.workload)
    log(f"[bench] generating {len(wl)} data sets")
    inputs = load_inputs(wl)
    bufs = [None] * len(inputs)
    if args.copy_probe_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    streams = [torch.cuda.Stream() for _ in range(max(1, args.streams))] if args.streams > 1 else None
    log(f"[bench] path {args.path}: warmup {args.warmup}, steps {args.steps}, streams {max(1, args.streams)}")
    cref_map = {}
    step_ms = []
    sec, recs = timed(inputs, args.path, args.steps, max(1, args.warmup), bufs, cref_map, args.chunk, streams,
                      step_ms=step_ms)
    cref = sum(r["cand_ref"] for r in recs[0])
    pairs = sum(r["pairs"] for r in recs[0])
    out = {
        "metric": METRIC,
        "value": cref / sec,
        "unit": "distance evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 3),
        "step_ms": {"min": round(min(step_ms), 3), "median": round(statistics.median(step_ms), 3),
                    "max": round(max(step_ms), 3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # tiles in the path's precision, FP64 recheck of the band
        "dtype": {"fp32_mfma": "f32+f64", "bf16_mfma": "bf16+f64", "bf16x3_mfma": "bf16x3+f64",
                  "fp8_mfma": "fp8+f64"}.get(args.path, "f64"),
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "path": args.path, "cand_ref_per_step": cref, "pairs_per_step": pairs,
                   "chunk": args.chunk, "streams": max(1, args.streams)},
        "per_dataset": [{k: (round(v, 4) if isinstance(v, float) and k != "eps" else v) for k, v in r.items()}
                        for r in recs[-1]],
    }
    # roofline of the dominant tile kernel from single-stream launches (nothing
    # else on the GPU: the duration rocprofv3 reports for the same launches);
    # with several streams the timed steps' launch times include sharing the
    # GPU with the other streams' kernels, kept under "shared"
    if streams:
        # one untimed pass on the single stream first: the library's caching
        # allocator keeps blocks per stream, so a first pass there would time
        # fresh allocations (and their first touch) instead of the kernels
        one_pass(inputs, args.path, bufs, None, chunk=args.chunk)
    iso = isolated(inputs, args.path, bufs, cref_map, args.chunk) if streams else recs[-1]
    cnt_iso = sum(r["count_kernel_ms"] for r in iso)
    emit_iso = sum(r["emit_kernel_ms"] for r in iso)
    kind = "emit" if emit_iso >= cnt_iso else "count"
    roof = roofline([iso], args.path, which=kind, workload=args.workload)
    roof["note"] = ("launch times from HIP events on the launching stream, one pass over the data sets on a "
                    "single stream" + (" after the timed steps" if streams else " (the last timed step)"))
    if streams:
        rs = roofline(recs, args.path, which=kind, workload=args.workload)
        roof["shared"] = {"avg_launch_ms": rs["avg_launch_ms"], "achieved": rs["achieved"], "frac": rs["frac"],
                          "note": f"the timed steps' launches, {len(streams)} streams sharing the GPU"}
    other = "count" if kind == "emit" else "emit"
    ro = roofline([iso], args.path, which=other, workload=args.workload)
    roof["other_kernel"] = {k: ro[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac",
                                                  "avg_launch_ms")}
    if not args.no_peaks:
        log("[bench] achievable peaks (microbenchmarks)")
        out["peaks_measured"] = measured_peaks()
        with_achievable(roof, out["peaks_measured"], args.path)
        with_achievable(roof["other_kernel"], out["peaks_measured"], args.path)
    out["roofline"] = roof
    # per-set single-stream kernel times of the FP64 MFMA, FP64 vector-ALU and
    # FP32 MFMA paths on the same data (the MFMA-vs-vector comparison per set)
    if args.workload in ("cfg2", "skewed", "prec") and not args.no_per_set:
        per = {}
        for pth in dict.fromkeys([args.path, "fp64_mfma", "fp64_valu", "fp32_mfma", "bf16x3_mfma"]):
            if pth == args.path and iso is not recs[-1]:
                rr = iso
            else:
                b2 = [None] * len(inputs)
                one_pass(inputs, pth, b2, None, chunk=args.chunk)  # warm
                rr = isolated(inputs, pth, b2, cref_map, args.chunk)
                del b2
            per[pth] = {r["name"]: {"build_ms": round(r["build_ms"], 4), "count_kernel_ms": round(r["count_kernel_ms"], 4),
                                    "emit_kernel_ms": round(r["emit_kernel_ms"], 4),
                                    "rechecked": r["rechecked"], "band_rel": r["band_rel"]} for r in rr}
        names = [r["name"] for r in iso]
        out["per_set_isolated"] = per
        out["mfma_vs_valu_count"] = {nm: round(per["fp64_valu"][nm]["count_kernel_ms"] /
                                               max(per["fp64_mfma"][nm]["count_kernel_ms"], 1e-9), 3) for nm in names}
    if args.workload == "brute":
        log("[bench] per-size times and the dense GEMM reference")
        per = brute_compare(inputs, args.path, bufs)
        for r, rec in zip(per, recs[-1]):
            r["pairs"] = rec["pairs"]
        out["per_size"] = per
    if args.compare:
        log(f"[bench] compare path {args.compare}")
        bufs2 = [None] * len(inputs)
        sec2, recs2 = timed(inputs, args.compare, args.steps, max(1, args.warmup), bufs2, {}, args.chunk, streams)
        for rec in recs2:
            for r in rec:
                r["cand_ref"] = cref_map[r["name"]]
        out["compare"] = {"path": args.compare, "value": cref / sec2, "ms_per_step": round(sec2 * 1e3, 3),
                          "speedup_of_headline": round(sec2 / sec, 3),
                          "count_kernel_ms": [round(r["count_kernel_ms"], 4) for r in recs2[-1]],
                          "emit_kernel_ms": [round(r["emit_kernel_ms"], 4) for r in recs2[-1]]}
        del bufs2
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(inputs)
    if args.workload == "cfg2" and not args.no_other:
        del bufs
        inputs = None
        torch.cuda.empty_cache()
        out["other_workloads"] = other_workloads()
    print(json.dumps(out))


if __name__ == "__main__":
    main()

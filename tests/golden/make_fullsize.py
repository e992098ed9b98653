"""Writes tests/golden/fullsize.json: the oracle's results on the full-size
workloads, for the GPU tests that compare whole results at those sizes.

Calls only the oracle (oracle/) and the seeded input generators (workloads/).
Per data set it stores the input's sha256 (so a change of the generator is
caught as such), |R| (Eq. (1) of Section II-A over all ordered pairs, the
self-pairs included), C_ref and the indexed dimension count of the reference
grid, the two order-independent pair-set checksums (oracle.grid_digest), and
the sha256 of the per-point counts (int32, little-endian, input order).

    python tests/golden/make_fullsize.py [--only cfg2,prec,skewed,batched] [--jobs 8]

The batched workload's 256 problems run in a process pool (one oracle thread
each: most of their cost sits in the few cells of the 8- and 16-dimensional
problems, which the oracle's cell-parallel threads cannot split).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "fullsize.json")


def _entry(w, nthreads):
    import numpy as np

    import oracle
    from workloads import generators as gen
    X = gen.make(w["dist"], w["n"], w["d"], seed=w["seed"])
    t0 = time.time()
    total, pp, cref, k, dig = oracle.grid_digest(X, w["eps"], nthreads=nthreads)
    return {"name": w["name"], "dist": w["dist"], "n": w["n"], "d": w["d"], "seed": w["seed"],
            "eps": w["eps"], "x_sha256": hashlib.sha256(X.tobytes()).hexdigest(),
            "total": int(total), "cand_ref": int(cref), "k": int(k),
            "digest": [str(dig[0]), str(dig[1])],
            "counts_sha256": hashlib.sha256(pp.astype("<i4").tobytes()).hexdigest(),
            "oracle_s": round(time.time() - t0, 2)}


def _batch_one(w):
    return _entry(w, 1)


def main():
    from workloads import configs
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="cfg2,prec,skewed,batched")
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    parts = a.only.split(",")
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    named = {"cfg2": configs.CFG2, "prec": configs.PREC, "skewed": configs.SKEWED}
    for part in ("cfg2", "prec", "skewed"):
        if part not in parts:
            continue
        for nm in named[part]:
            e = _entry(configs.workload(nm), a.jobs)
            data[nm] = e
            print(nm, e["total"], e["oracle_s"], "s", flush=True)
            json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
    if "batched" in parts:
        ws = configs.batched_workload()
        # longest first: near brute force for d = 8, 16
        order = sorted(range(len(ws)), key=lambda b: -ws[b]["n"] ** 2 * ws[b]["d"])
        res = [None] * len(ws)
        with ProcessPoolExecutor(max_workers=a.jobs) as ex:
            futs = {b: ex.submit(_batch_one, ws[b]) for b in order}
            for done, b in enumerate(order):
                res[b] = futs[b].result()
                print("batch", b, res[b]["n"], res[b]["d"], res[b]["oracle_s"], "s",
                      f"({done + 1}/{len(ws)})", flush=True)
        data["batched"] = {"count": len(ws), "seed": 0, "s": 32.0, "problems": res}
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()

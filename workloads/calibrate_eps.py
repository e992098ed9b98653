"""Calibrates the search distance of each synthetic workload to a target
selectivity s = (|R| - n) / n (Section IV-A), using only the CPU oracle, and
writes workloads/eps.json. The paper's figures (which carry its eps values)
are not available, so eps is set per workload from the selectivity.

Bisection on log(eps) over the oracle's grid count restricted to a seeded
sample of queries; stops at 2% of the target and freezes eps to 4
significant digits.

    python -m workloads.calibrate_eps [--only NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs, generators  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "eps.json")


def selectivity(X, eps, sample):
    counts, _ = oracle.grid_count_sample(X, eps, sample)
    return float(counts.mean() - 1.0)


def calibrate(X, target, guess, nsample=20000, seed=0):
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    sample = rng.choice(n, size=min(n, nsample), replace=False)
    lo, hi = guess / 4, guess * 4
    s_lo, s_hi = selectivity(X, lo, sample), selectivity(X, hi, sample)
    while s_lo > target:
        lo /= 2
        s_lo = selectivity(X, lo, sample)
    while s_hi < target:
        hi *= 2
        s_hi = selectivity(X, hi, sample)
    eps = guess
    for _ in range(40):
        eps = math.sqrt(lo * hi)
        s = selectivity(X, eps, sample)
        if abs(s / target - 1) < 0.02:
            break
        if s < target:
            lo = eps
        else:
            hi = eps
    return float(f"{eps:.4g}"), s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    table = {}
    if os.path.exists(OUT):
        table = json.load(open(OUT))
    for w in configs.calibration_list():
        if args.only and w["name"] != args.only:
            continue
        X = generators.make(w["dist"], w["n"], w["d"], seed=w["seed"])
        eps, s = calibrate(X, w["target_s"], w["guess"])
        table[w["name"]] = {"eps": eps, "target_s": w["target_s"], "sample_s": round(s, 3)}
        print(w["name"], table[w["name"]], flush=True)
        json.dump(table, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()

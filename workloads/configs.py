"""The synthetic workloads (shapes of the paper's Section IV datasets, Table I:
uniform and exponential sets, d in {2, 3, 4}, n in the millions), with search
distances calibrated to a target selectivity by calibrate_eps.py (oracle
only) and frozen in eps.json.

  small   : n = 20,000, d = 2, uniform, seed 0, eps = 0.0218 (s ~ 29)
  cfg2    : n = 2,000,000, d in {2, 3, 4}, uniform and exponential(40),
            eps for s ~ 64 -- the measured workload
  prec    : n = 1,000,000, d in {16, 32, 64}, Gaussian mixture, s ~ 50
  skewed  : n = 10,000,000, d = 3, exponential(40), s ~ 100
  brute   : index-free mode (one cell, every ordered pair a candidate) on
            d = 16, exponential(40), n = 2^11 .. 2^17 (Fig. 3's sizes), one
            eps for all sizes, calibrated for s ~ 64 at n = 2^17
"""
from __future__ import annotations

import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_EPS = os.path.join(_HERE, "eps.json")

# first guesses (closed-form / Monte-Carlo estimates), refined by calibration
_GUESS = {
    "uniform_d2_n2M": 0.003196, "uniform_d3_n2M": 0.01984, "uniform_d4_n2M": 0.05136,
    "expo_d2_n2M": 1.600e-4, "expo_d3_n2M": 9.996e-4, "expo_d4_n2M": 2.614e-3,
    "gmm_d16_n1M": 0.0641, "gmm_d32_n1M": 0.1100, "gmm_d64_n1M": 0.1757,
    "expo_d3_n10M": 6.750e-4,
    "expo_d16_n131072": 0.05,
}


def _entry(name, dist, n, d, target_s, seed=0):
    return {"name": name, "dist": dist, "n": n, "d": d, "target_s": target_s, "seed": seed,
            "guess": _GUESS[name]}


def calibration_list():
    out = []
    for dist in ("uniform", "expo"):
        for d in (2, 3, 4):
            out.append(_entry(f"{dist}_d{d}_n2M", dist, 2_000_000, d, 64.0))
    for d in (16, 32, 64):
        out.append(_entry(f"gmm_d{d}_n1M", "gmm", 1_000_000, d, 50.0))
    out.append(_entry("expo_d3_n10M", "expo", 10_000_000, 3, 100.0))
    out.append(_entry("expo_d16_n131072", "expo", 1 << 17, 16, 64.0))
    return out


def eps_table():
    if os.path.exists(_EPS):
        return json.load(open(_EPS))
    return {}


def workload(name):
    """Dict with dist, n, d, seed, eps for a named workload."""
    if name == "small":
        return {"name": "small", "dist": "uniform", "n": 20000, "d": 2, "seed": 0, "eps": 0.0218}
    for w in calibration_list():
        if w["name"] == name:
            tab = eps_table()
            eps = tab.get(name, {}).get("eps", w["guess"])
            return {"name": name, "dist": w["dist"], "n": w["n"], "d": w["d"], "seed": w["seed"],
                    "eps": eps}
    raise KeyError(name)


def brute_workloads():
    """The index-free sizes: 16-D exponential(40), n = 2^11 .. 2^17, one eps."""
    eps = workload("expo_d16_n131072")["eps"]
    return [{"name": f"brute_expo_d16_n{1 << e}", "dist": "expo", "n": 1 << e, "d": 16, "seed": 0,
             "eps": eps} for e in range(11, 18)]


CFG2 = [f"{dist}_d{d}_n2M" for dist in ("uniform", "expo") for d in (2, 3, 4)]
PREC = [f"gmm_d{d}_n1M" for d in (16, 32, 64)]
SKEWED = ["expo_d3_n10M"]


def batch_eps(n: int, d: int, s: float) -> float:
    """Search distance for about `s` mean neighbours among n uniform points in
    [0,1]^d, from the volume of the d-ball (boundary losses ignored)."""
    import math
    vol = math.pi ** (d / 2) / math.gamma(d / 2 + 1)
    return float((s / max(n - 1, 1) / vol) ** (1.0 / d))


def batched_workload(count: int = 256, seed: int = 0, s: float = 32.0):
    """The batched workload: `count` independent problems, n log-uniform in
    [1e3, 2e5], d from {2, 3, 4, 8, 16}, uniform points (problem b drawn with
    seed [seed, b]), eps for ~s mean neighbours each. Returns a list of dicts
    with n, d, seed, eps."""
    from workloads import generators as gen
    return [{"name": f"batch{b}", "dist": "uniform", "n": n, "d": d, "seed": [seed, b],
             "eps": batch_eps(n, d, s)}
            for b, (n, d) in enumerate(gen.batch_problems(count, seed=seed))]

"""Helpers for the GPU tests: run the HIP path through the C ABI, compare with
the oracle as pair sets (the result set is unique, its order is not)."""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pair_keys(pairs) -> np.ndarray:
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return np.sort((p[:, 0] << 32) | p[:, 1])


def gpu_join(X: np.ndarray, eps: float, path: str, want_pairs=True, want_d2=False, capacity=None,
             index_dims=0, short_circuit=0, dim_order=0, symmetric=0):
    """Runs build + count (+ pairs) on cuda:0. Returns dict of host arrays."""
    import torch
    from paper_2209_11287_amd import SelfJoin, selfjoin_grid_info

    xt = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    sj = SelfJoin(xt, eps, index_dims=index_dims, short_circuit=short_circuit, dim_order=dim_order,
                  symmetric=symmetric)
    try:
        total, pp, st = sj.count(path, per_point=True)
        out = {"total": total, "per_point": pp.cpu().numpy() if pp is not None else None, "stats": st,
               "info": selfjoin_grid_info(sj.grid)}
        if want_pairs:
            r = sj.all_pairs(path, want_d2=want_d2, capacity=capacity)
            if want_d2:
                out["pairs"] = r[0].cpu().numpy()
                out["d2"] = r[1].cpu().numpy()
            else:
                out["pairs"] = r.cpu().numpy()
        torch.cuda.synchronize()
        return out
    finally:
        sj.close()


# Pair-set checksums on the device (test bookkeeping): the sums modulo 2^64
# of SplitMix64's finaliser of key = i * 2^32 + j and of key + G over the
# pairs (i, j), as oracle.grid_digest / oracle.pairs_digest compute them on
# the CPU. int64 arithmetic wraps like uint64; right shifts are made logical
# by masking.
_M1 = 0xbf58476d1ce4e5b9 - (1 << 64)
_M2 = 0x94d049bb133111eb - (1 << 64)
_G = 0x9e3779b97f4a7c15 - (1 << 64)


def _srl(z, s):
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix_t(z):
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def digest_pairs_t(pairs_t, step: int = 1 << 26):
    """Checksums of an (m, 2) int32 tensor of pairs (any device), in chunks of
    `step` rows; returns two Python ints in [0, 2^64)."""
    import torch
    a = torch.zeros((), dtype=torch.int64, device=pairs_t.device)
    b = torch.zeros((), dtype=torch.int64, device=pairs_t.device)
    for s in range(0, pairs_t.shape[0], step):
        p = pairs_t[s:s + step]
        key = (p[:, 0].to(torch.int64) << 32) | p[:, 1].to(torch.int64)
        a += _mix_t(key).sum()
        b += _mix_t(key + _G).sum()
    return int(a) % (1 << 64), int(b) % (1 << 64)


def add_digest(x, y):
    return (x[0] + y[0]) % (1 << 64), (x[1] + y[1]) % (1 << 64)

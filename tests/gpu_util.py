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
             index_dims=0):
    """Runs build + count (+ pairs) on cuda:0. Returns dict of host arrays."""
    import torch
    from paper_2209_11287_amd import SelfJoin, selfjoin_grid_info

    xt = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    sj = SelfJoin(xt, eps, index_dims=index_dims)
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

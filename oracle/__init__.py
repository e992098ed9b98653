"""CPU oracle for the epsilon-distance self-join -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It loads `liboracle.so`, compiled from
`selfjoin_oracle.c` by `build()` with gcc; it never imports the product
package and shares no code with it.

Every function follows the definitions cited in `selfjoin_oracle.c`:
Eq. (1) of Section II-A (distance, self-join), Eq. (2) of Section III-A
(dimension-ascending multiply-accumulate order), Section IV-A (self-pairs in
the result), and the uniform eps-grid of Sections II-D and III-B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "selfjoin_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no FP contraction, portable -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_d2.restype = ctypes.c_double
        lib.oracle_d2.argtypes = [_f64p, _f64p, ctypes.c_int]
        lib.oracle_eps2.restype = ctypes.c_double
        lib.oracle_eps2.argtypes = [ctypes.c_double]
        lib.oracle_cell_side.restype = ctypes.c_double
        lib.oracle_cell_side.argtypes = [ctypes.c_double]
        lib.oracle_bruteforce.restype = _i64
        lib.oracle_bruteforce.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double,
                                          _i32p, _i32p, _i64]
        lib.oracle_query.restype = _i64
        lib.oracle_query.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double, _i64,
                                     _i32p, _i64]
        lib.oracle_grid_count.restype = _i64
        lib.oracle_grid_count.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_int, _i32p, _i64p,
                                          ctypes.POINTER(ctypes.c_int)]
        lib.oracle_grid_pairs.restype = _i64
        lib.oracle_grid_pairs.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double,
                                          _i32p, _i32p, _f64p, _i64]
        lib.oracle_grid_digest.restype = _i64
        lib.oracle_grid_digest.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, _i32p, _i64p,
                                           ctypes.POINTER(ctypes.c_int), _u64p]
        lib.oracle_pairs_digest.restype = None
        lib.oracle_pairs_digest.argtypes = [_i32p, _i64, _u64p]
        lib.oracle_grid_count_sample.restype = _i64
        lib.oracle_grid_count_sample.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_double,
                                                 _i64p, _i64, _i32p, _i64p]
        _lib = lib
    return _lib


def _pts(X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2:
        raise ValueError("points must be an (n, d) array")
    return X


def _ptr(a, t):
    return a.ctypes.data_as(t)


def d2(a, b) -> float:
    """Squared distance in the order of Eq. (2): fma chain from +0.0."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return _load().oracle_d2(_ptr(a, _f64p), _ptr(b, _f64p), a.shape[0])


def eps2(eps: float) -> float:
    return _load().oracle_eps2(eps)


def cell_side(eps: float) -> float:
    return _load().oracle_cell_side(eps)


def bruteforce(X, eps, want_pairs=True):
    """All ordered pairs by brute force. Returns (count, per_point, pairs)."""
    X = _pts(X)
    n, d = X.shape
    lib = _load()
    pp = np.zeros(n, dtype=np.int32)
    total = lib.oracle_bruteforce(_ptr(X, _f64p), n, d, eps, _ptr(pp, _i32p), None, 0)
    if total < 0:
        raise ValueError("invalid input")
    pairs = None
    if want_pairs:
        pairs = np.zeros((max(total, 1), 2), dtype=np.int32)
        lib.oracle_bruteforce(_ptr(X, _f64p), n, d, eps, None, _ptr(pairs, _i32p), total)
        pairs = pairs[:total]
    return total, pp, pairs


def query(X, eps, q) -> np.ndarray:
    """Brute-force range query of point q: sorted indices j within eps."""
    X = _pts(X)
    n, d = X.shape
    lib = _load()
    c = lib.oracle_query(_ptr(X, _f64p), n, d, eps, int(q), None, 0)
    if c < 0:
        raise ValueError("invalid input")
    js = np.zeros(max(c, 1), dtype=np.int32)
    lib.oracle_query(_ptr(X, _f64p), n, d, eps, int(q), _ptr(js, _i32p), c)
    return js[:c]


def grid_count(X, eps, nthreads=None):
    """Grid self-join count. Returns (count, per_point, C_ref, k)."""
    X = _pts(X)
    n, d = X.shape
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    lib = _load()
    pp = np.zeros(n, dtype=np.int32)
    cref = ctypes.c_int64(0)
    k = ctypes.c_int(0)
    total = lib.oracle_grid_count(_ptr(X, _f64p), n, d, eps, int(nthreads), _ptr(pp, _i32p),
                                  ctypes.byref(cref), ctypes.byref(k))
    if total < 0:
        raise ValueError("invalid input")
    return total, pp, cref.value, k.value


def grid_pairs(X, eps, want_d2=False):
    """Grid self-join pair list. Returns (count, per_point, pairs[, d2])."""
    X = _pts(X)
    n, d = X.shape
    lib = _load()
    total, pp, _, _ = grid_count(X, eps)
    pairs = np.zeros((max(total, 1), 2), dtype=np.int32)
    dd = np.zeros(max(total, 1), dtype=np.float64) if want_d2 else None
    t2 = lib.oracle_grid_pairs(_ptr(X, _f64p), n, d, eps, None, _ptr(pairs, _i32p),
                               _ptr(dd, _f64p) if want_d2 else None, total)
    if t2 != total:
        raise RuntimeError("oracle grid pairs disagree with grid count")
    if want_d2:
        return total, pp, pairs[:total], dd[:total]
    return total, pp, pairs[:total]


def grid_pairs_into(X, eps, pairs):
    """Grid self-join pair list written into a preallocated (cap, 2) int32
    C-contiguous array (rows beyond cap are counted, not written). Returns
    |R|."""
    X = _pts(X)
    n, d = X.shape
    if pairs.dtype != np.int32 or pairs.ndim != 2 or pairs.shape[1] != 2 or not pairs.flags.c_contiguous:
        raise ValueError("pairs must be a C-contiguous (cap, 2) int32 array")
    t = _load().oracle_grid_pairs(_ptr(X, _f64p), n, d, eps, None, _ptr(pairs, _i32p), None, pairs.shape[0])
    if t < 0:
        raise ValueError("invalid input")
    return t


def grid_digest(X, eps, nthreads=None):
    """Grid self-join count with the pair-set checksums (test bookkeeping: the
    sums modulo 2^64 of two SplitMix64 mixes of key = i * 2^32 + j over the
    pairs (i, j); independent of pair order and chunking).
    Returns (count, per_point, C_ref, k, (sum0, sum1))."""
    X = _pts(X)
    n, d = X.shape
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    lib = _load()
    pp = np.zeros(n, dtype=np.int32)
    cref = ctypes.c_int64(0)
    k = ctypes.c_int(0)
    sums = np.zeros(2, dtype=np.uint64)
    total = lib.oracle_grid_digest(_ptr(X, _f64p), n, d, eps, int(nthreads), _ptr(pp, _i32p),
                                   ctypes.byref(cref), ctypes.byref(k), _ptr(sums, _u64p))
    if total < 0:
        raise ValueError("invalid input")
    return total, pp, cref.value, k.value, (int(sums[0]), int(sums[1]))


def pairs_digest(pairs):
    """The same two checksums of an explicit (m, 2) int32 pair list."""
    p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    sums = np.zeros(2, dtype=np.uint64)
    _load().oracle_pairs_digest(_ptr(p, _i32p), p.shape[0], _ptr(sums, _u64p))
    return int(sums[0]), int(sums[1])


def grid_count_sample(X, eps, queries):
    """Per-query counts for the listed queries through the grid.
    Returns (counts, C_ref restricted to those queries)."""
    X = _pts(X)
    n, d = X.shape
    q = np.ascontiguousarray(queries, dtype=np.int64)
    counts = np.zeros(max(len(q), 1), dtype=np.int32)
    cref = ctypes.c_int64(0)
    t = _load().oracle_grid_count_sample(_ptr(X, _f64p), n, d, eps, _ptr(q, _i64p), len(q),
                                         _ptr(counts, _i32p), ctypes.byref(cref))
    if t < 0:
        raise ValueError("invalid input")
    return counts[:len(q)], cref.value


def knn_within_eps(X, eps, k):
    """k nearest neighbours of every point among the points within eps of it
    (the self-join result R of Eq. (1), Section II-A, reused for kNN as
    Section I names it), the point itself excluded, ordered by the exact
    squared distance of Eq. (2) and then by the smaller index.
    Returns (nbr [n, k] int32, -1 past the end; d2 [n, k], +inf past the
    end; found [n] int32)."""
    X = _pts(X)
    n = X.shape[0]
    _, _, pairs, dd = grid_pairs(X, eps, want_d2=True)
    i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    keep = i != j
    i, j, dd = i[keep], j[keep], dd[keep]
    order = np.lexsort((j, dd, i))  # by query, then distance, then index
    i, j, dd = i[order], j[order], dd[order]
    nbr = np.full((n, k), -1, dtype=np.int32)
    out_d2 = np.full((n, k), np.inf, dtype=np.float64)
    found = np.zeros(n, dtype=np.int32)
    starts = np.searchsorted(i, np.arange(n))
    ends = np.searchsorted(i, np.arange(n), side="right")
    for q in range(n):
        m = min(k, ends[q] - starts[q])
        nbr[q, :m] = j[starts[q]:starts[q] + m]
        out_d2[q, :m] = dd[starts[q]:starts[q] + m]
        found[q] = m
    return nbr, out_d2, found

"""Python binding of the MI355X epsilon-distance self-join (include/selfjoin.h).

PyTorch supplies device memory and the current stream only; every step runs
in libselfjoin.so. Functions carry the C ABI's names:

    g = selfjoin_build_grid(points_cuda_f64, eps)
    total, per_point, stats = selfjoin_count(g, "fp64_mfma", per_point=True)
    written, nxt, stats = selfjoin_pairs(g, "fp64_mfma", cursor, pairs, d2)
    selfjoin_free_grid(g)

`SelfJoin` wraps the same calls for convenience.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import PATHS, SelfJoinError, check


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _path_id(path) -> int:
    if isinstance(path, int):
        return path
    try:
        return PATHS[path]
    except KeyError:
        raise ValueError(f"unknown path {path!r}; one of {sorted(PATHS)}") from None


class GridHandle:
    """Owns a sj_grid*; freed on close() or garbage collection."""

    def __init__(self, ptr, n, d, eps, device):
        self.ptr = ptr
        self.n = n
        self.d = d
        self.eps = eps
        self.device = device
        self.hook = None  # allocator hook of the handle (must outlive it)

    def close(self, stream=None):
        if self.ptr:
            lib = _lib.load()
            torch = _torch()
            with torch.cuda.device(self.device):
                lib.selfjoin_free_grid(self.ptr, _stream_ptr(stream))
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TorchAllocHook:
    """sj_opts.alloc / free served by torch's caching allocator on one device
    (the library then allocates nothing itself for the handle). Keep the
    object alive as long as the handle: GridHandle holds it."""

    def __init__(self, device):
        torch = _torch()
        self.device = torch.device(device).index or 0

        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:
                return None

        def _free(ptr, stream, ctx):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = _lib.ALLOC_FN(_alloc)
        self.free = _lib.FREE_FN(_free)


def selfjoin_build_grid(points, eps: float, index_dims: int = 0, stream=None, torch_alloc: bool = False,
                        short_circuit: int = 0, dim_order: int = 0, symmetric: int = 0) -> GridHandle:
    """points: CUDA float64 tensor (n, d), C-contiguous. torch_alloc: every
    device buffer of the handle comes from torch's caching allocator through
    the sj_opts allocator hook. short_circuit, dim_order, symmetric: sj_opts
    fields of the same names (the result does not depend on them)."""
    torch = _torch()
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise ValueError("points must be a CUDA tensor")
    if points.dtype != torch.float64 or points.dim() != 2:
        raise ValueError("points must be float64 of shape (n, d)")
    points = points.contiguous()
    lib = _lib.load()
    opts = _lib.sj_opts()
    opts.index_dims = index_dims
    opts.short_circuit = short_circuit
    opts.dim_order = dim_order
    opts.symmetric = symmetric
    hook = TorchAllocHook(points.device) if torch_alloc else None
    if hook is not None:
        opts.alloc = hook.alloc
        opts.free = hook.free
    out = ctypes.c_void_p()
    n, d = points.shape
    with torch.cuda.device(points.device):
        st = lib.selfjoin_build_grid(ctypes.c_void_p(points.data_ptr()), n, d, float(eps),
                                     ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(out))
    check(st, "selfjoin_build_grid")
    h = GridHandle(out, n, d, float(eps), points.device)
    h.hook = hook
    return h


def selfjoin_count(g: GridHandle, path="fp64_mfma", per_point: bool = False, stream=None):
    """Returns (total, per_point int32 tensor or None, stats dict)."""
    torch = _torch()
    lib = _lib.load()
    pp = torch.empty(g.n, dtype=torch.int32, device=g.device) if per_point else None
    total = ctypes.c_int64(0)
    stats = _lib.sj_stats()
    with torch.cuda.device(g.device):
        st = lib.selfjoin_count(g.ptr, _path_id(path),
                                ctypes.c_void_p(pp.data_ptr()) if pp is not None and g.n else None,
                                ctypes.byref(total), ctypes.byref(stats), _stream_ptr(stream))
    check(st, "selfjoin_count")
    return total.value, pp, stats.as_dict()


def selfjoin_count_noalloc(points, eps: float, path="fp64_mfma", per_point: bool = False, stream=None):
    """Build + count in one call with every temporary in the library's static
    device scratch (nothing allocated by the library; `per_point`, if asked,
    is allocated here by torch). Returns (total, per_point int32 tensor or
    None)."""
    torch = _torch()
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise ValueError("points must be a CUDA tensor")
    if points.dtype != torch.float64 or points.dim() != 2:
        raise ValueError("points must be float64 of shape (n, d)")
    points = points.contiguous()
    lib = _lib.load()
    n, d = points.shape
    pp = torch.empty(n, dtype=torch.int32, device=points.device) if per_point else None
    total = ctypes.c_int64(0)
    with torch.cuda.device(points.device):
        st = lib.selfjoin_count_noalloc(ctypes.c_void_p(points.data_ptr()), n, d, float(eps), _path_id(path),
                                        ctypes.c_void_p(pp.data_ptr()) if pp is not None and n else None,
                                        ctypes.byref(total), _stream_ptr(stream))
    check(st, "selfjoin_count_noalloc")
    return total.value, pp


def selfjoin_core_points(g: GridHandle, min_pts: int, path="fp64_mfma", stream=None):
    """DBSCAN core points: returns (uint8 CUDA tensor, 1 = core, input order;
    number of core points). Reuses the handle's counts or counts with `path`."""
    torch = _torch()
    lib = _lib.load()
    flags = torch.empty(g.n, dtype=torch.uint8, device=g.device)
    ncore = ctypes.c_int64(0)
    with torch.cuda.device(g.device):
        st = lib.selfjoin_core_points(g.ptr, _path_id(path), int(min_pts),
                                      ctypes.c_void_p(flags.data_ptr()) if g.n else None, ctypes.byref(ncore),
                                      _stream_ptr(stream))
    check(st, "selfjoin_core_points")
    return flags, ncore.value


def selfjoin_knn(g: GridHandle, k: int, path="fp64_mfma", want_d2=True, pair_budget=0, stream=None):
    """k nearest neighbours within eps (self excluded, by distance then
    index): returns (nbr int32 [n, k], d2 float64 [n, k] or None, nfound
    int32 [n]) as CUDA tensors in the input order."""
    torch = _torch()
    lib = _lib.load()
    nbr = torch.empty((g.n, int(k)), dtype=torch.int32, device=g.device)
    d2 = torch.empty((g.n, int(k)), dtype=torch.float64, device=g.device) if want_d2 else None
    nfound = torch.empty(g.n, dtype=torch.int32, device=g.device)
    vp = lambda t: ctypes.c_void_p(t.data_ptr()) if (t is not None and g.n) else None
    with torch.cuda.device(g.device):
        st = lib.selfjoin_knn(g.ptr, _path_id(path), int(k), int(pair_budget), vp(nbr), vp(d2), vp(nfound),
                              _stream_ptr(stream))
    check(st, "selfjoin_knn")
    return nbr, d2, nfound


def selfjoin_pairs(g: GridHandle, path, cursor: int, pairs, d2=None, capacity=None, stream=None):
    """Writes one chunk into `pairs` (int32 CUDA tensor (capacity, 2)) and
    optionally `d2` (float64 CUDA tensor (capacity,)). Returns
    (written, next_cursor, stats dict). Raises SelfJoinError with status
    SJ_ERR_CAPACITY (attribute `needed`) when the next query does not fit."""
    torch = _torch()
    lib = _lib.load()
    if capacity is None:
        capacity = pairs.shape[0]
    if pairs.dtype != torch.int32 or pairs.dim() != 2 or pairs.shape[1] != 2 or pairs.shape[0] < capacity:
        raise ValueError("pairs must be int32 of shape (>= capacity, 2)")
    if d2 is not None and (d2.dtype != torch.float64 or d2.shape[0] < capacity):
        raise ValueError("d2 must be float64 of length >= capacity")
    written = ctypes.c_int64(0)
    nxt = ctypes.c_int64(0)
    stats = _lib.sj_stats()
    with torch.cuda.device(g.device):
        st = lib.selfjoin_pairs(g.ptr, _path_id(path), int(cursor),
                                ctypes.c_void_p(pairs.data_ptr()),
                                ctypes.c_void_p(d2.data_ptr()) if d2 is not None else None,
                                int(capacity), ctypes.byref(written), ctypes.byref(nxt),
                                ctypes.byref(stats), _stream_ptr(stream))
    if st == _lib.SJ_ERR_CAPACITY:
        err = SelfJoinError(st, "selfjoin_pairs")
        err.needed = written.value
        raise err
    check(st, "selfjoin_pairs")
    return written.value, nxt.value, stats.as_dict()


def selfjoin_measure_error(g: GridHandle, path, stream=None):
    """Returns (max |fast - exact|, band half-width, violations)."""
    torch = _torch()
    lib = _lib.load()
    e = ctypes.c_double(0)
    b = ctypes.c_double(0)
    v = ctypes.c_int64(0)
    with torch.cuda.device(g.device):
        st = lib.selfjoin_measure_error(g.ptr, _path_id(path), ctypes.byref(e), ctypes.byref(b),
                                        ctypes.byref(v), _stream_ptr(stream))
    check(st, "selfjoin_measure_error")
    return e.value, b.value, v.value


def selfjoin_grid_info(g: GridHandle, stream=None) -> dict:
    """Grid facts; the first call computes C_ref (a pass over the cells)."""
    torch = _torch()
    lib = _lib.load()
    info = _lib.sj_grid_info()
    with torch.cuda.device(g.device):
        st = lib.selfjoin_grid_info(g.ptr, ctypes.byref(info), _stream_ptr(stream))
    check(st, "selfjoin_grid_info")
    return info.as_dict()


def selfjoin_probe_peaks(bytes_: int = 1 << 30, device: int = 0, stream=None) -> dict:
    """Achievable peaks of the GPU (matrix forms, FP64 vector FMA, HBM read
    and copy), measured by the library's microbenchmarks."""
    torch = _torch()
    lib = _lib.load()
    out = _lib.sj_peaks()
    with torch.cuda.device(device):
        st = lib.selfjoin_probe_peaks(int(bytes_), ctypes.byref(out), _stream_ptr(stream))
    check(st, "selfjoin_probe_peaks")
    return out.as_dict()


def selfjoin_free_grid(g: GridHandle, stream=None):
    g.close(stream)


class SelfJoin:
    """Convenience wrapper: grid + count + all pairs."""

    def __init__(self, points, eps, index_dims=0, stream=None, torch_alloc=False, short_circuit=0, dim_order=0,
                 symmetric=0):
        self.grid = selfjoin_build_grid(points, eps, index_dims, stream, torch_alloc=torch_alloc,
                                        short_circuit=short_circuit, dim_order=dim_order, symmetric=symmetric)
        self.stream = stream

    def count(self, path="fp64_mfma", per_point=False):
        return selfjoin_count(self.grid, path, per_point, self.stream)

    def core_points(self, min_pts, path="fp64_mfma"):
        return selfjoin_core_points(self.grid, min_pts, path, self.stream)

    def knn(self, k, path="fp64_mfma", want_d2=True, pair_budget=0):
        return selfjoin_knn(self.grid, k, path, want_d2, pair_budget, self.stream)

    def all_pairs(self, path="fp64_mfma", want_d2=False, capacity=None):
        """All pairs as one (|R|, 2) int32 tensor (and d2), chunked if
        `capacity` is given."""
        torch = _torch()
        total, _, _ = self.count(path)
        cap = total if capacity is None else capacity
        dev = self.grid.device
        out = torch.empty((max(total, 1), 2), dtype=torch.int32, device=dev)
        dd = torch.empty(max(total, 1), dtype=torch.float64, device=dev) if want_d2 else None
        buf = out if capacity is None else torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
        dbuf = dd if (capacity is None or not want_d2) else torch.empty(max(cap, 1), dtype=torch.float64,
                                                                         device=dev)
        cursor, pos = 0, 0
        while cursor < self.grid.n:
            w, cursor, _ = selfjoin_pairs(self.grid, path, cursor, buf, dbuf, cap, self.stream)
            if capacity is not None:
                out[pos:pos + w] = buf[:w]
                if want_d2:
                    dd[pos:pos + w] = dbuf[:w]
            pos += w
        if capacity is None and pos != total:
            raise RuntimeError("pair count mismatch")
        res = out[:total]
        return (res, dd[:total]) if want_d2 else res

    def close(self):
        self.grid.close(self.stream)


# ------------------------------------------------------------- batched form --

class BatchHandle:
    """Owns a sj_batch*; the input tensors are kept alive with it."""

    def __init__(self, ptr, ns, device, keep):
        self.ptr = ptr
        self.ns = list(ns)
        self.device = device
        self._keep = keep

    def close(self, stream=None):
        if self.ptr:
            lib = _lib.load()
            torch = _torch()
            with torch.cuda.device(self.device):
                lib.selfjoin_batch_free(self.ptr, _stream_ptr(stream))
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def selfjoin_batch_build(points_list, eps_list, index_dims: int = 0, tune: bool = False, tune_cache=None,
                         stream=None, short_circuit: int = 0, dim_order: int = 0,
                         symmetric: int = 0) -> BatchHandle:
    """points_list: list of CUDA float64 (n_i, d_i) tensors; eps_list: floats.
    index_dims / short_circuit / dim_order: sj_opts fields (ignored for the
    choices the tuner makes when tune is set); symmetric: the half-stencil
    count for every problem (no in-masks: the pairs launch re-runs the
    tiles)."""
    torch = _torch()
    pts = [p.contiguous() for p in points_list]
    B = len(pts)
    if len(eps_list) != B:
        raise ValueError("one eps per problem")
    for p in pts:
        if not p.is_cuda or p.dtype != torch.float64 or p.dim() != 2:
            raise ValueError("every problem must be a CUDA float64 (n, d) tensor")
    lib = _lib.load()
    ptrs = (ctypes.c_void_p * max(B, 1))(*[p.data_ptr() for p in pts])
    ns = (ctypes.c_int64 * max(B, 1))(*[p.shape[0] for p in pts])
    ds = (ctypes.c_int32 * max(B, 1))(*[p.shape[1] for p in pts])
    es = (ctypes.c_double * max(B, 1))(*[float(e) for e in eps_list])
    opts = _lib.sj_opts()
    opts.index_dims = index_dims
    opts.short_circuit = short_circuit
    opts.dim_order = dim_order
    opts.symmetric = symmetric
    opts.tune = 1 if tune else 0
    opts.tune_cache = tune_cache.encode() if tune_cache else None
    out = ctypes.c_void_p()
    dev = pts[0].device if B else torch.device("cuda:0")
    with torch.cuda.device(dev):
        st = lib.selfjoin_batch_build(B, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), ns, ds, es,
                                      ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(out))
    check(st, "selfjoin_batch_build")
    return BatchHandle(out, [p.shape[0] for p in pts], dev, pts)


def selfjoin_batch_count(b: BatchHandle, path="fp64_mfma", stream=None):
    """Returns (list of |R| per problem, stats dict)."""
    torch = _torch()
    lib = _lib.load()
    B = len(b.ns)
    totals = (ctypes.c_int64 * max(B, 1))()
    stats = _lib.sj_stats()
    with torch.cuda.device(b.device):
        st = lib.selfjoin_batch_count(b.ptr, _path_id(path), totals, ctypes.byref(stats), _stream_ptr(stream))
    check(st, "selfjoin_batch_count")
    return [totals[i] for i in range(B)], stats.as_dict()


def selfjoin_batch_pairs(b: BatchHandle, path, pairs, stream=None):
    """Writes all problems' pairs into `pairs` (int32 CUDA (capacity, 2)).
    Returns (offsets list of B + 1, stats dict)."""
    torch = _torch()
    lib = _lib.load()
    B = len(b.ns)
    offs = (ctypes.c_int64 * (B + 1))()
    stats = _lib.sj_stats()
    with torch.cuda.device(b.device):
        st = lib.selfjoin_batch_pairs(b.ptr, _path_id(path), ctypes.c_void_p(pairs.data_ptr()),
                                      int(pairs.shape[0]), offs, ctypes.byref(stats), _stream_ptr(stream))
    if st == _lib.SJ_ERR_CAPACITY:
        err = SelfJoinError(st, "selfjoin_batch_pairs")
        err.needed = offs[B]
        raise err
    check(st, "selfjoin_batch_pairs")
    return [offs[i] for i in range(B + 1)], stats.as_dict()


def selfjoin_batch_info(b: BatchHandle, i: int):
    lib = _lib.load()
    k = ctypes.c_int32(0)
    items = ctypes.c_int64(0)
    check(lib.selfjoin_batch_info(b.ptr, i, ctypes.byref(k), ctypes.byref(items)), "selfjoin_batch_info")
    return {"index_dims": k.value, "items": items.value}


def selfjoin_batch_free(b: BatchHandle, stream=None):
    b.close(stream)

"""MI355X-native epsilon-distance similarity self-join (gfx950 HIP kernels
behind the C ABI of include/selfjoin.h)."""
from ._lib import PATHS, SelfJoinError, load
from .selfjoin import (SelfJoin, selfjoin_batch_build, selfjoin_batch_count, selfjoin_batch_free,
                       selfjoin_batch_info, selfjoin_batch_pairs, selfjoin_build_grid, selfjoin_core_points, selfjoin_knn,
                       selfjoin_count, selfjoin_count_noalloc, selfjoin_free_grid, selfjoin_grid_info, selfjoin_measure_error,
                       selfjoin_pairs, selfjoin_probe_peaks)

__all__ = [
    "PATHS", "SelfJoinError", "load", "SelfJoin", "selfjoin_build_grid", "selfjoin_count", "selfjoin_core_points", "selfjoin_knn",
    "selfjoin_pairs", "selfjoin_measure_error", "selfjoin_grid_info", "selfjoin_free_grid",
    "selfjoin_batch_build", "selfjoin_batch_count", "selfjoin_batch_pairs", "selfjoin_batch_info",
    "selfjoin_batch_free", "selfjoin_count_noalloc", "selfjoin_probe_peaks",
]

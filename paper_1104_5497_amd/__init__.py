"""NPHC on MI355X: all stationary points of the power-law XY ring by total-degree
homotopy continuation, with the hot path in hand-written HIP kernels
(libnphc.so, C ABI in include/nphc.h)."""

__all__ = ["build", "pipeline", "find_all_sps"]


def find_all_sps(*args, **kwargs):
    from .pipeline import find_all_sps as f
    return f(*args, **kwargs)

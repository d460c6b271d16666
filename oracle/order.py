"""Ranking order of keys (oracle; test infrastructure only).

The paper evaluates unsigned 32-bit integers (Section 6) and states the
problem for "largest" (Section 1).  For float32 it is silent; this project's
reading is IEEE 754 totalOrder (negative NaNs lowest, then -inf ... -0, +0
... +inf, then positive NaNs), so every bit pattern has a place and -0 sorts
below +0.  Signed 32-bit integers take their ordinary order.

``rank_key`` maps values to int64 numbers whose ordinary integer order is the
ranking order.  For float32 it works on the signed 32-bit view of the bits:
non-negative patterns keep their value; a pattern with the sign bit set and
magnitude bits m maps to -1 - m, so a larger magnitude ranks lower and -0
(m = 0) lands just below +0.  This is deliberately a different formula from
the one the GPU library uses.
"""
from __future__ import annotations

import numpy as np

INVALID_INDEX = 0xFFFFFFFF


def rank_key(values: np.ndarray, dtype: str) -> np.ndarray:
    """int64 array whose natural order is the ranking order of ``values``."""
    v = np.asarray(values)
    if dtype == "u32":
        if v.dtype != np.uint32:
            raise TypeError(f"u32 keys must be a uint32 array, got {v.dtype}")
        return v.astype(np.int64)
    if dtype == "f32":
        if v.dtype != np.float32:
            raise TypeError(f"f32 keys must be a float32 array, got {v.dtype}")
        s = v.view(np.int32).astype(np.int64)
        mag = s & 0x7FFFFFFF
        return np.where(s >= 0, s, -1 - mag)
    if dtype == "i32":
        if v.dtype != np.int32:
            raise TypeError(f"i32 keys must be an int32 array, got {v.dtype}")
        return v.astype(np.int64)
    raise ValueError(f"unknown dtype {dtype!r}")


def bits(values: np.ndarray) -> np.ndarray:
    """Raw 32-bit patterns (for bitwise comparisons of outputs)."""
    v = np.asarray(values)
    return v.view(np.uint32)

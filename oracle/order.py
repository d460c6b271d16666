"""Ranking order of keys (oracle; test infrastructure only).

The paper evaluates unsigned 32-bit integers (Section 6) and states the
problem for "largest" (Section 1).  For floats it is silent; this project's
reading is IEEE 754 totalOrder (negative NaNs lowest, then -inf ... -0, +0
... +inf, then positive NaNs), so every bit pattern has a place and -0 sorts
below +0.  Signed integers take their ordinary order.  The paper's selections
run on key-value pairs (Section 5.1); 64-bit keys (uint64, int64, float64)
take the same definitions at twice the width.

``rank_key`` maps values to int64 numbers whose ordinary integer order is the
ranking order.  For floats it works on the signed view of the bits (int32 or
int64): non-negative patterns keep their value; a pattern with the sign bit
set and magnitude bits m maps to -1 - m, so a larger magnitude ranks lower
and -0 (m = 0) lands just below +0.  uint64 does not fit int64, so it is
shifted down by 2^63 (wrapping subtraction), which keeps its order.  These are
deliberately different formulas from the ones the GPU library uses.
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
    if dtype == "u64":
        if v.dtype != np.uint64:
            raise TypeError(f"u64 keys must be a uint64 array, got {v.dtype}")
        return (v - np.uint64(1 << 63)).view(np.int64)
    if dtype == "i64":
        if v.dtype != np.int64:
            raise TypeError(f"i64 keys must be an int64 array, got {v.dtype}")
        return v.copy()
    if dtype == "f64":
        if v.dtype != np.float64:
            raise TypeError(f"f64 keys must be a float64 array, got {v.dtype}")
        s = v.view(np.int64)
        mag = s & np.int64(0x7FFFFFFFFFFFFFFF)
        return np.where(s >= 0, s, np.int64(-1) - mag)
    raise ValueError(f"unknown dtype {dtype!r}")


WIDE = ("u64", "i64", "f64")  # 8-byte key types


def bits(values: np.ndarray) -> np.ndarray:
    """Raw bit patterns (uint32 or uint64 by element size) for bitwise comparisons."""
    v = np.asarray(values)
    return v.view(np.uint64 if v.dtype.itemsize == 8 else np.uint32)

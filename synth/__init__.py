"""Seeded synthetic inputs for the delegate-centric top-k tests and benchmarks.

This module only draws numbers.  It holds none of the selection arithmetic:
no ordering, no key encoding, no top-k.  Tests, ``bench.py`` and the oracle
checks all take their arrays from here, so the GPU path and the oracle always
see the same bytes.

Distributions follow the paper's evaluation setup (Section 6): the uniform
dataset is i.i.d. U[0, 2^32 - 1] over unsigned 32-bit keys.  The float32
standard-normal, ascending-sorted and heavy-duplicate variants are the
synthetic stand-ins this project uses for the paper's normal / customised /
real-world datasets, which are not available here.

Generator: a counter-based stream built on the SplitMix64 output function
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014).  Element i of a stream with seed s is
``mix64(base(s) + (i + 1) * 0x9E3779B97F4A7C15)`` where ``base(s) = mix64(s)``,
so any slice can be produced independently and in parallel.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
DEFAULT_SEED = 210908219

def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _base(seed: int) -> np.uint64:
    return mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]


def u64_stream(seed: int, start: int, count: int) -> np.ndarray:
    """Elements [start, start+count) of the uint64 stream for ``seed``."""
    b = _base(seed)
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(b + i * GOLDEN_GAMMA)


_LIB = None


def _lib():
    """The OpenMP generator library (built with gcc on first use if absent)."""
    global _LIB
    if _LIB is None:
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "libsynth.so")
        src = os.path.join(here, "csrc", "synth.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            build()
        lib = ctypes.CDLL(so)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.synth_u64.argtypes = [u64, u64, u64, p]
        lib.synth_uniform_u32.argtypes = [u64, u64, p]
        lib.synth_mod_u32.argtypes = [u64, u64, ctypes.c_uint32, p]
        lib.synth_normal_f32.argtypes = [u64, u64, p]
        lib.synth_normal_f64.argtypes = [u64, u64, p]
        lib.synth_mod_u64.argtypes = [u64, u64, u64, p]
        for f in (lib.synth_u64, lib.synth_uniform_u32, lib.synth_mod_u32, lib.synth_normal_f32,
                  lib.synth_normal_f64, lib.synth_mod_u64):
            f.restype = None
        _LIB = lib
    return _LIB


def build() -> None:
    """Compile the generator library in place (gcc, OpenMP)."""
    here = os.path.dirname(os.path.abspath(__file__))
    so = os.path.join(here, "libsynth.so")
    tmp = so + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                    os.path.join(here, "csrc", "synth.c"), "-lm"], check=True)
    os.replace(tmp, so)


def _seed64(seed: int) -> int:
    return seed & 0xFFFFFFFFFFFFFFFF


def uniform_u32(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """n i.i.d. uint32 uniform over [0, 2^32): the high 32 bits of the stream."""
    out = np.empty(n, dtype=np.uint32)
    _lib().synth_uniform_u32(_seed64(seed), n, out.ctypes.data)
    return out


def normal_f32(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """n float32 draws of N(0, 1) by Box-Muller in float64, rounded to float32.

    Element i uses stream elements 2i and 2i+1: u1 = (hi53(x_2i) + 1) / 2^53 in
    (0, 1], u2 = hi53(x_2i+1) / 2^53 in [0, 1); z = sqrt(-2 ln u1) cos(2 pi u2).
    """
    out = np.empty(n, dtype=np.float32)
    _lib().synth_normal_f32(_seed64(seed), n, out.ctypes.data)
    return out


def sorted_normal_f32(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """Globally ascending-sorted float32 N(0, 1) sample (adversarial for max delegates)."""
    x = normal_f32(n, seed)
    x.sort()
    return x


def heavy_dup_u32(n: int, seed: int = DEFAULT_SEED, distinct: int = 16) -> np.ndarray:
    """uint32 values uniform over [0, distinct): nearly every key is tied."""
    out = np.empty(n, dtype=np.uint32)
    _lib().synth_mod_u32(_seed64(seed), n, distinct, out.ctypes.data)
    return out


def uniform_u64(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """n i.i.d. uint64 uniform over [0, 2^64): the stream itself."""
    out = np.empty(n, dtype=np.uint64)
    _lib().synth_u64(_seed64(seed), 0, n, out.ctypes.data)
    return out


def normal_f64(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """n float64 draws of N(0, 1): normal_f32's Box-Muller draw, not rounded."""
    out = np.empty(n, dtype=np.float64)
    _lib().synth_normal_f64(_seed64(seed), n, out.ctypes.data)
    return out


def heavy_dup_u64(n: int, seed: int = DEFAULT_SEED, distinct: int = 16) -> np.ndarray:
    """uint64 values uniform over [0, distinct)."""
    out = np.empty(n, dtype=np.uint64)
    _lib().synth_mod_u64(_seed64(seed), n, distinct, out.ctypes.data)
    return out


# numpy restatements of the same streams, used to check the C library.
def ref_uniform_u64(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    return u64_stream(seed, 0, n)


def ref_normal_f64(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    x = u64_stream(seed, 0, 2 * n)
    a = (x[0::2] >> np.uint64(11)).astype(np.float64)
    b = (x[1::2] >> np.uint64(11)).astype(np.float64)
    u1 = (a + 1.0) * (1.0 / 9007199254740992.0)
    u2 = b * (1.0 / 9007199254740992.0)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)



def ref_uniform_u32(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    return (u64_stream(seed, 0, n) >> np.uint64(32)).astype(np.uint32)


def ref_heavy_dup_u32(n: int, seed: int = DEFAULT_SEED, distinct: int = 16) -> np.ndarray:
    return (u64_stream(seed, 0, n) % np.uint64(distinct)).astype(np.uint32)


def ref_normal_f32(n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    x = u64_stream(seed, 0, 2 * n)
    a = (x[0::2] >> np.uint64(11)).astype(np.float64)
    b = (x[1::2] >> np.uint64(11)).astype(np.float64)
    u1 = (a + 1.0) * (1.0 / 9007199254740992.0)
    u2 = b * (1.0 / 9007199254740992.0)
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)


def unit_uniform(n: int, seed: int) -> np.ndarray:
    """n float64 uniforms in [0, 1) with 53-bit resolution."""
    x = u64_stream(seed, 0, n)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def log_uniform_int(n: int, lo_exp: float, hi_exp: float, seed: int) -> np.ndarray:
    """round(2^(lo + (hi - lo) u)) for u uniform in [0, 1): log-uniform integers."""
    u = unit_uniform(n, seed)
    return np.rint(np.exp2(lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)


def derive_seed(base: int, i: int) -> int:
    """Per-instance seed: the SplitMix64 output of base + i."""
    return int(mix64(np.array([(base + i) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0])


def keys(kind: str, n: int, seed: int = DEFAULT_SEED) -> tuple[np.ndarray, str]:
    """Named workloads -> (array, dtype tag 'u32', 'f32', 'i32', 'u64', 'i64' or 'f64').

    uniform_i32 is the uniform uint32 stream read as int32 (uniform over the
    whole signed range); smallrange_i32 maps it onto [-1000, 1000] (ties and
    negatives everywhere); revsorted_f32 is the sorted normal sample in
    descending order (the adversarial layout for the k smallest)."""
    if kind == "uniform_u32":
        return uniform_u32(n, seed), "u32"
    if kind == "normal_f32":
        return normal_f32(n, seed), "f32"
    if kind == "sorted_f32":
        return sorted_normal_f32(n, seed), "f32"
    if kind == "revsorted_f32":
        return sorted_normal_f32(n, seed)[::-1].copy(), "f32"
    if kind == "heavydup_u32":
        return heavy_dup_u32(n, seed), "u32"
    if kind == "uniform_i32":
        return uniform_u32(n, seed).view(np.int32), "i32"
    if kind == "smallrange_i32":
        return (heavy_dup_u32(n, seed, 2001).astype(np.int64) - 1000).astype(np.int32), "i32"
    if kind == "uniform_u64":
        return uniform_u64(n, seed), "u64"
    if kind == "uniform_i64":
        return uniform_u64(n, seed).view(np.int64), "i64"
    if kind == "normal_f64":
        return normal_f64(n, seed), "f64"
    if kind == "sorted_f64":
        x = normal_f64(n, seed)
        x.sort()
        return x, "f64"
    if kind == "heavydup_u64":
        return heavy_dup_u64(n, seed), "u64"
    if kind == "smallrange_i64":
        return heavy_dup_u64(n, seed, 2001).astype(np.int64) - 1000, "i64"
    if kind == "highword_u64":
        # keys whose high 32 bits take only 16 values: order is decided by the low word
        return (heavy_dup_u64(n, seed, 16) << np.uint64(32)) | (uniform_u64(n, seed + 1) >> np.uint64(32)), "u64"
    raise ValueError(f"unknown workload kind {kind!r}")


def batched_workload(count: int, seed: int = DEFAULT_SEED, lo_exp: int = 10, hi_exp: int = 20,
                     k_cap: int = 2048) -> list[tuple[str, int, int, int]]:
    """Independent instances for the batched form: (kind, n, k, seed) each.

    Lengths are log-uniform in [2^lo_exp, 2^hi_exp]; each instance is uint32
    uniform or float32 standard normal (a fair coin from its own seed); k is
    uniform in [1, min(n, k_cap)]."""
    ns = log_uniform_int(count, lo_exp, hi_exp, derive_seed(seed, 1))
    coin = unit_uniform(count, derive_seed(seed, 2))
    ku = unit_uniform(count, derive_seed(seed, 3))
    out = []
    for i in range(count):
        n = int(ns[i])
        kind = "uniform_u32" if coin[i] < 0.5 else "normal_f32"
        k = 1 + int(ku[i] * min(n, k_cap))
        out.append((kind, n, k, derive_seed(seed, 1000 + i)))
    return out


def serving_workload(count: int, seed: int = DEFAULT_SEED, lo_exp: int = 12, hi_exp: int = 26,
                     k_hi_exp: int = 12) -> list[tuple[str, int, int]]:
    """Requests of the serving workload: (kind, n, k) each.  n is log-uniform in
    [2^lo_exp, 2^hi_exp]; the keys are uint32 uniform or float32 standard normal
    (a fair coin); k is log-uniform in [1, 2^k_hi_exp], capped at n."""
    ns = log_uniform_int(count, lo_exp, hi_exp, derive_seed(seed, 11))
    coin = unit_uniform(count, derive_seed(seed, 12))
    ks = log_uniform_int(count, 0, k_hi_exp, derive_seed(seed, 13))
    return [("uniform_u32" if coin[i] < 0.5 else "normal_f32", int(ns[i]), int(min(ks[i], ns[i])))
            for i in range(count)]


def poisson_arrivals(count: int, rate_per_s: float, seed: int = DEFAULT_SEED) -> np.ndarray:
    """Arrival times in microseconds of a Poisson process: cumulative sums of
    exponential gaps -ln(1 - u) / rate."""
    u = unit_uniform(count, derive_seed(seed, 21))
    gaps = -np.log1p(-u) / rate_per_s * 1e6
    return np.cumsum(gaps)

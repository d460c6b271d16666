"""Python binding of libdrtopk (delegate-centric top-k on MI355X).

Argument marshalling only: tensors are passed to the C-ABI as raw device
pointers with the current HIP stream; every step of the computation runs in
the library's HIP kernels.  There is no fallback: if the library is missing or
fails to load, every call raises.

    vals, idx = topk_select(keys, k)      # keys: torch uint32 or float32 on the GPU
    kth = kth_select(keys, k)
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdrtopk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "drtopk.h")

U32, F32 = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "device error", 4: "unsupported"}


class DrTopkError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("beta", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("subranges", ctypes.c_uint64), ("delegates", ctypes.c_uint64),
                ("scanned", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("t_key_bits", ctypes.c_uint32), ("t_idx", ctypes.c_uint32),
                ("step_ns", ctypes.c_uint32 * 20), ("err_flags", ctypes.c_uint32)]


class Problem(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("n", ctypes.c_uint64), ("k", ctypes.c_uint32),
                ("dtype", ctypes.c_uint32), ("out_vals", ctypes.c_void_p), ("out_idx", ctypes.c_void_p),
                ("out_kth", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded C library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python -m paper_2109_08219_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        sig = {
            "topk_select": [vp, u64, u32, i32, vp, vp, vp],
            "kth_select": [vp, u64, u32, i32, vp, vp],
            "topk_select_batched": [ctypes.POINTER(Problem), u32, vp],
            "topk_select_ex": [vp, u64, u32, i32, vp, vp, ctypes.POINTER(Options), ctypes.POINTER(Stats), vp],
            "drtopk_delegates": [vp, u64, i32, i32, i32, vp, vp, vp],
            "drtopk_candidates": [vp, u64, u32, i32, i32, i32, i32, vp, u64, ctypes.POINTER(u64),
                                  vp, vp],
            "drtopk_plan": [u64, u32, i32, ctypes.POINTER(Options)],
            "drtopk_release_workspace": [],
            "drtopk_timing_enable": [i32],
            "drtopk_timing_read": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(u64)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.drtopk_status_string.argtypes = [ctypes.c_int]
        L.drtopk_status_string.restype = ctypes.c_char_p
        L.drtopk_version.argtypes = []
        L.drtopk_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions include/drtopk.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def _check(status: int, what: str) -> None:
    if status != 0:
        raise DrTopkError(status, what)


def _torch():
    import torch
    return torch


def _dtype_code(t, dtype):
    torch = _torch()
    if dtype is not None:
        return {"u32": U32, "f32": F32}[dtype]
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.uint32:
        return U32
    raise TypeError(f"keys must be torch.uint32 or torch.float32 (got {t.dtype}); "
                    "pass dtype='u32' to read other 4-byte data as uint32")


def _prep(keys, dtype):
    if not keys.is_cuda:
        raise ValueError("keys must be a GPU tensor")
    if keys.dim() != 1 or not keys.is_contiguous() or keys.element_size() != 4:
        raise ValueError("keys must be a contiguous 1-D tensor of 4-byte elements")
    return _dtype_code(keys, dtype)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _opts(alpha, beta, mode, variant=0):
    if alpha is None and beta is None and mode is None and not variant:
        return None
    return Options(-1 if alpha is None else alpha, 0 if beta is None else beta, 0 if mode is None else mode,
                   variant)


def topk_select(keys, k: int, out_vals=None, out_idx=None, *, dtype=None, alpha=None, beta=None,
                mode=None, variant: int = 0, stats: bool = False, stream=None):
    """The k largest keys, sorted descending (ties: lower position first), and their positions.

    Returns (values, indices[, Stats]).  values has the keys' dtype; indices are int64-free uint32
    positions stored in a torch.int32 tensor (bit pattern of the uint32 position)."""
    torch = _torch()
    code = _prep(keys, dtype)
    if out_vals is None:
        out_vals = torch.empty(k, dtype=keys.dtype, device=keys.device)
    if out_idx is None:
        out_idx = torch.empty(k, dtype=torch.int32, device=keys.device)
    opts = _opts(alpha, beta, mode, variant)
    st = Stats() if stats else None
    rc = lib().topk_select_ex(ctypes.c_void_p(keys.data_ptr()), keys.numel(), k, code,
                              ctypes.c_void_p(out_vals.data_ptr()), ctypes.c_void_p(out_idx.data_ptr()),
                              ctypes.byref(opts) if opts is not None else None,
                              ctypes.byref(st) if st is not None else None, _stream(stream))
    if rc != 0 and st is not None and st.err_flags:
        raise DrTopkError(rc, f"topk_select (device check flags {st.err_flags:#x})")
    _check(rc, "topk_select")
    return (out_vals, out_idx, st) if stats else (out_vals, out_idx)


def kth_select(keys, k: int, out=None, *, dtype=None, stream=None):
    """The k-th largest key (counting multiplicity) as a 1-element tensor."""
    torch = _torch()
    code = _prep(keys, dtype)
    if out is None:
        out = torch.empty(1, dtype=keys.dtype, device=keys.device)
    rc = lib().kth_select(ctypes.c_void_p(keys.data_ptr()), keys.numel(), k, code,
                          ctypes.c_void_p(out.data_ptr()), _stream(stream))
    _check(rc, "kth_select")
    return out


def topk_select_batched(problems, *, stream=None):
    """problems: list of (keys, k) or (keys, k, dtype).  Returns a list of (values, indices, kth)."""
    torch = _torch()
    descs = (Problem * max(1, len(problems)))()
    outs = []
    for i, pr in enumerate(problems):
        keys, k = pr[0], pr[1]
        code = _prep(keys, pr[2] if len(pr) > 2 else None)
        v = torch.empty(k, dtype=keys.dtype, device=keys.device)
        ix = torch.empty(k, dtype=torch.int32, device=keys.device)
        kth = torch.empty(1, dtype=keys.dtype, device=keys.device)
        descs[i] = Problem(keys.data_ptr(), keys.numel(), k, code, v.data_ptr(), ix.data_ptr(), kth.data_ptr())
        outs.append((v, ix, kth))
    rc = lib().topk_select_batched(descs, len(problems), _stream(stream))
    _check(rc, "topk_select_batched")
    return outs


def delegates(keys, alpha: int, beta: int, *, dtype=None, stream=None):
    """The delegate vector (values, positions) as (S, beta) tensors."""
    torch = _torch()
    code = _prep(keys, dtype)
    n = keys.numel()
    S = -(-n // (1 << alpha))
    dk = torch.empty(S * beta, dtype=keys.dtype, device=keys.device)
    di = torch.empty(S * beta, dtype=torch.int32, device=keys.device)
    rc = lib().drtopk_delegates(ctypes.c_void_p(keys.data_ptr()), n, code, alpha, beta,
                                ctypes.c_void_p(dk.data_ptr()), ctypes.c_void_p(di.data_ptr()), _stream(stream))
    _check(rc, "drtopk_delegates")
    return dk.view(S, beta), di.view(S, beta)


def candidates(keys, k: int, alpha: int, beta: int, *, variant: int = 0, dtype=None, stream=None):
    """Positions (unordered) of the survivors of the delegate filter, and the
    threshold (key bit pattern, position): survivors are exactly the elements
    ranked at or above it."""
    torch = _torch()
    code = _prep(keys, dtype)
    n = keys.numel()
    cap = n
    out = torch.empty(cap, dtype=torch.int32, device=keys.device)
    cnt = ctypes.c_uint64(0)
    tout = (ctypes.c_uint32 * 2)()
    rc = lib().drtopk_candidates(ctypes.c_void_p(keys.data_ptr()), n, k, code, alpha, beta, variant,
                                 ctypes.c_void_p(out.data_ptr()), cap, ctypes.byref(cnt), tout, _stream(stream))
    _check(rc, "drtopk_candidates")
    return out[: cnt.value], (tout[0], tout[1])


@dataclass
class Plan:
    mode: int
    alpha: int
    beta: int


def plan(n: int, k: int, dtype: str = "u32") -> Plan:
    o = Options()
    _check(lib().drtopk_plan(n, k, {"u32": U32, "f32": F32}[dtype], ctypes.byref(o)), "drtopk_plan")
    return Plan(o.mode, o.alpha, o.beta)


def release_workspace() -> None:
    _check(lib().drtopk_release_workspace(), "drtopk_release_workspace")


def timing_enable(on: bool = True) -> None:
    _check(lib().drtopk_timing_enable(1 if on else 0), "drtopk_timing_enable")


def timing_read():
    """(delegate-pass ms, rest-of-path ms, calls) summed since the last read."""
    d, t, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    _check(lib().drtopk_timing_read(ctypes.byref(d), ctypes.byref(t), ctypes.byref(c)), "drtopk_timing_read")
    return d.value, t.value, c.value


def status_string(code: int) -> str:
    return lib().drtopk_status_string(code).decode()


def version() -> str:
    return lib().drtopk_version().decode()

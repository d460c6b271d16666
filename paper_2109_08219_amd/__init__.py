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
TUNING_PATH = os.path.join(HERE, "tuning.json")  # written by paper_2109_08219_amd.tune

U32, F32, I32, U64, I64, F64 = 0, 1, 2, 3, 4, 5
SMALLEST = 0x100  # OR-ed into a dtype code: the k smallest instead of the k largest
_DTYPES = {"u32": U32, "f32": F32, "i32": I32, "u64": U64, "i64": I64, "f64": F64}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "device error", 4: "unsupported",
          5: "workspace exceeds the no-allocation scratch buffer"}


CHECK_FLAGS = {1: "select", 2: "few survivors", 16: "capacity", 64: "wait timeout", 128: "sort group"}


class DrTopkError(RuntimeError):
    def __init__(self, status: int, what: str, flags: int = 0):
        extra = ""
        if flags:
            names = ", ".join(v for b, v in CHECK_FLAGS.items() if flags & b)
            extra = f"; device check flags {flags:#x} ({names})"
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status}){extra}")
        self.status = status
        self.flags = flags


class Options(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("beta", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("subranges", ctypes.c_uint64), ("delegates", ctypes.c_uint64),
                ("scanned", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("t_key_bits", ctypes.c_uint32), ("t_idx", ctypes.c_uint32),
                ("step_ns", ctypes.c_uint32 * 20), ("err_flags", ctypes.c_uint32)]


class Tune(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("lg_n", ctypes.c_int32), ("lg_k", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("n", ctypes.c_uint64), ("k", ctypes.c_uint32),
                ("dtype", ctypes.c_uint32), ("out_vals", ctypes.c_void_p), ("out_idx", ctypes.c_void_p),
                ("out_kth", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_batch", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("plain", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64), ("launched_items", ctypes.c_uint64),
                ("max_inflight_bytes", ctypes.c_uint64), ("mean_us", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("max_us", ctypes.c_double)]


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
            "topk_select_noalloc": [vp, u64, u32, i32, vp, vp, vp],
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
            "drtopk_tune_set": [ctypes.POINTER(Tune), u32],
            "drtopk_tune_get": [ctypes.POINTER(Tune), u32, ctypes.POINTER(u32)],
            "drtopk_batched_alpha": [u64, u32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)],
            "drtopk_footprint": [u64, u32, i32, ctypes.POINTER(u64)],
            "drtopk_read_probe": [vp, u64, vp, vp],
            "topk_select_host": [vp, u64, u32, i32, u64, vp, vp, vp],
            "topk_select_payload": [vp, u64, u32, i32, vp, i32, vp, vp, vp, vp],
            "drtopk_server_create": [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)],
            "drtopk_server_submit": [vp, ctypes.POINTER(Problem), ctypes.POINTER(u64)],
            "drtopk_server_wait": [vp, u64, ctypes.POINTER(ctypes.c_double)],
            "drtopk_server_drain": [vp],
            "drtopk_server_stats": [vp, ctypes.POINTER(ServerStats), i32],
            "drtopk_server_replay": [vp, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_double), u32,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
            "drtopk_server_destroy": [vp],
            "drtopk_check": [vp, ctypes.POINTER(u32)],
            "drtopk_set_survivor_cap": [u64],
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
        if os.path.exists(TUNING_PATH):
            load_tuning(TUNING_PATH)
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
        return _DTYPES[dtype]
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.uint64:
        return U64
    if t.dtype == torch.int64:
        return I64
    if t.dtype == torch.uint32:
        return U32
    if t.dtype == torch.int32:
        return I32
    raise TypeError(f"keys must be torch.uint32, torch.int32 or torch.float32 (got {t.dtype}); "
                    "pass dtype='u32' to read other 4-byte data as uint32")


def _prep(keys, dtype, largest: bool = True):
    if not keys.is_cuda:
        raise ValueError("keys must be a GPU tensor")
    if keys.dim() != 1 or not keys.is_contiguous() or keys.element_size() not in (4, 8):
        raise ValueError("keys must be a contiguous 1-D tensor of 4- or 8-byte elements")
    return _dtype_code(keys, dtype) | (0 if largest else SMALLEST)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _opts(alpha, beta, mode, variant=0):
    if alpha is None and beta is None and mode is None and not variant:
        return None
    return Options(-1 if alpha is None else alpha, 0 if beta is None else beta, 0 if mode is None else mode,
                   variant)


def check_stream(stream=None) -> None:
    """Synchronises the stream and raises DrTopkError (with .flags) if a kernel of any call
    enqueued on it since the previous check failed an internal consistency check."""
    f = ctypes.c_uint32(0)
    rc = lib().drtopk_check(_stream(stream), ctypes.byref(f))
    if rc != 0:
        raise DrTopkError(rc, "drtopk_check", f.value)


check = check_stream


def set_survivor_cap(cap: int) -> None:
    """Testing hook: caps the delegate method's survivor buffers (0 = planner's bound)."""
    _check(lib().drtopk_set_survivor_cap(int(cap)), "drtopk_set_survivor_cap")


def topk_select(keys, k: int, out_vals=None, out_idx=None, *, dtype=None, largest: bool = True, alpha=None,
                beta=None, mode=None, variant: int = 0, stats: bool = False, check: bool = False, stream=None):
    """The k largest keys, sorted descending (ties: lower position first), and their positions;
    largest=False: the k smallest, sorted ascending (ties: lower position first).

    Returns (values, indices[, Stats]).  values has the keys' dtype; indices are int64-free uint32
    positions stored in a torch.int32 tensor (bit pattern of the uint32 position).  check=True
    synchronises the stream afterwards and raises if a device check failed (see check())."""
    torch = _torch()
    code = _prep(keys, dtype, largest)
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
        raise DrTopkError(rc, "topk_select", st.err_flags)
    _check(rc, "topk_select")
    if check:
        check_stream(stream)
    return (out_vals, out_idx, st) if stats else (out_vals, out_idx)


def topk_select_noalloc(keys, k: int, out_vals, out_idx=None, *, dtype=None, largest: bool = True,
                        stream=None) -> None:
    """topk_select into caller-provided outputs with the library's fixed device workspace: the
    call allocates nothing (no torch or HIP allocation).  out_idx may be None (positions not
    written).  Raises DrTopkError with status 5 if the problem needs more workspace than the
    fixed buffer holds.  Calls on one device share that buffer: do not overlap them."""
    code = _prep(keys, dtype, largest)
    rc = lib().topk_select_noalloc(ctypes.c_void_p(keys.data_ptr()), keys.numel(), k, code,
                                   ctypes.c_void_p(out_vals.data_ptr()),
                                   ctypes.c_void_p(out_idx.data_ptr()) if out_idx is not None else None,
                                   _stream(stream))
    _check(rc, "topk_select_noalloc")


def kth_select(keys, k: int, out=None, *, dtype=None, largest: bool = True, check: bool = False, stream=None):
    """The k-th largest key (largest=False: k-th smallest), counting multiplicity, as a 1-element tensor.
    check=True: synchronise and raise on a failed device check."""
    torch = _torch()
    code = _prep(keys, dtype, largest)
    if out is None:
        out = torch.empty(1, dtype=keys.dtype, device=keys.device)
    rc = lib().kth_select(ctypes.c_void_p(keys.data_ptr()), keys.numel(), k, code,
                          ctypes.c_void_p(out.data_ptr()), _stream(stream))
    _check(rc, "kth_select")
    if check:
        check_stream(stream)
    return out


class Batch:
    """A fixed set of top-k problems with packed device outputs, reusable across calls.

    problems: list of (keys, k), (keys, k, dtype) or (keys, k, dtype, largest) -- dtype None
    = from the tensor, largest False = the k smallest.  All outputs of problem i live in
    three packed int32 buffers: vals[voff[i] : voff[i] + w_i k_i] (bit patterns of the keys'
    dtype; w_i = 1 for 4-byte and 2 for 8-byte keys, whose offsets are even),
    idx[off[i] : off[i] + k_i] (uint32 positions) and kth[2i : 2i + w_i].  kth_only=True
    asks for the k-th values alone (no vals / idx buffers).  The descriptors are built
    once; run() enqueues one topk_select_batched call on `stream`.
    """

    def __init__(self, problems, *, kth_only: bool = False):
        torch = _torch()
        self.count = len(problems)
        self.keys = [pr[0] for pr in problems]
        self.ks = [int(pr[1]) for pr in problems]
        self.codes = [_prep(pr[0], pr[2] if len(pr) > 2 else None, pr[3] if len(pr) > 3 else True)
                      for pr in problems]
        self.words = [t.element_size() // 4 for t in self.keys]
        self.kth_only = kth_only
        dev = self.keys[0].device if self.keys else torch.device("cuda")
        self.off = [0] * self.count
        self.voff = [0] * self.count
        total = vtotal = 0
        for i, k in enumerate(self.ks):
            self.off[i] = total
            total += k
            vtotal += vtotal % self.words[i]  # 8-byte values start at an even word
            self.voff[i] = vtotal
            vtotal += k * self.words[i]
        self.total_k = total
        self.kth = torch.empty(max(2, 2 * self.count), dtype=torch.int32, device=dev)
        if kth_only:
            self.vals = self.idx = None
        else:
            self.vals = torch.empty(max(1, vtotal), dtype=torch.int32, device=dev)
            self.idx = torch.empty(max(1, total), dtype=torch.int32, device=dev)
        self._descs = (Problem * max(1, self.count))()
        vb = self.vals.data_ptr() if self.vals is not None else 0
        ib = self.idx.data_ptr() if self.idx is not None else 0
        kb = self.kth.data_ptr()
        for i in range(self.count):
            kt = self.keys[i]
            self._descs[i] = Problem(kt.data_ptr(), kt.numel(), self.ks[i], self.codes[i],
                                     vb + 4 * self.voff[i] if vb else None,
                                     ib + 4 * self.off[i] if ib else None, kb + 8 * i)

    def run(self, stream=None, check: bool = False) -> None:
        rc = lib().topk_select_batched(self._descs, self.count, _stream(stream))
        _check(rc, "topk_select_batched")
        if check:
            check_stream(stream)

    def _as_keys(self, t, i):
        return t.view(self.keys[i].dtype)

    def values(self, i: int):
        return self._as_keys(self.vals[self.voff[i]:self.voff[i] + self.words[i] * self.ks[i]], i)

    def indices(self, i: int):
        return self.idx[self.off[i]:self.off[i] + self.ks[i]]

    def kth_value(self, i: int):
        return self._as_keys(self.kth[2 * i:2 * i + self.words[i]], i)


def topk_select_batched(problems, *, check: bool = False, stream=None):
    """problems as for Batch.  Returns a list of (values, indices, kth)."""
    b = Batch(problems)
    b.run(stream, check)
    return [(b.values(i), b.indices(i), b.kth_value(i)) for i in range(b.count)]


def kth_select_batched(problems, *, check: bool = False, stream=None):
    """problems as for topk_select_batched.  Returns a list of 1-element k-th value tensors."""
    b = Batch(problems, kth_only=True)
    b.run(stream, check)
    return [b.kth_value(i) for i in range(b.count)]


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


def _dtype_arg(dtype) -> int:
    """'u32' / 'f32' / 'i32', optionally with a '-min' suffix (the k smallest), or a code."""
    if isinstance(dtype, int):
        return dtype
    base, _, order = dtype.partition("-")
    return _DTYPES[base] | (SMALLEST if order == "min" else 0)


def plan(n: int, k: int, dtype: str = "u32") -> Plan:
    o = Options()
    _check(lib().drtopk_plan(n, k, _dtype_arg(dtype), ctypes.byref(o)), "drtopk_plan")
    return Plan(o.mode, o.alpha, o.beta)


FORM_SINGLE, FORM_BATCHED = 0, 1


def tune_set(entries) -> None:
    """Replaces the autotuner table: entries of (form, lg_n, lg_k, alpha, beta)."""
    entries = list(entries)
    arr = (Tune * max(1, len(entries)))(*[Tune(*map(int, e)) for e in entries])
    _check(lib().drtopk_tune_set(arr, len(entries)), "drtopk_tune_set")


def tune_get() -> list[tuple[int, int, int, int, int]]:
    n = ctypes.c_uint32()
    _check(lib().drtopk_tune_get(None, 0, ctypes.byref(n)), "drtopk_tune_get")
    arr = (Tune * max(1, n.value))()
    _check(lib().drtopk_tune_get(arr, n.value, ctypes.byref(n)), "drtopk_tune_get")
    return [(e.form, e.lg_n, e.lg_k, e.alpha, e.beta) for e in arr[:n.value]]


def load_tuning(path: str = TUNING_PATH) -> int:
    """Loads a tuning table written by paper_2109_08219_amd.tune; returns its entry count."""
    import json
    with open(path) as f:
        doc = json.load(f)
    entries = [(e["form"], e["lg_n"], e["lg_k"], e["alpha"], e["beta"]) for e in doc["entries"]]
    tune_set(entries)
    return len(entries)


def batched_plan(n: int, k: int) -> tuple[int, int, int]:
    """(route, alpha, beta) of a batched problem: route 0 single-problem path, 1 sorted in the
    workgroup, 2 delegate method in the workgroup (alpha, beta delegates per subrange),
    3 workgroup radix select."""
    r, a, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().drtopk_batched_alpha(n, k, ctypes.byref(r), ctypes.byref(a), ctypes.byref(b)),
           "drtopk_batched_alpha")
    return r.value, a.value, b.value


def batched_route(n: int, k: int) -> tuple[int, int]:
    """(route, alpha) of a batched problem (batched_plan without beta)."""
    return batched_plan(n, k)[:2]


def footprint(n: int, k: int, dtype: str = "u32") -> int:
    """HBM bytes a problem occupies while in flight (input, outputs, workspace)."""
    b = ctypes.c_uint64()
    _check(lib().drtopk_footprint(n, k, _dtype_arg(dtype), ctypes.byref(b)), "drtopk_footprint")
    return b.value


class Server:
    """Continuous-batching server over device-resident arrays (see drtopk_server_* in the C header).

    Requests are (keys, k) pairs or a Batch of them; results land in the Batch's packed outputs."""

    def __init__(self, *, hbm_budget: int = 0, max_batch: int = 256, streams: int = 4, plain: bool = False):
        cfg = ServerConfig(hbm_budget, max_batch, streams, 1 if plain else 0, 0)
        h = ctypes.c_void_p()
        _check(lib().drtopk_server_create(ctypes.byref(cfg), ctypes.byref(h)), "drtopk_server_create")
        self._h = h

    def replay(self, batch: "Batch", arrival_us):
        """Submits batch problem i at arrival_us[i] (microseconds from now); returns
        (latencies_us list, elapsed_us)."""
        import numpy as np
        arr = np.ascontiguousarray(np.asarray(arrival_us, dtype=np.float64))
        if arr.shape[0] != batch.count:
            raise ValueError("one arrival time per problem")
        lat = np.zeros(max(1, batch.count), dtype=np.float64)
        el = ctypes.c_double()
        dp = ctypes.POINTER(ctypes.c_double)
        rc = lib().drtopk_server_replay(self._h, batch._descs, arr.ctypes.data_as(dp), batch.count,
                                        lat.ctypes.data_as(dp), ctypes.byref(el))
        _check(rc, "drtopk_server_replay")
        return lat[:batch.count], el.value

    def submit(self, batch: "Batch", i: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().drtopk_server_submit(self._h, ctypes.byref(batch._descs[i]), ctypes.byref(t)),
               "drtopk_server_submit")
        return t.value

    def wait(self, ticket: int) -> float:
        lat = ctypes.c_double()
        _check(lib().drtopk_server_wait(self._h, ticket, ctypes.byref(lat)), "drtopk_server_wait")
        return lat.value

    def drain(self) -> None:
        _check(lib().drtopk_server_drain(self._h), "drtopk_server_drain")

    def stats(self, reset: bool = False) -> ServerStats:
        st = ServerStats()
        _check(lib().drtopk_server_stats(self._h, ctypes.byref(st), 1 if reset else 0), "drtopk_server_stats")
        return st

    def close(self) -> None:
        if self._h:
            h, self._h = self._h, None
            _check(lib().drtopk_server_destroy(h), "drtopk_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def topk_select_payload(keys, payload, k: int, *, dtype=None, largest: bool = True, stream=None):
    """Top-k of keys (as topk_select) and the payload of each selected key:
    payload is a device tensor of n 4- or 8-byte elements.  Returns (values,
    indices, payloads)."""
    torch = _torch()
    code = _prep(keys, dtype, largest)
    if not payload.is_cuda or payload.dim() != 1 or not payload.is_contiguous() or payload.numel() != keys.numel():
        raise ValueError("payload must be a contiguous 1-D device tensor with one element per key")
    if payload.element_size() not in (4, 8):
        raise ValueError("payload elements must be 4 or 8 bytes")
    out_vals = torch.empty(k, dtype=keys.dtype, device=keys.device)
    out_idx = torch.empty(k, dtype=torch.int32, device=keys.device)
    out_pay = torch.empty(k, dtype=payload.dtype, device=keys.device)
    rc = lib().topk_select_payload(ctypes.c_void_p(keys.data_ptr()), keys.numel(), k, code,
                                   ctypes.c_void_p(payload.data_ptr()), payload.element_size(),
                                   ctypes.c_void_p(out_vals.data_ptr()), ctypes.c_void_p(out_idx.data_ptr()),
                                   ctypes.c_void_p(out_pay.data_ptr()), _stream(stream))
    _check(rc, "topk_select_payload")
    return out_vals, out_idx, out_pay


def topk_select_host(keys, k: int, *, chunk: int = 0, largest: bool = True, dtype=None, stream=None):
    """Top-k of a numpy array in host memory (uint32 / int32 / float32), streamed
    through the device in chunks of `chunk` keys (0 = library choice).  Returns
    (values, indices) as device tensors, like topk_select; synchronises `stream`."""
    import numpy as np
    torch = _torch()
    keys = np.ascontiguousarray(keys)
    if keys.ndim != 1 or keys.itemsize != 4:
        raise ValueError("keys must be a 1-D array of 4-byte elements")
    if dtype is None:
        dtype = {np.dtype(np.uint32): "u32", np.dtype(np.float32): "f32", np.dtype(np.int32): "i32"}.get(keys.dtype)
        if dtype is None:
            raise TypeError(f"keys must be uint32, int32 or float32 (got {keys.dtype})")
    code = _DTYPES[dtype] | (0 if largest else SMALLEST)
    tdt = {"u32": torch.uint32, "f32": torch.float32, "i32": torch.int32}[dtype]
    out_vals = torch.empty(k, dtype=tdt, device="cuda")
    out_idx = torch.empty(k, dtype=torch.int32, device="cuda")
    rc = lib().topk_select_host(ctypes.c_void_p(keys.ctypes.data), keys.shape[0], k, code, chunk,
                                ctypes.c_void_p(out_vals.data_ptr()), ctypes.c_void_p(out_idx.data_ptr()),
                                _stream(stream))
    _check(rc, "topk_select_host")
    return out_vals, out_idx


def read_probe(keys, out=None, *, stream=None):
    """Runs the read-bandwidth probe over keys (a 16-byte aligned device tensor of
    4-byte elements, at least 2^20 of them); returns the 1-element output tensor."""
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=keys.device)
    _check(lib().drtopk_read_probe(ctypes.c_void_p(keys.data_ptr()), keys.numel(), ctypes.c_void_p(out.data_ptr()),
                                   _stream(stream)), "drtopk_read_probe")
    return out


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

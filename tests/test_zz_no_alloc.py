"""topk_select_noalloc (fixed device workspace, no allocation) through the C
ABI: its outputs equal topk_select's bit for bit and the oracle's, on calls in
a row over one device's shared scratch buffer, each later call on a smaller
input than the one before (so stale contents of a larger call are present);
problems whose workspace exceeds the buffer are refused before any work."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from checks import check_exact, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _noalloc(t, k, code, vals, idx, stream):
    return drt.lib().topk_select_noalloc(ctypes.c_void_p(t.data_ptr()), t.numel(), k, code,
                                         ctypes.c_void_p(vals.data_ptr()),
                                         ctypes.c_void_p(idx.data_ptr()) if idx is not None else None,
                                         ctypes.c_void_p(stream.cuda_stream))


# (kind, n, k, largest): each smaller than the one before; the routes are the
# delegate method (device-wide tail), the plain radix select (k > n/16) and
# one workgroup (n <= 2^16)
CALLS = [("uniform_u32", (1 << 24) + 37, 1024, True),
         ("normal_f32", (1 << 22) + 5, 3000, False),
         ("uniform_u32", 200003, 20000, True),
         ("smallrange_i32", 40000, 777, True)]


def test_noalloc_equals_topk_select():
    stream = torch.cuda.current_stream()
    for i, (kind, n, k, largest) in enumerate(CALLS):
        say("noalloc call", i, kind, "n", n, "k", k, "largest", largest)
        x, dt = synth.keys(kind, n, 7100 + i)
        t = torch.from_numpy(x).cuda()
        code = drt._prep(t, None, largest)
        vals = torch.empty(k, dtype=t.dtype, device="cuda")
        idx = torch.empty(k, dtype=torch.int32, device="cuda")
        vals.fill_(0x5A5A5A5A if t.dtype != torch.float32 else 3.5)
        idx.fill_(-1)
        assert _noalloc(t, k, code, vals, idx, stream) == 0
        f = ctypes.c_uint32(0)
        assert drt.lib().drtopk_check(ctypes.c_void_p(stream.cuda_stream), ctypes.byref(f)) == 0, f.value
        wv, wi = drt.topk_select(t, k, largest=largest)
        torch.cuda.synchronize()
        assert (to_np(vals).view(np.uint32) == to_np(wv).view(np.uint32)).all(), (kind, n, k)
        assert (to_np(idx) == to_np(wi)).all(), (kind, n, k)
        check_exact(x, k, dt, to_np(vals), to_np(idx), f"noalloc {kind} n={n} k={k}", largest=largest)


def test_noalloc_without_positions_and_repeat():
    stream = torch.cuda.current_stream()
    x, dt = synth.keys("normal_f32", (1 << 21) + 3, 7200)
    t = torch.from_numpy(x).cuda()
    k = 5000
    vals = torch.empty(k, dtype=t.dtype, device="cuda")
    for rep in range(2):
        say("noalloc without positions, repeat", rep)
        assert _noalloc(t, k, drt.F32, vals, None, stream) == 0
        torch.cuda.synchronize()
        want, _ = drt.topk_select(t, k)
        torch.cuda.synchronize()
        assert (to_np(vals).view(np.uint32) == to_np(want).view(np.uint32)).all()


def test_noalloc_refuses_oversized_workspace():
    t = torch.zeros(16, dtype=torch.int32, device="cuda")
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    # n = 2^30, k = 131072 needs far more than the fixed buffer: refused before
    # the keys are touched (the pointer only has to be non-null)
    rc = drt.lib().topk_select_noalloc(ctypes.c_void_p(t.data_ptr()), 1 << 30, 131072, drt.U32,
                                       ctypes.c_void_p(out.data_ptr()), None, None)
    assert rc == 5
    assert drt.lib().drtopk_status_string(5).decode().startswith("workspace exceeds")

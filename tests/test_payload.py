"""Top-k of keys with a payload per key: the payloads of the selected keys,
for 4- and 8-byte payloads, with and without a position output, both orders;
values and positions equal topk_select's bit for bit and match the oracle."""
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


@pytest.mark.parametrize("kind,largest", [("uniform_u32", True), ("normal_f32", False), ("smallrange_i32", True)])
def test_payload_follows_the_keys(kind, largest):
    n = (1 << 20) + 11
    x, dt = synth.keys(kind, n, 4040)
    t = torch.from_numpy(x).cuda()
    p4 = torch.arange(n, dtype=torch.int32, device="cuda") * 3 + 7
    p8 = torch.arange(n, dtype=torch.int64, device="cuda") * 11 - (1 << 40)
    for k in (1, 500, 9000):
        for pay in (p4, p8):
            say(kind, "k", k, "payload bytes", pay.element_size())
            v, ix, out = drt.topk_select_payload(t, pay, k, largest=largest)
            wv, wi = drt.topk_select(t, k, largest=largest)
            torch.cuda.synchronize()
            assert (to_np(v).view(np.uint32) == to_np(wv).view(np.uint32)).all()
            assert (to_np(ix) == to_np(wi)).all()
            gi = to_np(ix).view(np.uint32).astype(np.int64)
            assert (to_np(out) == to_np(pay)[gi]).all()
            check_exact(x, k, dt, to_np(v), to_np(ix), f"{kind} k={k}", largest=largest)


def test_payload_without_position_output():
    x, dt = synth.keys("uniform_u32", 300007, 41)
    t = torch.from_numpy(x).cuda()
    pay = torch.arange(300007, dtype=torch.int64, device="cuda") * 5
    k = 777
    vals = torch.empty(k, dtype=t.dtype, device="cuda")
    out = torch.empty(k, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    say("payload, no positions")
    rc = drt.lib().topk_select_payload(ctypes.c_void_p(t.data_ptr()), t.numel(), k, drt.U32,
                                       ctypes.c_void_p(pay.data_ptr()), 8, ctypes.c_void_p(vals.data_ptr()), None,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    wv, wi = drt.topk_select(t, k)
    torch.cuda.synchronize()
    assert (to_np(vals).view(np.uint32) == to_np(wv).view(np.uint32)).all()
    assert (to_np(out) == to_np(wi).view(np.uint32).astype(np.int64) * 5).all()

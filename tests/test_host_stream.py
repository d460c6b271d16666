"""Top-k of keys in host memory streamed through the device in chunks, against
the oracle and, bit for bit, against topk_select on the whole input in device
memory: ragged chunks, k larger than a chunk, one chunk, both orders and every
key type."""
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


@pytest.mark.parametrize("kind,largest", [("uniform_u32", True), ("normal_f32", True), ("normal_f32", False),
                                          ("heavydup_u32", True), ("smallrange_i32", False), ("revsorted_f32", False),
                                          ("sorted_f32", True)])
def test_chunks_equal_whole(kind, largest):
    n = (1 << 24) + 13
    x, dt = synth.keys(kind, n, 5150)
    t = torch.from_numpy(x).cuda()
    for k, chunk in [(1, (1 << 21) + 5), (100, (1 << 21) + 5), (5000, 1 << 22), (70000, (1 << 21) + 5), (300, n)]:
        say(kind, "largest" if largest else "smallest", "k", k, "chunk", chunk)
        v, ix = drt.topk_select_host(x, k, chunk=chunk, largest=largest)
        wv, wi = drt.topk_select(t, k, largest=largest)
        torch.cuda.synchronize()
        assert (to_np(v).view(np.uint32) == to_np(wv).view(np.uint32)).all(), (kind, k, chunk)
        assert (to_np(ix) == to_np(wi)).all(), (kind, k, chunk)
        if k <= 5000:
            check_exact(x, k, dt, to_np(v), to_np(ix), f"{kind} k={k} chunk={chunk}", largest=largest)


def test_k_larger_than_chunk_and_tiny_inputs():
    x, dt = synth.keys("uniform_u32", (1 << 20) + 3, 77)
    say("k 5000 over chunks of 1000")
    v, ix = drt.topk_select_host(x, 5000, chunk=1000)
    check_exact(x, 5000, dt, to_np(v), to_np(ix), "k > chunk")
    for n in (1, 2, 7):
        y, dy = synth.keys("normal_f32", n, 3 + n)
        for k in range(1, n + 1):
            say("tiny", n, k)
            v, ix = drt.topk_select_host(y, k, chunk=1)
            check_exact(y, k, dy, to_np(v), to_np(ix), f"tiny n={n} k={k}")

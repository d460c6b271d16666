"""Calls from several host threads at once, each on its own stream (the
library keeps one workspace per device and stream, locked for each enqueue):
every result equals the same call made alone, bit for bit."""
import sys
import threading

import numpy as np
import pytest

import synth
from checks import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_threads_on_separate_streams():
    jobs = []
    kinds = ["uniform_u32", "normal_f32", "smallrange_i32", "heavydup_u32"]
    for i in range(16):
        x, _ = synth.keys(kinds[i % 4], (1 << 20) + 37 * i, 9000 + i)
        k = [1, 100, 3000, 20000][(i // 4) % 4]
        jobs.append((torch.from_numpy(x).cuda(), k, i % 3 != 0))
    ref = []
    for t, k, largest in jobs:
        v, ix = drt.topk_select(t, k, largest=largest)
        ref.append((to_np(v).view(np.uint32).copy(), to_np(ix).copy()))
    torch.cuda.synchronize()
    results = [[None] * len(jobs) for _ in range(4)]
    errors = []

    def worker(w):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(3):
                    for j in range(w, len(jobs), 4) if rep % 2 == 0 else range(len(jobs) - 1 - w, -1, -4):
                        t, k, largest = jobs[j]
                        v, ix = drt.topk_select(t, k, largest=largest, stream=s)
                        s.synchronize()
                        results[w][j] = (to_np(v).view(np.uint32).copy(), to_np(ix).copy())
        except Exception as e:  # reported by the main thread
            errors.append(repr(e))

    say("4 threads x 3 rounds")
    ths = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errors, errors
    for w in range(4):
        for j, r in enumerate(results[w]):
            if r is None:
                continue
            assert (r[0] == ref[j][0]).all() and (r[1] == ref[j][1]).all(), (w, j)

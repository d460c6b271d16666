"""A seeded random sweep of single problems against the oracle, element by
element: n log-uniform up to 2^22 (ragged sizes), k from 1 to n with small k
favoured, every input kind, both orders, and in a third of the cases explicit
method parameters (subrange size, delegates per subrange, route, tail
variant).  Each case prints its parameters first, so a failure names it."""
import sys

import numpy as np
import pytest

import oracle
import synth
from checks import check_exact, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")

KINDS = ["uniform_u32", "normal_f32", "sorted_f32", "revsorted_f32", "heavydup_u32", "uniform_i32",
         "smallrange_i32"]


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def draw_cases(count, seed):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        n = int(np.rint(2.0 ** rng.uniform(0, 22)))
        n = max(1, n + int(rng.integers(0, 7)))
        u = rng.random()
        k = 1 + int(rng.integers(0, min(n, 64))) if u < 0.5 else 1 + int(rng.integers(0, n))
        opts = {}
        if rng.random() < 1 / 3 and n > 64:
            mode = int(rng.integers(1, 3))
            opts["mode"] = mode
            if mode == 1:
                opts["alpha"] = int(rng.integers(0, 15))
                opts["beta"] = int(rng.choice([1, 2, 4, 8]))
                opts["variant"] = int(rng.integers(0, 2))
        cases.append((KINDS[int(rng.integers(0, len(KINDS)))], n, k, bool(rng.random() < 0.7), opts,
                      synth.derive_seed(seed, i)))
    return cases


@pytest.mark.parametrize("part", range(4))
def test_random_sweep(part):
    for kind, n, k, largest, opts, s in draw_cases(150, 777 + part):
        x, dt = synth.keys(kind, n, s)
        say(kind, "n", n, "k", k, "largest" if largest else "smallest", opts)
        vals, idx = drt.topk_select(torch.from_numpy(x).cuda(), k, largest=largest, stats=True, check=True, **opts)[:2]
        torch.cuda.synchronize()
        check_exact(x, k, dt, to_np(vals), to_np(idx), f"{kind} n={n} k={k} {opts}", largest=largest)

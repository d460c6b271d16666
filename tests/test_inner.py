"""The delegate method with other top-k algorithms inside (variant 2: bitonic
top-k, k <= 256; variant 3: bucket select), against the oracle element by
element across subrange sizes, delegates per subrange, orders and key types,
plus their first selection checked stage-wise: the survivors of the filter
are exactly the oracle's candidate set (both find the exact k-th delegate)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import stages
from checks import check_exact, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")

KINDS = ["uniform_u32", "normal_f32", "sorted_f32", "heavydup_u32", "smallrange_i32"]


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(t, k, **kw):
    vals, idx, _ = drt.topk_select(t, k, stats=True, check=True, mode=1, **kw)
    torch.cuda.synchronize()
    return to_np(vals), to_np(idx)


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("kind", KINDS)
def test_variant_alpha_beta_sweep(kind, variant):
    n = (1 << 18) + 77
    x, dt = synth.keys(kind, n, 31 + variant)
    t = dev(x)
    ks = (1, 7, 100, 256) if variant == 2 else (1, 100, 3000, 20000)
    for k in ks:
        for largest in (True, False):
            want = oracle.topk_reference(x, k, dt, largest)
            for alpha in (2, 5, 8, 10, 12):
                for beta in (1, 2, 4, 8):
                    say(kind, "variant", variant, "k", k, "alpha", alpha, "beta", beta, "largest", largest)
                    vals, idx = run(t, k, alpha=alpha, beta=beta, variant=variant, largest=largest)
                    assert (idx.view(np.uint32) == want[1]).all(), (kind, variant, k, alpha, beta, largest)
                    assert (vals.view(np.uint32) == want[0].view(np.uint32)).all()


@pytest.mark.parametrize("variant", [2, 3])
def test_variant_planner_alpha_sizes(variant):
    """The planner's subranges, sizes across delegate chunks and ragged tails,
    fewer delegates than k (every subrange qualifies), and k-selection."""
    for kind in ("uniform_u32", "normal_f32", "heavydup_u32"):
        for n in (1000, 65537, (1 << 20) + 13, (1 << 22) + 5):
            x, dt = synth.keys(kind, n, 700 + n)
            t = dev(x)
            for k in (1, 33, 256) if variant == 2 else (1, 33, 1000, 9000):
                if k > n:
                    continue
                say("planner alpha", kind, "variant", variant, "n", n, "k", k)
                vals, idx = run(t, k, variant=variant)
                check_exact(x, k, dt, vals, idx, f"{kind} v{variant} n={n} k={k}")
        # fewer real delegates than k: 1000 keys in subranges of 256
        x, dt = synth.keys(kind, 1000, 5)
        say("all qualify", kind, variant)
        vals, idx = run(dev(x), 100, alpha=8, beta=1, variant=variant)
        check_exact(x, 100, dt, vals, idx, f"{kind} v{variant} all qualify")


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("kind", ["uniform_u32", "normal_f32", "sorted_f32", "heavydup_u32"])
def test_variant_candidate_stage(kind, variant):
    n = (1 << 17) + 3
    x, dt = synth.keys(kind, n, 12)
    for alpha, beta, k in [(4, 1, 50), (6, 2, 200), (8, 1, 256), (5, 8, 64), (2, 1, 7), (9, 4, 3000)]:
        if variant == 2 and k > 256:
            continue
        _, _, info = stages.method_topk(x, k, dt, alpha, beta)
        say("candidates", kind, "variant", variant, alpha, beta, k)
        got, (tbits, tpos) = drt.candidates(dev(x), k, alpha, beta, variant=variant)
        got = np.sort(to_np(got).view(np.uint32).astype(np.int64))
        assert (got == info["candidates"]).all(), (kind, variant, alpha, beta, k, got.size, info["candidates"].size)
        if info["t"] is not None:  # the exact k-th delegate
            tv = oracle.rank_key(np.array([tbits], dtype=np.uint32).view(x.dtype), dt)[0]
            assert (tv, tpos) == info["t"], (kind, variant, alpha, beta, k)


def test_bitonic_rejects_large_k():
    t = dev(synth.uniform_u32(10000, 1))
    with pytest.raises(drt.DrTopkError):
        drt.topk_select(t, 257, mode=1, variant=2)

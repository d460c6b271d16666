"""The k smallest, and int32 keys, through the C-ABI, against the oracle.

Both come from the key codec alone (the same kernels run on complemented or
sign-flipped encodings), so the cases sweep sizes, k, explicit subrange
sizes and delegate counts, the batched form with codecs and orders mixed in
one launch, the serving loop, float specials, and one large input per codec
checked by invariants that fix the answer uniquely.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from checks import check_exact, check_invariants, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def kth_bits(x, k, dt, largest):
    return int(np.asarray(oracle.kth_value(x, k, dt, largest)).view(np.uint32))


CASES = [("uniform_u32", False), ("normal_f32", False), ("revsorted_f32", False), ("sorted_f32", False),
         ("heavydup_u32", False), ("uniform_i32", False), ("uniform_i32", True), ("smallrange_i32", False),
         ("smallrange_i32", True)]


@pytest.mark.parametrize("kind,largest", CASES)
def test_sizes_and_k(kind, largest):
    for n in (1, 3, 1000, 8193, 65537, 300007, (1 << 20) + 13):
        x, dt = synth.keys(kind, n, 3000 + n)
        t = dev(x)
        for k in sorted({k for k in (1, 2, 33, 1024, 8193, 20000, n) if k <= n}):
            say(kind, "largest" if largest else "smallest", "n", n, "k", k)
            vals, idx = drt.topk_select(t, k, largest=largest, stats=True, check=True)[:2]
            kth = drt.kth_select(t, k, largest=largest)
            torch.cuda.synchronize()
            check_exact(x, k, dt, to_np(vals), to_np(idx), f"{kind} n={n} k={k}", largest=largest)
            assert int(to_np(kth).view(np.uint32)[0]) == kth_bits(x, k, dt, largest), (kind, n, k)


@pytest.mark.parametrize("kind", ["normal_f32", "smallrange_i32", "revsorted_f32"])
def test_alpha_beta_invariance_smallest(kind):
    n = (1 << 18) + 77
    x, dt = synth.keys(kind, n, 8)
    t = dev(x)
    for k in (1, 100, 5000):
        want = oracle.topk_reference(x, k, dt, False)
        for alpha in (0, 3, 8, 10, 12):
            for beta in (1, 2, 4, 8):
                say(kind, "smallest k", k, "alpha", alpha, "beta", beta)
                vals, idx = drt.topk_select(t, k, largest=False, alpha=alpha, beta=beta, mode=1, stats=True, check=True)[:2]
                torch.cuda.synchronize()
                assert (to_np(idx).view(np.uint32) == want[1]).all(), (kind, k, alpha, beta)
                assert (to_np(vals).view(np.uint32) == np.asarray(want[0]).view(np.uint32)).all()


def test_float_specials_smallest():
    """Every class of float32 bit pattern, smallest first by IEEE totalOrder."""
    pats = np.array([0xFFFFFFFF, 0xFF800001, 0xFF800000, 0xBF800000, 0x80000001, 0x80000000, 0x00000000,
                     0x00000001, 0x3F800000, 0x7F800000, 0x7FC00000, 0x7FFFFFFF], dtype=np.uint32)
    rng = np.random.default_rng(3)
    x = pats[rng.integers(0, pats.shape[0], size=100003)].view(np.float32)
    for k in (1, 7, 5000, 100003):
        say("float specials smallest", k)
        vals, idx = drt.topk_select(dev(x), k, largest=False, stats=True, check=True)[:2]
        torch.cuda.synchronize()
        check_exact(x, k, "f32", to_np(vals), to_np(idx), f"specials k={k}", largest=False)


def _mixed_problems(count, seed):
    """The batched workload with codecs and orders varied per instance."""
    hosts = []
    kinds = ["uniform_u32", "normal_f32", "uniform_i32", "smallrange_i32", "revsorted_f32"]
    for i, (_, n, k, s) in enumerate(synth.batched_workload(count, seed)):
        x, dt = synth.keys(kinds[i % len(kinds)], n, s)
        hosts.append((x, dt, k, (i // len(kinds)) % 2 == 0))
    return hosts


def beta2_table():
    """Rule 4's alpha with two delegates per subrange in every bucket of the batched form."""
    drt.tune_set([])
    entries = []
    for lg_n in range(12, 23):
        for lg_k in range(0, 12):
            n, k = max(1 << lg_n, 4097), 1 << lg_k
            if k <= n:
                r, a, _ = drt.batched_plan(n, k)
                if r == 2:
                    entries.append((drt.FORM_BATCHED, lg_n, lg_k, a, 2))
    return entries


@pytest.mark.parametrize("beta", [1, 2])
def test_batched_mixed_codecs_and_orders(beta):
    saved = drt.tune_get()
    try:
        if beta == 2:
            drt.tune_set(beta2_table())
        batched_mixed(beta)
    finally:
        drt.tune_set(saved)


def batched_mixed(beta):
    hosts = _mixed_problems(300, 611)
    # split problems (several workgroups per delegate vector) in both orders
    for j, kind in enumerate(("normal_f32", "uniform_i32")):
        x, dt = synth.keys(kind, (1 << 20) + 5, 90 + j)
        hosts.append((x, dt, 2048, j == 1))
        hosts.append((x, dt, 1000, j == 0))
    tensors = [(dev(x), k, None, largest) for x, dt, k, largest in hosts]
    if beta == 2:
        assert sum(drt.batched_plan(x.shape[0], k)[2] == 2 for x, _, k, _ in hosts) > len(hosts) // 2
    say("batched mixed", len(hosts), "beta", beta)
    b = drt.Batch(tensors)
    b.run()
    torch.cuda.synchronize()
    for i, (x, dt, k, largest) in enumerate(hosts):
        check_exact(x, k, dt, to_np(b.values(i)), to_np(b.indices(i)), f"batched #{i}", largest=largest)
        assert int(to_np(b.kth_value(i)).view(np.uint32)[0]) == kth_bits(x, k, dt, largest), i
    for i in range(0, len(hosts), 23):  # bit for bit the single-problem path
        t, k, _, largest = tensors[i]
        v, ix = drt.topk_select(t, k, largest=largest)
        torch.cuda.synchronize()
        assert (to_np(v).view(np.uint32) == to_np(b.values(i)).view(np.uint32)).all(), i
        assert (to_np(ix) == to_np(b.indices(i))).all(), i


def test_serving_mixed_orders():
    hosts = _mixed_problems(120, 612)
    tensors = [(dev(x), k, None, largest) for x, dt, k, largest in hosts]
    b = drt.Batch(tensors)
    arr = synth.poisson_arrivals(len(tensors), 30000.0, 4)
    say("serving mixed orders")
    with drt.Server(streams=4, max_batch=32) as srv:
        srv.replay(b, arr)
        st = srv.stats()
    torch.cuda.synchronize()
    assert st.completed == len(tensors)
    for i, (x, dt, k, largest) in enumerate(hosts):
        check_exact(x, k, dt, to_np(b.values(i)), to_np(b.indices(i)), f"serving #{i}", largest=largest)


@pytest.mark.parametrize("kind,ks", [("normal_f32", (1, 1024, 131072)), ("uniform_i32", (16384,)),
                                     ("smallrange_i32", (4096,))])
def test_large_smallest(kind, ks):
    """2^28 keys, the k smallest, checked by the invariants I1-I6 in reverse order."""
    x, dt = synth.keys(kind, 1 << 28, synth.DEFAULT_SEED)
    t = dev(x)
    for k in ks:
        say("large smallest", kind, "k", k)
        vals, idx, st = drt.topk_select(t, k, largest=False, stats=True, check=True)
        say("  alpha", st.alpha, "beta", st.beta, "scanned", st.scanned, "candidates", st.candidates)
        check_invariants(x, k, dt, to_np(vals), to_np(idx), f"{kind} 2^28 k={k}", largest=False)
    del t
    torch.cuda.empty_cache()

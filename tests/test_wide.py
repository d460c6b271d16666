"""64-bit keys (uint64, int64, float64 by totalOrder) on the HIP path, through
the C ABI, against the oracle element by element: sizes across delegate
chunks and ragged tails, both orders, every route (delegate method with
subranges of 2^7..2^13 keys, plain radix select, few and many survivors,
k above one workgroup's sort), keys whose order is decided by the low word,
ties, float64 specials, 8-byte-aligned (not 16) inputs, k-selection, batches
mixing 32- and 64-bit problems, payloads, the no-allocation entry point, and
N = 2^28 exactly and 2^29 by invariants."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
import oracle_pins as pins
from checks import check_exact, check_invariants, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")

KINDS = ["uniform_u64", "uniform_i64", "normal_f64", "sorted_f64", "heavydup_u64", "smallrange_i64", "highword_u64"]


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(t, k, **kw):
    vals, idx, st = drt.topk_select(t, k, stats=True, check=True, **kw)
    torch.cuda.synchronize()
    return to_np(vals), to_np(idx), st


@pytest.mark.parametrize("kind", KINDS)
def test_sizes_and_k(kind):
    for n in (1, 7, 1000, 8193, 65539, 300007, (1 << 22) + 17):
        x, dt = synth.keys(kind, n, 5000 + n)
        t = dev(x)
        for k in sorted({k for k in (1, 17, 1000, 5000, n) if 1 <= k <= n}):
            for largest in (True, False):
                say(kind, "n", n, "k", k, "largest", largest)
                v, i, st = run(t, k, largest=largest)
                check_exact(x, k, dt, v, i, f"{kind} n={n} k={k} largest={largest} mode={st.mode}", largest=largest)


@pytest.mark.parametrize("alpha", [7, 8, 10, 13])
def test_delegate_method_alpha(alpha):
    n = (1 << 21) + 5
    for kind in ("uniform_u64", "normal_f64", "highword_u64", "sorted_f64"):
        x, dt = synth.keys(kind, n, 77 + alpha)
        t = dev(x)
        for k in (1, 100, 4096, 4097, 9000):
            if (n >> alpha) < k:
                continue
            say(kind, "alpha", alpha, "k", k)
            v, i, st = run(t, k, alpha=alpha, mode=1)
            assert st.mode == 1 and st.alpha == alpha
            check_exact(x, k, dt, v, i, f"{kind} alpha={alpha} k={k}")


def test_plain_radix_mode():
    n = (1 << 20) + 3
    for kind in ("uniform_i64", "normal_f64", "heavydup_u64"):
        x, dt = synth.keys(kind, n, 31)
        t = dev(x)
        for k in (1, 64, 4096, 70000):
            say("mode 2", kind, "k", k)
            v, i, st = run(t, k, mode=2)
            assert st.mode == 2
            check_exact(x, k, dt, v, i, f"mode 2 {kind} k={k}")


def test_float64_specials():
    chain = pins.f64_chain()
    rng = np.random.default_rng(3)
    body = synth.normal_f64(50000, 9)
    x = np.concatenate([body.view(np.uint64), np.repeat(chain, 37)])
    x = x[rng.permutation(x.shape[0])].view(np.float64)
    t = dev(x)
    for k in (1, 5, 100, 900, 5000):
        for largest in (True, False):
            say("f64 specials k", k, largest)
            v, i, _ = run(t, k, largest=largest)
            check_exact(x, k, "f64", v, i, f"f64 specials k={k}", largest=largest)


def test_unaligned_8_byte():
    x, dt = synth.keys("uniform_u64", (1 << 20) + 9, 12)
    base = dev(x)
    t = base[1:]  # 8-byte but not 16-byte aligned
    assert t.data_ptr() % 16 == 8
    for k in (1, 3000):
        say("unaligned k", k)
        v, i, _ = run(t, k, mode=1, alpha=8)  # 4097 subranges >= k
        check_exact(x[1:], k, dt, v, i, f"unaligned k={k}")


def test_kth_select_wide():
    for kind in ("uniform_u64", "smallrange_i64", "normal_f64"):
        x, dt = synth.keys(kind, (1 << 22) + 1, 44)
        t = dev(x)
        for k in (1, 777, 8192, 100000):
            for largest in (True, False):
                say("kth", kind, k, largest)
                got = to_np(drt.kth_select(t, k, largest=largest, check=True))[0]
                want = oracle.kth_value(x, k, dt, largest)
                assert oracle.order.bits(np.array([got]))[0] == oracle.order.bits(np.array([want]))[0], (kind, k)


def test_batched_mix_and_payload_and_noalloc():
    probs = []
    for j, kind in enumerate(("uniform_u32", "normal_f64", "uniform_i64", "normal_f32", "highword_u64")):
        x, dt = synth.keys(kind, 100000 + 77 * j, 900 + j)
        probs.append((x, dt, dev(x), 50 + 300 * j))
    say("batched mix of 32- and 64-bit problems")
    res = drt.topk_select_batched([(t, k) for _, _, t, k in probs], check=True)
    torch.cuda.synchronize()
    for (x, dt, t, k), (v, i, kth) in zip(probs, res):
        check_exact(x, k, dt, to_np(v), to_np(i), f"batched {dt} k={k}")
        wv, wi = drt.topk_select(t, k)
        assert (oracle.order.bits(to_np(v)) == oracle.order.bits(to_np(wv))).all()
        assert oracle.order.bits(to_np(kth))[0] == oracle.order.bits(to_np(wv))[-1]
    # payload gathered by the selected positions
    x, dt = synth.keys("normal_f64", 500001, 5)
    t = dev(x)
    pay = torch.arange(500001, dtype=torch.int64, device="cuda") * 3
    say("payload with 64-bit keys")
    v, i, p = drt.topk_select_payload(t, pay, 2000)
    torch.cuda.synchronize()
    check_exact(x, 2000, dt, to_np(v), to_np(i), "payload f64")
    assert (to_np(p) == to_np(i).view(np.uint32).astype(np.int64) * 3).all()
    # the no-allocation entry point
    stream = torch.cuda.current_stream()
    vals = torch.empty(3000, dtype=t.dtype, device="cuda")
    idx = torch.empty(3000, dtype=torch.int32, device="cuda")
    say("noalloc with 64-bit keys")
    rc = drt.lib().topk_select_noalloc(ctypes.c_void_p(t.data_ptr()), t.numel(), 3000, drt.F64,
                                       ctypes.c_void_p(vals.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                       ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0
    drt.check_stream()
    check_exact(x, 3000, dt, to_np(vals), to_np(idx), "noalloc f64")


@pytest.mark.parametrize("kind,k", [("uniform_u64", 1024), ("normal_f64", 131072), ("sorted_f64", 16384),
                                    ("highword_u64", 4096)])
def test_large(kind, k):
    n = (1 << 26) + 3
    x, dt = synth.keys(kind, n, 2026)
    t = dev(x)
    say("large", kind, "n 2^26+3 k", k)
    v, i, st = run(t, k)
    check_exact(x, k, dt, v, i, f"{kind} n=2^26+3 k={k} mode={st.mode}")


@pytest.mark.parametrize("kind", ["uniform_u64", "normal_f64"])
def test_full_size_2p28(kind):
    n = 1 << 28
    x, dt = synth.keys(kind, n, synth.DEFAULT_SEED)
    t = dev(x)
    for k in (1, 1024, 131072):
        say("2^28", kind, "k", k)
        v, i, st = run(t, k)
        check_exact(x, k, dt, v, i, f"{kind} n=2^28 k={k}")
    del t
    torch.cuda.empty_cache()


def test_full_size_2p29_invariants():
    n = 1 << 29
    x, dt = synth.keys("uniform_i64", n, 29)
    t = dev(x)
    for k in (16384,):
        for largest in (True, False):
            say("2^29 i64 k", k, largest)
            v, i, _ = run(t, k, largest=largest)
            check_invariants(x, k, dt, v, i, f"i64 n=2^29 k={k}", largest=largest)
    del t
    torch.cuda.empty_cache()

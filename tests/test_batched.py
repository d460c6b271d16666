"""Batched form vs the oracle and vs the single-problem path, through the C-ABI.

Every batched problem must equal the oracle's answer for it and, bit for bit,
what topk_select / kth_select give for the same problem alone.  The cases
reach each route a problem can take in the persistent kernel (sorted
outright, delegate method in LDS, radix select when the survivors overflow)
and the single-problem path for problems too large for one workgroup.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from checks import check_exact, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(autouse=True)
def default_tuning():
    """Each test starts and ends with the table the binding loads by default."""
    saved = drt.tune_get()
    yield
    drt.tune_set(saved)


def run_batch(hosts, *, kth_only=False, offsets=None):
    """hosts: list of (x, dtype, k).  Returns the Batch after it ran."""
    tensors = []
    for i, (x, dt, k) in enumerate(hosts):
        off = offsets[i] if offsets else 0
        t = dev(np.concatenate([np.zeros(off, dtype=x.dtype), x]))[off:] if off else dev(x)
        tensors.append((t, k))
    b = drt.Batch(tensors, kth_only=kth_only)
    b.run(check=True)
    return b


def check_batch(hosts, b, what):
    for i, (x, dt, k) in enumerate(hosts):
        kth = to_np(b.kth_value(i)).view(np.uint32)[0]
        want_kth = np.asarray(oracle.kth_value(x, k, dt)).view(np.uint32)
        assert kth == want_kth, (what, i, x.shape[0], k)
        if not b.kth_only:
            check_exact(x, k, dt, to_np(b.values(i)), to_np(b.indices(i)), f"{what} #{i} n={x.shape[0]} k={k}")


def workload_hosts(count, seed):
    hosts = []
    for kind, n, k, s in synth.batched_workload(count, seed):
        x, dt = synth.keys(kind, n, s)
        hosts.append((x, dt, k))
    return hosts


def test_routes_are_planned():
    drt.tune_set([])  # Rule 4's plan; the fixture restores the tuned table
    assert drt.batched_route(4096, 100) == (1, 0)
    r, a = drt.batched_route(1 << 20, 1024)
    # split across workgroups: the delegate vector in global memory, up to 32768 entries
    assert r == 2 and a >= 4 and -(-(1 << 20) // (1 << a)) <= 32768
    r, a = drt.batched_route(1 << 18, 1024)  # above 2^16 keys the vector may live in global memory too
    assert r == 2 and a >= 4 and -(-(1 << 18) // (1 << a)) <= 32768
    r, a = drt.batched_route(1 << 16, 1024)  # one workgroup: the vector in its LDS
    assert r == 2 and -(-(1 << 16) // (1 << a)) <= 4096
    assert drt.batched_route((1 << 22) + 1, 10)[0] == 0
    assert drt.batched_route(1 << 16, 2049)[0] == 0


def test_workload_sample_exact():
    """The batched workload recipe (lengths log-uniform in [2^10, 2^20], k <= 2048,
    uint32 uniform or float32 normal per instance) on 256 instances."""
    hosts = workload_hosts(256, 4242)
    say("workload 256")
    b = run_batch(hosts)
    check_batch(hosts, b, "workload")


def test_each_route():
    drt.tune_set([])  # Rule 4's plan, so the routes below are the ones asserted
    hosts = []
    # sorted outright in the workgroup
    for n, k in [(1, 1), (2, 2), (3, 1), (100, 37), (1000, 1000), (4095, 3), (4096, 2048)]:
        for kind in ("uniform_u32", "normal_f32", "heavydup_u32"):
            x, dt = synth.keys(kind, n, 31 + n)
            assert drt.batched_route(n, k)[0] == 1
            hosts.append((x, dt, k))
    # delegate method in LDS, short and long subranges, ragged last subrange
    for n, k in [(4097, 5), (8193, 1), (8193, 2048), (65541, 1), (65541, 7), (65541, 2048), ((1 << 20) + 5, 1000),
                 ((1 << 22), 2048), ((1 << 22) - 3, 1), (300000, 1), (300000, 1999)]:
        for kind in ("uniform_u32", "normal_f32"):
            x, dt = synth.keys(kind, n, 57 + n)
            assert drt.batched_route(n, k)[0] == 2
            hosts.append((x, dt, k))
    # too few subranges for k: radix select in the workgroup
    for n, k in [(8192, 2048), (6000, 1600)]:
        for kind in ("uniform_u32", "heavydup_u32"):
            x, dt = synth.keys(kind, n, 71 + n)
            assert drt.batched_route(n, k)[0] == 3
            hosts.append((x, dt, k))
    # survivors overflow the workgroup: ascending input and 16 distinct values
    for n, k in [(1 << 18, 2000), (100003, 64), (1 << 20, 2048)]:
        for kind in ("sorted_f32", "heavydup_u32"):
            x, dt = synth.keys(kind, n, 91 + n)
            hosts.append((x, dt, k))
    say("routes", len(hosts))
    b = run_batch(hosts)
    check_batch(hosts, b, "routes")


@pytest.mark.parametrize("beta", [1, 2])
@pytest.mark.parametrize("alpha", [2, 3, 5, 8, 9, 11, 13, 16])
def test_tuned_alpha_is_exact(alpha, beta):
    """Any table entry gives the same (exact) results: the kernel only raises
    alpha to fit its delegate vector or lowers it to keep more delegates than k."""
    hosts = []
    for i, (n, k) in enumerate([(9000, 1), (9000, 1500), (40000, 33), (200000, 2048), (600001, 300),
                                ((1 << 20) + 1, 2000)]):
        x, dt = synth.keys("normal_f32" if i % 2 else "uniform_u32", n, 300 + i)
        hosts.append((x, dt, k))
    entries = []
    for x, dt, k in hosts:
        lg_n, lg_k = int(np.log2(x.shape[0])), int(np.log2(k))
        entries.append((drt.FORM_BATCHED, lg_n, lg_k, alpha, beta))
    drt.tune_set(entries)
    for x, dt, k in hosts:
        r, _, b = drt.batched_plan(x.shape[0], k)
        assert r != 2 or b == beta
    say("tuned alpha", alpha, "beta", beta)
    b = run_batch(hosts)
    check_batch(hosts, b, f"alpha {alpha} beta {beta}")


def test_batched_equals_single_bitwise():
    hosts = workload_hosts(64, 777)
    big = [(synth.keys("uniform_u32", (1 << 22) + 1, 5)[0], "u32", 100),
           (synth.keys("normal_f32", 1 << 16, 6)[0], "f32", 3000)]
    hosts = hosts[:32] + big + hosts[32:]
    say("batched vs single", len(hosts))
    b = run_batch(hosts)
    for i, (x, dt, k) in enumerate(hosts):
        t = dev(x)
        v, ix = drt.topk_select(t, k)
        kth = drt.kth_select(t, k)
        torch.cuda.synchronize()
        assert (to_np(b.values(i)).view(np.uint32) == to_np(v).view(np.uint32)).all(), i
        assert (to_np(b.indices(i)) == to_np(ix)).all(), i
        assert to_np(b.kth_value(i)).view(np.uint32)[0] == to_np(kth).view(np.uint32)[0], i
    check_batch(hosts, b, "mixed")


def test_kth_only_and_unaligned():
    hosts = workload_hosts(48, 99)
    say("kth only")
    b = run_batch(hosts, kth_only=True)
    check_batch(hosts, b, "kth only")
    say("unaligned")
    b = run_batch(hosts, offsets=[1 + (i % 3) for i in range(len(hosts))])
    check_batch(hosts, b, "unaligned")


def test_repeat_reuse_and_side_stream():
    hosts = workload_hosts(40, 123)
    tensors = [(dev(x), k) for x, _, k in hosts]
    b = drt.Batch(tensors)
    small = drt.Batch(tensors[:5])
    s = torch.cuda.Stream()
    for rep in range(3):
        say("repeat", rep)
        b.vals.fill_(0)
        with torch.cuda.stream(s):
            b.run(stream=s)
            small.run(stream=s)
        s.synchronize()
        check_batch(hosts, b, f"repeat {rep}")
        check_batch(hosts[:5], small, f"repeat small {rep}")


def test_errors():
    t = dev(synth.uniform_u32(100, 1))
    with pytest.raises(drt.DrTopkError):
        drt.topk_select_batched([(t, 5), (t, 101)])
    with pytest.raises(ValueError):  # 2-byte elements
        drt.topk_select_batched([(t.view(torch.float16), 5)])


def test_full_workload_4096():
    """The full batched workload: 4096 instances, every one checked exactly."""
    hosts = workload_hosts(4096, synth.DEFAULT_SEED)
    say("full 4096")
    b = run_batch(hosts)
    check_batch(hosts, b, "full")


def beta2_table():
    """Rule 4's alpha for every bucket the batched kernel owns, with two
    delegates per subrange."""
    drt.tune_set([])
    entries = []
    for lg_n in range(12, 23):
        for lg_k in range(0, 12):
            n, k = max(1 << lg_n, 4097), 1 << lg_k  # n = 2^12 itself is sorted outright
            if k > n:
                continue
            r, a, _ = drt.batched_plan(n, k)
            if r == 2:
                entries.append((drt.FORM_BATCHED, lg_n, lg_k, a, 2))
    return entries


def test_beta2_workload_exact():
    """Two delegates per subrange (Rule 3) in every bucket of the workload:
    exact, and bit for bit what single calls give (problems of at most 2^16
    keys take the one-workgroup path there, with the same beta)."""
    drt.tune_set(beta2_table())
    hosts = workload_hosts(1024, 4321)
    n2 = sum(drt.batched_plan(x.shape[0], k)[2] == 2 for x, _, k in hosts)
    assert n2 > len(hosts) // 2, n2
    say("beta 2 workload", len(hosts), "with beta 2:", n2)
    b = run_batch(hosts)
    check_batch(hosts, b, "beta 2")
    for i, (x, dt, k) in enumerate(hosts[:: 16]):
        t = dev(x)
        v, ix, st = drt.topk_select(t, k, stats=True, check=True)
        torch.cuda.synchronize()
        r, a, beta = drt.batched_plan(x.shape[0], k)
        if st.mode == 3 and st.alpha:
            assert (st.alpha, st.beta, st.delegates) == (a, beta, beta * st.subranges)
        check_exact(x, k, dt, to_np(v), to_np(ix), f"beta 2 single n={x.shape[0]} k={k}")
    say("beta 2 unaligned + k only")
    b = run_batch(hosts[:200], offsets=[1 + (i % 3) for i in range(200)])
    check_batch(hosts[:200], b, "beta 2 unaligned")
    b = run_batch(hosts[:200], kth_only=True)
    check_batch(hosts[:200], b, "beta 2 k only")


@pytest.mark.parametrize("beta", [1, 2])
def test_split_problems(beta):
    """Problems above 2^16 keys on the delegate route: several workgroups build
    the delegate vector, the last to arrive finishes.  Ragged tails, unaligned
    views, k-only outputs, adversarial inputs (survivor overflow after the
    split) and repeated launches (the arrival counters restart at zero)."""
    drt.tune_set(beta2_table() if beta == 2 else [])
    hosts = []
    for i, (n, k) in enumerate([((1 << 18) + 1, 1), ((1 << 18) + 3, 7), ((1 << 19) + 2, 500), ((1 << 20) + 7, 2048),
                                ((1 << 22) - 1, 1000), (1 << 22, 1), (3 << 19, 64), ((1 << 16) + 5, 2048),
                                ((1 << 17) + 3, 1500), (3 << 16, 900)]):
        for kind in ("uniform_u32", "normal_f32"):
            x, dt = synth.keys(kind, n, 800 + 2 * i + (kind == "normal_f32"))
            assert drt.batched_plan(n, k)[::2] == (2, beta)
            hosts.append((x, dt, k))
    for kind in ("sorted_f32", "heavydup_u32"):
        x, dt = synth.keys(kind, (1 << 20) + 5, 901)
        hosts.append((x, dt, 2048))
    small = [h for h in workload_hosts(40, 55)]
    allh = hosts + small
    say("split problems", len(allh))
    b = run_batch(allh)
    check_batch(allh, b, "split")
    b.run(check=True)  # second launch on the same descriptors
    check_batch(allh, b, "split repeat")
    say("split, unaligned + k only")
    b = run_batch(hosts, offsets=[1 + (i % 3) for i in range(len(hosts))])
    check_batch(hosts, b, "split unaligned")
    b = run_batch(hosts, kth_only=True)
    check_batch(hosts, b, "split k only")

"""HIP path vs the oracle, element by element, through the C-ABI.

Sizes span several delegate chunks, subrange shapes and ragged tails; the
workloads follow the paper's uniform dataset plus this project's normal,
sorted and heavy-duplicate stand-ins; the full-size cases run the planner's
choice at N = 2^30 (and 2^29 for the adversarial inputs) and are checked by
invariants that fix the answer uniquely.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import stages
from checks import check_exact, check_invariants, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

drt = pytest.importorskip("paper_2109_08219_amd")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_topk(x, k, **kw):
    # stats=True and check=True synchronise and raise if a kernel flagged an internal inconsistency
    vals, idx = drt.topk_select(dev(x), k, stats=True, check=True, **kw)[:2]
    torch.cuda.synchronize()
    return to_np(vals), to_np(idx)


KINDS = ["uniform_u32", "normal_f32", "sorted_f32", "heavydup_u32"]


def ks_for(n):
    return sorted({k for k in (1, 2, 33, 1024, 8192, 8193, 20000, n) if 1 <= k <= n})


def test_config_small_uniform_k1024():
    """N = 2^20 uint32 uniform, k = 1024: sorted values, positions and k-th value."""
    x = synth.uniform_u32(1 << 20, synth.DEFAULT_SEED)
    say("n=2^20 u32 uniform k=1024")
    vals, idx = run_topk(x, 1024)
    check_exact(x, 1024, "u32", vals, idx, "config small")
    kth = to_np(drt.kth_select(dev(x), 1024))
    assert int(kth[0]) == int(oracle.kth_value(x, 1024, "u32"))


@pytest.mark.parametrize("kind", KINDS)
def test_sizes_and_k(kind):
    for n in (1, 3, 64, 1000, 8192, 8193, 65537, 300007, (1 << 20) + 13):
        x, dt = synth.keys(kind, n, 1000 + n)
        for k in ks_for(n):
            say(kind, "n", n, "k", k)
            vals, idx = run_topk(x, k)
            check_exact(x, k, dt, vals, idx, f"{kind} n={n} k={k}")


@pytest.mark.parametrize("kind", KINDS)
def test_alpha_beta_invariance(kind):
    n = (1 << 18) + 77
    x, dt = synth.keys(kind, n, 7)
    for k in (1, 100, 5000):
        want = oracle.topk_reference(x, k, dt)
        for alpha in (0, 1, 2, 3, 5, 7, 8, 9, 12):
            for beta in (1, 2, 4, 8):
                say(kind, "k", k, "alpha", alpha, "beta", beta)
                vals, idx = run_topk(x, k, alpha=alpha, beta=beta, mode=1)
                assert (idx.view(np.uint32) == want[1]).all(), (kind, k, alpha, beta)
                assert (vals.view(np.uint32) == want[0].view(np.uint32)).all()


@pytest.mark.parametrize("kind", ["uniform_u32", "normal_f32", "heavydup_u32", "sorted_f32"])
def test_delegate_vector_stage(kind):
    for n in (1000, (1 << 16) + 5):
        x, dt = synth.keys(kind, n, 11)
        for alpha in (0, 1, 2, 4, 7, 8, 10):
            for beta in (1, 2, 4, 8):
                say("delegates", kind, n, alpha, beta)
                dk, di = drt.delegates(dev(x), alpha, beta)
                torch.cuda.synchronize()
                got_i = to_np(di).view(np.uint32).astype(np.int64)
                _, want_i = stages.delegates(x, dt, alpha, beta)
                assert (got_i == want_i).all(), (kind, n, alpha, beta)
                real = want_i != oracle.INVALID_INDEX
                gk = to_np(dk).view(np.uint32)
                assert (gk[real] == x.view(np.uint32)[want_i[real]]).all()


@pytest.mark.parametrize("kind", KINDS)
def test_candidate_stage(kind):
    """Survivors of the filter.  The one-kernel-per-step tail uses the exact
    k-th delegate t and must keep exactly the oracle's candidate set; the
    default tail uses a key t' <= t and must keep exactly {i : key[i] >= t'},
    a superset of the oracle's set."""
    n = (1 << 17) + 3
    x, dt = synth.keys(kind, n, 12)
    rk = oracle.rank_key(x, dt)
    for alpha, beta, k in [(4, 1, 50), (6, 2, 500), (8, 1, 3000), (9, 4, 3000), (5, 8, 64), (2, 1, 7)]:
        _, _, info = stages.method_topk(x, k, dt, alpha, beta)
        say("candidates", kind, alpha, beta, k, "variant 1")
        got, _ = drt.candidates(dev(x), k, alpha, beta, variant=1)
        got = np.sort(to_np(got).view(np.uint32).astype(np.int64))
        assert (got == info["candidates"]).all(), (kind, alpha, beta, k, got.size, info["candidates"].size)
        say("candidates", kind, alpha, beta, k, "variant 0")
        got, (tbits, tpos) = drt.candidates(dev(x), k, alpha, beta, variant=0)
        got = np.sort(to_np(got).view(np.uint32).astype(np.int64))
        tv = oracle.rank_key(np.array([tbits], dtype=np.uint32).view(x.dtype), dt)[0]
        pos = np.arange(n)
        want = np.flatnonzero((rk > tv) | ((rk == tv) & (pos <= tpos)))
        assert (got == want).all(), (kind, alpha, beta, k, got.size, want.size)
        assert np.isin(info["candidates"], got).all()
        if info["t"] is not None:  # Rule 2: the threshold ranks no higher than the k-th delegate
            assert tv < info["t"][0] or (tv == info["t"][0] and tpos >= info["t"][1])


@pytest.mark.parametrize("kind", KINDS + ["dup4_u32"])
def test_survivor_sort_routes(kind):
    """Survivor counts from about 600 to 9000, sorted by one workgroup (bucket
    rank by the top bits, or the bitonic network when keys crowd a bin: the
    16-value heavy-duplicate input), and beyond, sorted in bucket groups by
    many workgroups.  dup4_u32 holds each value about 4 times: bins of tied
    keys whose order comes from the positions alone."""
    n = (1 << 20) + 9
    if kind == "dup4_u32":
        x, dt = synth.heavy_dup_u32(n, 4321, distinct=1 << 18), "u32"
    else:
        x, dt = synth.keys(kind, n, 4321)
    for k, alpha, beta in [(600, None, None), (1100, None, None), (2100, None, None), (4096, None, None),
                           (4096, 7, 1), (5000, 6, 1), (7000, 5, 1), (8192, None, None), (30000, None, None)]:
        say("survivor sort", kind, k, alpha, beta)
        vals, idx = run_topk(x, k, alpha=alpha, beta=beta, mode=1)
        check_exact(x, k, dt, vals, idx, f"{kind} k={k} alpha={alpha} beta={beta}")


def test_many_survivors_scatter():
    """Millions of survivors (sorted input, short subranges, small beta): the
    bucket scatter takes claims of 16 or 32 survivors per thread, and at
    beta = 8 the qualify phase reads whole delegate lists as vectors."""
    n = (1 << 23) + 5
    x = synth.sorted_normal_f32(n, 4242)
    for k, alpha, beta in [(4096, 10, 1), (2500, 10, 1), (16384, 11, 8), (3000, 9, 4)]:
        say("many survivors", n, k, alpha, beta)
        vals, idx, st = drt.topk_select(dev(x), k, alpha=alpha, beta=beta, mode=1, stats=True, check=True)
        torch.cuda.synchronize()
        assert beta > 1 or st.candidates >= 1 << 21, (k, alpha, beta, st.candidates)
        check_exact(x, k, "f32", to_np(vals), to_np(idx), f"sorted n={n} k={k} alpha={alpha} beta={beta}")


@pytest.mark.parametrize("kind", KINDS)
def test_tail_variants_agree(kind):
    """The cooperative tail kernel and the one-kernel-per-step tail give identical output."""
    for n, k, alpha, beta in [((1 << 20) + 9, 1, None, None), ((1 << 20) + 9, 1024, None, None),
                              ((1 << 21) + 1, 20000, None, None), ((1 << 20) + 9, 3000, 8, 1),
                              ((1 << 20) + 9, 3000, 6, 4), (300000, 150, 2, 8)]:
        x, dt = synth.keys(kind, n, 77)
        want = oracle.topk_reference(x, k, dt)
        for variant in (0, 1):
            say(kind, n, k, alpha, beta, "variant", variant)
            vals, idx = run_topk(x, k, alpha=alpha, beta=beta, mode=1, variant=variant)
            assert (idx.view(np.uint32) == want[1]).all(), (kind, n, k, alpha, beta, variant)
            assert (vals.view(np.uint32) == want[0].view(np.uint32)).all()


def test_plain_radix_mode():
    for kind in ("uniform_u32", "normal_f32", "heavydup_u32"):
        for n, k in [(5000, 4999), (100000, 17), (100000, 9000), (300001, 150000)]:
            x, dt = synth.keys(kind, n, 5)
            say("plain radix", kind, n, k)
            vals, idx = run_topk(x, k, mode=2)
            check_exact(x, k, dt, vals, idx, f"plain {kind} {n} {k}")


def test_float_specials():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(50000).astype(np.float32)
    specials = np.array([0x7FC00000, 0xFFC00000, 0x7F800000, 0xFF800000, 0x80000000, 0x00000000,
                         0x00000001, 0x80000001, 0x7F7FFFFF, 0xFF7FFFFF, 0x7FFFFFFF, 0xFFFFFFFF],
                        dtype=np.uint32).view(np.float32)
    pos = rng.integers(0, x.shape[0], size=600)
    x[pos] = specials[rng.integers(0, specials.shape[0], size=600)]
    for k in (1, 5, 300, 2000, 50000):
        say("float specials k", k)
        vals, idx = run_topk(x, k)
        check_exact(x, k, "f32", vals, idx, f"specials k={k}")
        vals, idx = run_topk(x, k, alpha=4, beta=2, mode=1)
        check_exact(x, k, "f32", vals, idx, f"specials delegates k={k}")


def test_unaligned_input():
    x = synth.uniform_u32((1 << 20) + 3, 21)
    t = dev(x)
    for off in (1, 2, 3):
        sub = t[off:]
        say("unaligned offset", off)
        vals, idx = drt.topk_select(sub, 777)
        check_exact(x[off:], 777, "u32", to_np(vals), to_np(idx), f"offset {off}")


def test_side_stream_and_repeat():
    x = synth.normal_f32((1 << 21) + 5, 31)
    t = dev(x)
    s = torch.cuda.Stream()
    want = oracle.topk_reference(x, 4096, "f32")
    for rep in range(3):
        say("side stream rep", rep)
        with torch.cuda.stream(s):
            vals, idx = drt.topk_select(t, 4096, stream=s)
        s.synchronize()
        assert (to_np(idx).view(np.uint32) == want[1]).all()


def test_kth_select_matches():
    for kind in KINDS:
        for n, k in [(100, 37), (70000, 1), (70000, 9999), (300001, 1), ((1 << 20) + 1, 1), ((1 << 20) + 1, 20000)]:
            x, dt = synth.keys(kind, n, 41)
            say("kth", kind, n, k)
            got = to_np(drt.kth_select(dev(x), k))[0]
            assert got.view(np.uint32) == np.asarray(oracle.kth_value(x, k, dt)).view(np.uint32)


def test_batched_equals_single():
    probs, hosts = [], []
    for i in range(24):
        n = int(synth.log_uniform_int(1, 10, 18, 500 + i)[0])
        kind = "uniform_u32" if i % 2 == 0 else "normal_f32"
        x, dt = synth.keys(kind, n, 600 + i)
        k = 1 + int(synth.unit_uniform(1, 700 + i)[0] * min(n, 2048))
        probs.append((dev(x), k))
        hosts.append((x, dt, k))
    say("batched 24")
    outs = drt.topk_select_batched(probs)
    torch.cuda.synchronize()
    for (x, dt, k), (v, ix, kth) in zip(hosts, outs):
        check_exact(x, k, dt, to_np(v), to_np(ix), "batched")
        assert to_np(kth).view(np.uint32)[0] == to_np(v).view(np.uint32)[k - 1]


def test_errors_on_gpu():
    t = dev(synth.uniform_u32(100, 1))
    with pytest.raises(drt.DrTopkError):
        drt.topk_select(t, 0)
    with pytest.raises(drt.DrTopkError):
        drt.topk_select(t, 101)
    with pytest.raises(ValueError):  # 2-byte elements
        drt.topk_select(t.to(torch.float16), 3)
    with pytest.raises(KeyError):  # not a key type
        drt.topk_select(t, 3, dtype="u16")
    with pytest.raises(ValueError):
        drt.topk_select(t.cpu(), 3)
    # 64-bit keys at an address that is not 8-byte aligned: refused before any work
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    assert drt.lib().topk_select(ctypes.c_void_p(t.data_ptr() + 4), 25, 3, drt.U64, ctypes.c_void_p(out.data_ptr()),
                                 None, None) == 1


# ---------------------------------------------------------------------------
# full sizes, planner's launch configuration (the one bench.py times)

@pytest.fixture(scope="module")
def full_u32():
    return synth.uniform_u32(1 << 30, synth.DEFAULT_SEED)


@pytest.fixture(scope="module")
def full_f32():
    return synth.normal_f32(1 << 30, synth.DEFAULT_SEED)


def _full_case(x, dt, ks):
    t = dev(x)
    full = oracle.rank_key(x, dt)
    for k in ks:
        say("full size", dt, "k", k)
        vals, idx, st = drt.topk_select(t, k, stats=True, check=True)
        say("  alpha", st.alpha, "beta", st.beta, "scanned", st.scanned, "candidates", st.candidates)
        check_invariants_fast(x, full, k, dt, to_np(vals), to_np(idx))
        say("full size kth_select", dt, "k", k)
        check_kth_fast(x, full, k, drt.kth_select(t, k, check=True), to_np(vals))
    del t
    torch.cuda.empty_cache()


def check_kth_fast(x, full, k, got, vals=None):
    """kth_select's value is the k-th largest: fewer than k keys rank above it and at
    least k at or above it (rank keys from the oracle's order); it is bit-identical to
    slot k-1 of the (invariant-checked) top-k output when one is given."""
    g = to_np(got).reshape(-1)[:1].view(x.dtype)
    kv = oracle.rank_key(g, "f32" if x.dtype == np.float32 else "u32")[0]
    greater = int(np.count_nonzero(full > kv))
    assert greater < k <= greater + int(np.count_nonzero(full == kv)), (k, greater)
    if vals is not None:
        assert g.view(np.uint32)[0] == vals.view(np.uint32)[k - 1]


def check_invariants_fast(x, full, k, dt, vals, idx):
    gi = idx.view(np.uint32).astype(np.int64)
    assert np.unique(gi).shape[0] == k
    assert (x.view(np.uint32)[gi] == vals.view(np.uint32)).all()
    rk = full[gi]
    assert ((rk[:-1] > rk[1:]) | ((rk[:-1] == rk[1:]) & (gi[:-1] < gi[1:]))).all()
    kth = rk[-1]
    greater = int(np.count_nonzero(full > kth))
    eq = np.flatnonzero(full == kth)
    assert greater < k <= greater + eq.shape[0]
    tied = np.sort(gi[rk == kth])
    assert tied.shape[0] == k - greater and (tied == eq[: k - greater]).all()


def test_full_size_uniform_u32(full_u32):
    _full_case(full_u32, "u32", (1, 1024, 131072))


def test_full_size_normal_f32(full_f32):
    _full_case(full_f32, "f32", (1, 1024, 131072))


def test_full_size_adversarial():
    x = synth.sorted_normal_f32(1 << 29, synth.DEFAULT_SEED)
    t = dev(x)
    full = oracle.rank_key(x, "f32")
    for beta in (1, 2, 4, 8):
        say("sorted 2^29 k=16384 beta", beta)
        vals, idx, st = drt.topk_select(t, 16384, beta=beta, stats=True, check=True)
        say("  alpha", st.alpha, "scanned", st.scanned, "candidates", st.candidates)
        check_invariants_fast(x, full, 16384, "f32", to_np(vals), to_np(idx))
    say("sorted 2^29 kth_select k=16384 and k=1")
    check_kth_fast(x, full, 16384, drt.kth_select(t, 16384, check=True), to_np(vals))
    check_kth_fast(x, full, 1, drt.kth_select(t, 1, check=True))
    del t, x, full
    h = synth.heavy_dup_u32(1 << 29, synth.DEFAULT_SEED)
    th = dev(h)
    fullh = oracle.rank_key(h, "u32")
    say("heavy-dup 2^29 k=16384")
    vals, idx, st = drt.topk_select(th, 16384, stats=True, check=True)
    say("  alpha", st.alpha, "beta", st.beta, "scanned", st.scanned, "candidates", st.candidates)
    check_invariants_fast(h, fullh, 16384, "u32", to_np(vals), to_np(idx))
    say("heavy-dup 2^29 kth_select k=16384")
    check_kth_fast(h, fullh, 16384, drt.kth_select(th, 16384, check=True), to_np(vals))
    # closed form: the lowest 16384 positions holding 15
    assert (to_np(idx).view(np.uint32) == np.flatnonzero(h == 15)[:16384]).all()


def test_read_probe_reads_every_key():
    """The bandwidth probe reads keys[0 .. n - n mod 2^20) once: its maximum
    equals the maximum of those keys."""
    x = synth.uniform_u32((1 << 21) + 7, 61)
    x[12345] = 0xFFFFFFF0  # a planted maximum inside the probed range
    x[(1 << 21) + 3] = 0xFFFFFFFF  # beyond it: not read
    out = drt.read_probe(dev(x))
    torch.cuda.synchronize()
    assert int(to_np(out).view(np.uint32)[0]) == int(x[: 1 << 21].max()) == 0xFFFFFFF0


@pytest.mark.parametrize("kind", ["uniform_u32", "sorted_f32"])
def test_grouped_lane_delegates(kind):
    """beta >= 2 with subranges of 2^9..2^11 keys and large chunks: groups of
    lanes own subranges (n = 2^24 + 5 so whole groups fit each wave's range;
    the ragged tail takes the masked path).  Delegate vector and output exact."""
    n = (1 << 24) + 5
    x, dt = synth.keys(kind, n, 404)
    want = {k: oracle.topk_reference(x, k, dt) for k in (1, 5000)}
    for alpha in (9, 10, 11):
        for beta in (2, 4):
            say("grouped delegates", kind, alpha, beta)
            dk, di = drt.delegates(dev(x), alpha, beta)
            torch.cuda.synchronize()
            got_i = to_np(di).view(np.uint32).astype(np.int64)
            _, want_i = stages.delegates(x, dt, alpha, beta)
            assert (got_i == want_i).all(), (kind, alpha, beta)
            for k, (wv, wi) in want.items():
                vals, idx = run_topk(x, k, alpha=alpha, beta=beta, mode=1)
                assert (idx.view(np.uint32) == wi).all(), (kind, alpha, beta, k)
                assert (vals.view(np.uint32) == wv.view(np.uint32)).all()

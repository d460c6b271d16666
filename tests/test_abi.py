"""The C-ABI library on the CPU: it loads, exports every declared function,
plans without a device, and rejects bad arguments before touching the GPU."""
import ctypes
import subprocess

import pytest

import paper_2109_08219_amd as drt


def test_exports_every_declared_symbol():
    names = drt.declared_functions()
    assert {"topk_select", "kth_select", "topk_select_batched"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", drt.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = drt.lib()
    for n in names:
        assert hasattr(L, n)


def test_status_strings_and_version():
    assert drt.status_string(0) == "ok"
    assert drt.status_string(1) == "invalid argument"
    assert drt.status_string(99) == "unknown status"
    assert "gfx950" in drt.version()


@pytest.fixture
def no_tuning():
    saved = drt.tune_get()
    drt.tune_set([])
    yield
    drt.tune_set(saved)


def test_planner(no_tuning):
    # Rule 4 with const = 3, rounded down, for the delegate method; on inputs of
    # 2^24 keys and more beta = 1 takes one more, at most 13 (measured)
    assert drt.plan(2 ** 30, 1) == drt.Plan(1, 13, 1)  # Rule 4: 16
    assert drt.plan(2 ** 30, 1024) == drt.Plan(1, 12, 1)  # Rule 4: 11
    assert drt.plan(2 ** 20, 1024) == drt.Plan(1, 6, 1)  # Rule 4 as is below 2^24
    p = drt.plan(2 ** 30, 131072)
    assert p.mode == 1 and p.beta == 2 and p.alpha == 10  # beta = 2 shifts Rule 4's alpha by 2
    assert drt.plan(2 ** 22, 2 ** 14) == drt.Plan(1, 5, 1)  # large k, n < 2^25: beta = 1, Rule 4
    assert drt.plan(2 ** 25, 2 ** 14).beta == 2
    # small inputs and large k/n fall back to a plain radix select
    assert drt.plan(4096, 7).mode == 3  # one workgroup (n <= 2^16, k <= 2048)
    assert drt.plan(1 << 16, 2048).mode == 3 and drt.plan((1 << 16) + 1, 2048).mode == 1
    assert drt.plan(4096, 2049).mode == 2
    assert drt.plan(10 ** 6, 10 ** 5).mode == 2


@pytest.mark.parametrize("n,k,dtype", [(0, 1, 0), (10, 0, 0), (10, 11, 0), (2 ** 32, 1, 0), (10, 1, 7)])
def test_argument_errors_without_gpu(n, k, dtype):
    L = drt.lib()
    dummy = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    out = ctypes.c_void_p(32)
    assert L.topk_select(dummy, n, k, dtype, out, None, None) == 1
    assert L.kth_select(dummy, n, k, dtype, out, None) == 1


def test_dtype_codes_without_gpu():
    """int32 keys and the k-smallest flag are valid with every key type; other codes are not."""
    L = drt.lib()
    o = drt.Options()
    for code in (0, 1, 2, 3, 4, 5, 0x100, 0x101, 0x102, 0x103, 0x104, 0x105):
        assert L.drtopk_plan(1 << 20, 100, code, ctypes.byref(o)) == 0, code
    for code in (6, 7, 0x106, 0x200, 0x300, -1):
        assert L.drtopk_plan(1 << 20, 100, code, ctypes.byref(o)) == 1, code
    assert drt.plan(1 << 20, 100, "i32-min") == drt.plan(1 << 20, 100, "u32")
    assert drt.footprint(1 << 24, 1000, "f32-min") == drt.footprint(1 << 24, 1000, "f32")


def test_wide_keys_without_gpu():
    """64-bit keys: planned with one delegate per subrange of at least 128 keys or the
    plain radix select; 8-byte alignment required; beta > 1, the delegate and
    candidate stage calls and host streaming refused before any device work."""
    L = drt.lib()
    o = drt.Options()
    for code in (drt.U64, drt.I64, drt.F64, drt.F64 | drt.SMALLEST):
        assert L.drtopk_plan(1 << 28, 1024, code, ctypes.byref(o)) == 0
        assert (o.mode, o.beta) == (1, 1) and 7 <= o.alpha <= 13, (o.mode, o.alpha, o.beta)
        assert L.drtopk_plan(1 << 20, 100000, code, ctypes.byref(o)) == 0 and o.mode == 2  # k > n/16
        assert L.drtopk_plan(5000, 10, code, ctypes.byref(o)) == 0 and o.mode == 2  # small input
    d16, d12, out = ctypes.c_void_p(16), ctypes.c_void_p(12), ctypes.c_void_p(32)
    assert L.topk_select(d12, 1000, 5, drt.U64, out, None, None) == 1  # keys not 8-byte aligned
    assert L.kth_select(d12, 1000, 5, drt.F64, out, None) == 1
    opt = drt.Options(-1, 2, 1, 0)
    assert L.topk_select_ex(d16, 1 << 20, 100, drt.I64, out, None, ctypes.byref(opt), None, None) == 4  # beta 2
    opt = drt.Options(5, 1, 1, 0)
    assert L.topk_select_ex(d16, 1 << 20, 100, drt.I64, out, None, ctypes.byref(opt), None, None) == 1  # alpha < 7
    opt = drt.Options(-1, 0, 3, 0)
    assert L.topk_select_ex(d16, 1 << 12, 100, drt.I64, out, None, ctypes.byref(opt), None, None) == 4  # one workgroup
    assert L.drtopk_delegates(d16, 1 << 20, drt.U64, 8, 1, out, out, None) == 4
    host = (ctypes.c_uint64 * 16)()
    assert L.topk_select_host(host, 16, 1, drt.U64, 0, out, None, None) == 4
    # footprint: 8-byte keys and values, 4-byte positions, plus the workspace
    f64 = drt.footprint(1 << 24, 1000, "f64")
    assert f64 > 8 * (1 << 24) + 12 * 1000
    assert drt.footprint(1 << 24, 1000, "u64") == f64


def test_payload_arguments_without_gpu():
    L = drt.lib()
    d = ctypes.c_void_p(16)
    out = ctypes.c_void_p(32)
    assert L.topk_select_payload(d, 100, 5, 0, None, 4, out, None, out, None) == 1  # no payload
    assert L.topk_select_payload(d, 100, 5, 0, d, 2, out, None, out, None) == 1  # 2-byte payload
    assert L.topk_select_payload(d, 100, 5, 0, d, 8, out, None, None, None) == 1  # no payload output
    assert L.topk_select_payload(d, 100, 101, 0, d, 8, out, None, out, None) == 1  # k > n
    assert L.topk_select_payload(d, 100, 5, 0, d, 8, None, None, out, None) == 1  # no value output


def test_noalloc_arguments_without_gpu():
    L = drt.lib()
    d = ctypes.c_void_p(16)
    out = ctypes.c_void_p(32)
    assert L.topk_select_noalloc(None, 100, 5, 0, out, None, None) == 1  # no input
    assert L.topk_select_noalloc(d, 100, 5, 0, None, None, None) == 1  # no output
    assert L.topk_select_noalloc(d, 100, 101, 0, out, None, None) == 1  # k > n
    assert L.topk_select_noalloc(d, 100, 5, 3 | 0x200, out, None, None) == 1  # not a key type
    # a workspace beyond the fixed 128 MiB is refused before any device work
    assert L.topk_select_noalloc(d, 1 << 30, 131072, 0, out, None, None) == 5
    assert L.topk_select_noalloc(d, 1 << 30, 2048, 1, out, None, None) == 5
    assert drt.status_string(5).startswith("workspace exceeds")


def test_host_stream_arguments_without_gpu():
    L = drt.lib()
    host = (ctypes.c_uint32 * 16)()
    out = ctypes.c_void_p(32)
    assert L.topk_select_host(None, 16, 1, 0, 0, out, None, None) == 1  # no input
    assert L.topk_select_host(host, 16, 1, 0, 0, None, None, None) == 1  # no output
    assert L.topk_select_host(host, 16, 17, 0, 0, out, None, None) == 1  # k > n
    assert L.topk_select_host(host, 16, 1, 0, 17, out, None, None) == 1  # chunk > n
    assert L.topk_select_host(host, 16, 1, 6, 0, out, None, None) == 1  # not a key type


def test_null_pointers_rejected():
    L = drt.lib()
    assert L.topk_select(None, 10, 1, 0, ctypes.c_void_p(32), None, None) == 1
    assert L.topk_select(ctypes.c_void_p(16), 10, 1, 0, None, None, None) == 1
    assert L.kth_select(ctypes.c_void_p(16), 10, 1, 0, None, None) == 1
    assert L.drtopk_plan(10, 1, 0, None) == 1
    assert L.drtopk_delegates(ctypes.c_void_p(16), 10, 0, 30, 1, ctypes.c_void_p(32), ctypes.c_void_p(48), None) == 1
    assert L.drtopk_delegates(ctypes.c_void_p(16), 10, 0, 3, 3, ctypes.c_void_p(32), ctypes.c_void_p(48), None) == 1


@pytest.mark.parametrize("alpha,beta,mode", [(25, 1, 1), (3, 3, 1), (3, 1, 4), (3, 1, -1)])
def test_explicit_options_validated_without_gpu(alpha, beta, mode):
    L = drt.lib()
    o = drt.Options(alpha, beta, mode, 0)
    assert L.topk_select_ex(ctypes.c_void_p(16), 1 << 20, 5, 0, ctypes.c_void_p(32), None, ctypes.byref(o),
                            None, None) == 1


def test_batched_validates_every_problem_first():
    L = drt.lib()
    probs = (drt.Problem * 2)()
    probs[0] = drt.Problem(16, 10, 1, 0, 32, 0, 0)
    probs[1] = drt.Problem(16, 10, 11, 0, 32, 0, 0)  # k > n
    assert L.topk_select_batched(probs, 2, None) == 1
    assert L.topk_select_batched(None, 1, None) == 1
    assert L.topk_select_batched(None, 0, None) == 0


def test_tune_table_roundtrip_and_validation():
    saved = drt.tune_get()
    try:
        drt.tune_set([])
        assert drt.tune_get() == []
        entries = [(drt.FORM_SINGLE, 30, 10, 12, 1), (drt.FORM_BATCHED, 16, 5, 9, 1)]
        drt.tune_set(entries)
        assert drt.tune_get() == entries
        # form-0 entries steer the planner, explicit options aside
        assert drt.plan(2 ** 30, 1024) == drt.Plan(1, 12, 1)
        assert drt.plan(2 ** 30, 2047) == drt.Plan(1, 12, 1)  # same floor(log2 k)
        assert drt.plan(2 ** 30, 2048) == drt.Plan(1, 12, 1)  # no entry: Rule 4 (11) + 1
        L = drt.lib()
        for bad in [(2, 16, 5, 9, 1), (0, 16, 5, 25, 1), (0, 16, 5, 9, 3), (0, -1, 5, 9, 1), (1, 16, 32, 9, 1)]:
            arr = (drt.Tune * 1)(drt.Tune(*bad))
            assert L.drtopk_tune_set(arr, 1) == 1, bad
        assert drt.tune_get() == entries  # a rejected table leaves the old one
        assert L.drtopk_tune_set(None, 1) == 1
        assert L.drtopk_tune_get(None, 0, None) == 1
    finally:
        drt.tune_set(saved)


def test_batched_routes_without_gpu():
    saved = drt.tune_get()
    try:
        drt.tune_set([])
        assert drt.batched_route(1, 1) == (1, 0)
        assert drt.batched_route(4096, 2048) == (1, 0)
        for n in (4097, 8193, 65541, 1 << 20, 1 << 22):
            for k in (1, 7, 1024, 2048):
                r, a = drt.batched_route(n, k)
                if -(-n // 4) <= k:  # even 4-key subranges give no more than k delegates
                    assert (r, a) == (3, 0), (n, k, r, a)
                    continue
                S = -(-n // (1 << a))
                # one workgroup's LDS holds the delegate vector; problems that may be split
                # across workgroups (n > 2^16) keep it in global memory, up to 32768
                # entries, with subranges of at least 16 keys
                if n > (1 << 16):
                    assert r == 2 and 4 <= a <= 24 and k < S <= 32768, (n, k, r, a)
                else:
                    assert r == 2 and 2 <= a <= 24 and k < S <= 4096, (n, k, r, a)
        assert drt.batched_route(1 << 20, 1) == (2, 11)  # Rule 4: floor((20 - 0 + 3) / 2)
        assert drt.batched_route(1 << 20, 1024) == (2, 6)  # Rule 4: floor((20 - 10 + 3) / 2)
        assert drt.batched_route(1 << 22, 2048) == (2, 7)  # Rule 4: floor((22 - 11 + 3) / 2), S = 32768
        assert drt.batched_route((1 << 22) + 1, 1) == (0, 0)
        assert drt.batched_route(1 << 20, 2049) == (0, 0)
        drt.tune_set([(drt.FORM_BATCHED, 16, 2, 3, 1)])
        assert drt.batched_route(1 << 16, 5) == (2, 4)  # raised until S <= 4096
        drt.tune_set([(drt.FORM_BATCHED, 16, 10, 16, 1)])
        r, a = drt.batched_route(1 << 16, 1024)
        assert r == 2 and -(-(1 << 16) // (1 << a)) > 1024  # lowered until S > k
        # beta 2 from the table: the delegate vector holds 2S entries, within the same bounds
        for lg_n, lg_k in ((16, 5), (20, 10), (22, 11), (13, 0)):
            n, k = 1 << lg_n, 1 << lg_k
            drt.tune_set([(drt.FORM_BATCHED, lg_n, lg_k, 6, 2)])
            r, a, b = drt.batched_plan(n, k)
            E = 2 * -(-n // (1 << a))
            assert r == 2 and b == 2 and k < E <= (32768 if n > (1 << 18) else 4096), (lg_n, lg_k, a, b)
        drt.tune_set([(drt.FORM_BATCHED, 20, 10, 6, 4)])  # only 1 and 2 run in the workgroup
        assert drt.batched_plan(1 << 20, 1024)[2] == 1
        drt.tune_set([(drt.FORM_BATCHED, 20, 10, 0, 2)])  # alpha 0: radix select, no delegates
        assert drt.batched_plan(1 << 20, 1024) == (3, 0, 1)
        drt.tune_set([])
        assert drt.batched_plan(1 << 20, 1024) == (2, 6, 1)
        L = drt.lib()
        r, al, be = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert L.drtopk_batched_alpha(0, 1, ctypes.byref(r), ctypes.byref(al), None) == 1
        assert L.drtopk_batched_alpha(10, 11, ctypes.byref(r), ctypes.byref(al), None) == 1
        assert L.drtopk_batched_alpha(10, 1, None, ctypes.byref(al), None) == 1
        assert L.drtopk_batched_alpha(10, 1, ctypes.byref(r), ctypes.byref(al), ctypes.byref(be)) == 0
        assert (r.value, al.value, be.value) == (1, 0, 1)
    finally:
        drt.tune_set(saved)


def test_server_and_footprint_arguments_without_gpu():
    L = drt.lib()
    h = ctypes.c_void_p()
    for bad in [(0, 0, 1, 0), (0, 1, 0, 0), (0, 1, 17, 0), (0, 1, 1, 2)]:
        cfg = drt.ServerConfig(bad[0], bad[1], bad[2], bad[3], 0)
        assert L.drtopk_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1, bad
    assert L.drtopk_server_create(None, ctypes.byref(h)) == 1
    t = ctypes.c_uint64()
    p = drt.Problem(16, 10, 1, 0, 32, 0, 0)
    assert L.drtopk_server_submit(None, ctypes.byref(p), ctypes.byref(t)) == 1
    assert L.drtopk_server_wait(None, 0, None) == 1
    assert L.drtopk_server_drain(None) == 1
    assert L.drtopk_server_destroy(None) == 1
    # footprint: input + outputs + workspace of the route
    # (a batched problem: its 64-byte descriptor plus work item and arrival counter)
    assert drt.footprint(1000, 10) == 4000 + 84 + 64 + 16
    # a batched problem split across workgroups also holds its global delegate vector
    r, a = drt.batched_route(1 << 20, 1000)
    assert drt.footprint(1 << 20, 1000) == 4 * (1 << 20) + 8004 + 80 + 4 * 4 + 8 * ((1 << 20) >> a)
    saved = drt.tune_get()
    try:  # beta 2: twice the entries, tiles of half the keys
        drt.tune_set([(drt.FORM_BATCHED, 20, 9, 6, 2)])
        r, a, b = drt.batched_plan(1 << 20, 1000)
        assert (r, a, b) == (2, 6, 2)
        tiles = (1 << 20) >> 17
        assert drt.footprint(1 << 20, 1000) == 4 * (1 << 20) + 8004 + 80 + 4 * tiles + 16 * ((1 << 20) >> a)
    finally:
        drt.tune_set(saved)
    assert drt.footprint(1 << 24, 100) > 4 * (1 << 24) + 804
    b = ctypes.c_uint64()
    assert L.drtopk_footprint(10, 11, 0, ctypes.byref(b)) == 1
    assert L.drtopk_footprint(10, 1, 0, None) == 1


def test_read_probe_arguments_without_gpu():
    L = drt.lib()
    out = ctypes.c_void_p(64)
    assert L.drtopk_read_probe(None, 1 << 20, out, None) == 1
    assert L.drtopk_read_probe(ctypes.c_void_p(16), (1 << 20) - 1, out, None) == 1
    assert L.drtopk_read_probe(ctypes.c_void_p(20), 1 << 20, out, None) == 1  # not 16-byte aligned
    assert L.drtopk_read_probe(ctypes.c_void_p(16), 1 << 20, None, None) == 1

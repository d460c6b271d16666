"""Device check flags reach the caller through the plain C-ABI.

The survivor-capacity testing hook shrinks the delegate method's survivor
buffers below what the input needs, from the host: the kernels then drop the
writes past the cap, raise flag 16 (capacity) and usually 2 (fewer survivors
than k), and every kernel still exits normally.  The flags must arrive through
a plain topk_select / kth_select followed by drtopk_check (no stats), stay
set until checked, and fail every request of a server launch they hit.
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


@pytest.fixture
def capped():
    drt.check()  # nothing left over from earlier tests on this stream
    drt.set_survivor_cap(512)
    try:
        yield
    finally:
        drt.set_survivor_cap(0)


def test_capacity_flag_reaches_plain_topk(capped):
    x = synth.uniform_u32(1 << 20, 5150)
    t = torch.from_numpy(x).cuda()
    say("capped topk_select n=2^20 k=1024")
    assert drt.plan(1 << 20, 1024).mode == 1
    drt.topk_select(t, 1024)  # plain call: returns OK, enqueue only
    with pytest.raises(drt.DrTopkError) as e:
        drt.check()
    assert e.value.flags & 16, e.value.flags
    drt.check()  # the record was cleared by the failing check
    drt.set_survivor_cap(0)
    say("uncapped topk_select")
    vals, idx = drt.topk_select(t, 1024, check=True)
    check_exact(x, 1024, "u32", to_np(vals), to_np(idx), "after the cap is lifted")


def test_flags_are_sticky_until_checked(capped):
    x = synth.normal_f32((1 << 20) + 3, 5151)
    t = torch.from_numpy(x).cuda()
    say("capped kth_select, then clean calls before the check")
    drt.kth_select(t, 2000)
    drt.set_survivor_cap(0)
    for _ in range(3):
        drt.topk_select(t, 10)
    with pytest.raises(drt.DrTopkError) as e:
        drt.check()
    assert e.value.flags & 16
    out = drt.kth_select(t, 2000, check=True)
    assert to_np(out).view(np.uint32)[0] == np.asarray(oracle.kth_value(x, 2000, "f32")).view(np.uint32)


def test_flags_are_per_stream(capped):
    x = synth.uniform_u32(1 << 20, 5152)
    t = torch.from_numpy(x).cuda()
    s = torch.cuda.Stream()
    say("capped call on a side stream")
    with torch.cuda.stream(s):
        drt.topk_select(t, 1024, stream=s)
    drt.check()  # the default stream saw no failure
    with pytest.raises(drt.DrTopkError):
        drt.check(s)


def test_stats_report_flags(capped):
    x = synth.uniform_u32(1 << 20, 5153)
    with pytest.raises(drt.DrTopkError) as e:
        drt.topk_select(torch.from_numpy(x).cuda(), 1024, stats=True)
    assert e.value.flags & 16
    with pytest.raises(drt.DrTopkError):
        drt.check()


def test_server_fails_flagged_launch(capped):
    """A request too large for a workgroup runs the single-problem path on a
    server stream; under the cap its launch is flagged and the request fails,
    while small requests (the workgroup kernel, which the cap does not touch)
    still succeed."""
    big = synth.uniform_u32((1 << 23) + 1, 5154)
    small = synth.uniform_u32(5000, 5155)
    tb, ts = torch.from_numpy(big).cuda(), torch.from_numpy(small).cuda()
    b = drt.Batch([(tb, 1024), (ts, 100)])
    with drt.Server(streams=2, max_batch=4) as srv:
        say("server: capped large request")
        t0 = srv.submit(b, 0)
        with pytest.raises(drt.DrTopkError) as e:
            srv.wait(t0)
        assert e.value.status == 3
        t1 = srv.submit(b, 1)
        srv.wait(t1)
        with pytest.raises(drt.DrTopkError):
            srv.drain()
    check_exact(small, 100, "u32", to_np(b.values(1)), to_np(b.indices(1)), "small request beside a flagged one")

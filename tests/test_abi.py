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


def test_planner():
    # Rule 4 with const = 3, rounded down, for the delegate method
    assert drt.plan(2 ** 30, 1) == drt.Plan(1, 16, 1)
    assert drt.plan(2 ** 30, 1024) == drt.Plan(1, 11, 1)
    assert drt.plan(2 ** 20, 1024) == drt.Plan(1, 6, 1)
    p = drt.plan(2 ** 30, 131072)
    assert p.mode == 1 and p.beta == 2 and p.alpha == 10  # beta = 2 shifts Rule 4's alpha by 2
    # small inputs and large k/n fall back to a plain radix select
    assert drt.plan(4096, 7).mode == 2
    assert drt.plan(10 ** 6, 10 ** 5).mode == 2


@pytest.mark.parametrize("n,k,dtype", [(0, 1, 0), (10, 0, 0), (10, 11, 0), (2 ** 32, 1, 0), (10, 1, 7)])
def test_argument_errors_without_gpu(n, k, dtype):
    L = drt.lib()
    dummy = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    out = ctypes.c_void_p(32)
    assert L.topk_select(dummy, n, k, dtype, out, None, None) == 1
    assert L.kth_select(dummy, n, k, dtype, out, None) == 1


def test_null_pointers_rejected():
    L = drt.lib()
    assert L.topk_select(None, 10, 1, 0, ctypes.c_void_p(32), None, None) == 1
    assert L.topk_select(ctypes.c_void_p(16), 10, 1, 0, None, None, None) == 1
    assert L.kth_select(ctypes.c_void_p(16), 10, 1, 0, None, None) == 1
    assert L.drtopk_plan(10, 1, 0, None) == 1
    assert L.drtopk_delegates(ctypes.c_void_p(16), 10, 0, 30, 1, ctypes.c_void_p(32), ctypes.c_void_p(48), None) == 1
    assert L.drtopk_delegates(ctypes.c_void_p(16), 10, 0, 3, 3, ctypes.c_void_p(32), ctypes.c_void_p(48), None) == 1


def test_batched_validates_every_problem_first():
    L = drt.lib()
    probs = (drt.Problem * 2)()
    probs[0] = drt.Problem(16, 10, 1, 0, 32, 0, 0)
    probs[1] = drt.Problem(16, 10, 11, 0, 32, 0, 0)  # k > n
    assert L.topk_select_batched(probs, 2, None) == 1
    assert L.topk_select_batched(None, 1, None) == 1
    assert L.topk_select_batched(None, 0, None) == 0

"""The oracle against facts outside itself: brute force, closed forms,
library routines, IEEE totalOrder and the paper's worked example."""
import numpy as np
import pytest

import oracle
from oracle import stages
import oracle_pins as pins



def topk_threaded3(values, k, dtype, largest=True):
    """The threaded route with three parts, so tiny inputs still exercise the merge."""
    return oracle.topk_threaded(values, k, dtype, largest, threads=3)


ROUTES = [oracle.topk_sort, oracle.topk_select, oracle.topk_heap, topk_threaded3]


@pytest.mark.parametrize("fn", ROUTES + [oracle.topk_bruteforce], ids=lambda f: f.__name__)
def test_exhaustive_tiny(fn):
    pins.pin_exhaustive_u32(fn, max_len=5 if fn is not oracle.topk_bruteforce else 4)


@pytest.mark.parametrize("fn", ROUTES, ids=lambda f: f.__name__)
def test_closed_forms(fn):
    pins.pin_closed_forms_u32(fn)


@pytest.mark.parametrize("fn", ROUTES + [oracle.topk_bruteforce], ids=lambda f: f.__name__)
def test_float_total_order(fn):
    pins.pin_float_order(fn)


def test_kth():
    pins.pin_kth(oracle.kth_value)


@pytest.mark.parametrize("fn", ROUTES + [oracle.topk_bruteforce], ids=lambda f: f.__name__)
def test_smallest_and_i32(fn):
    pins.pin_smallest_and_i32(fn)


def test_kth_smallest():
    pins.pin_kth_smallest(oracle.kth_value)


@pytest.mark.parametrize("fn", ROUTES + [oracle.topk_bruteforce], ids=lambda f: f.__name__)
def test_wide_keys(fn):
    pins.pin_wide(fn)


def test_kth_wide():
    pins.pin_kth_wide(oracle.kth_value)


@pytest.mark.parametrize("largest", [True, False])
@pytest.mark.parametrize("dtype", ["u32", "f32", "i32", "u64", "i64", "f64"])
def test_routes_agree_random(dtype, largest):
    rng = np.random.default_rng(1)
    for n in (1, 2, 63, 64, 65, 1000, 4097):
        if dtype == "u32":
            v = rng.integers(0, 2 ** 32, size=n, dtype=np.uint32)
            v[rng.integers(0, n, size=n // 4)] = v[0]  # plant ties
        elif dtype == "i32":
            v = rng.integers(-2 ** 31, 2 ** 31, size=n).astype(np.int32)
            v[rng.integers(0, n, size=n // 4)] = v[0]
        elif dtype == "u64":
            v = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.uint64) * np.uint64(2)
            v[rng.integers(0, n, size=n // 4)] = v[0]
        elif dtype == "i64":
            v = rng.integers(-2 ** 63, 2 ** 63 - 1, size=n, dtype=np.int64)
            v[rng.integers(0, n, size=n // 4)] = v[0]
        elif dtype == "f64":
            v = rng.standard_normal(n)
            v[rng.integers(0, n, size=n // 4)] = v[0]
        else:
            v = rng.standard_normal(n).astype(np.float32)
            v[rng.integers(0, n, size=n // 4)] = v[0]
        for k in sorted({1, n, max(1, n // 2), min(n, 17)}):
            a = oracle.topk_sort(v, k, dtype, largest)[1]
            b = oracle.topk_select(v, k, dtype, largest)[1]
            assert (a == b).all()
            if n <= 1000:
                c = oracle.topk_heap(v, k, dtype, largest)[1]
                assert (a == c).all()
            for threads in (2, 5, 16):
                assert (a == oracle.topk_threaded(v, k, dtype, largest, threads=threads)[1]).all()


def test_argument_errors():
    v = np.zeros(4, dtype=np.uint32)
    for k in (0, 5):
        with pytest.raises(ValueError):
            oracle.topk_select(v, k, "u32")
    with pytest.raises(TypeError):
        oracle.topk_select(v.astype(np.int32), 1, "u32")


def test_delegates_bruteforce():
    pins.pin_delegates_bruteforce(stages.delegates)


def test_paper_worked_example():
    pins.pin_paper_example(stages)


@pytest.mark.parametrize("kind", ["heavydup", "allequal", "ascending", "descending"])
def test_threaded_route_ties_across_parts(kind):
    """Ties and runs that straddle part boundaries: the merged answer is the
    definition's (positions of tied keys in ascending order across parts)."""
    n = 10007
    if kind == "heavydup":
        v = np.random.default_rng(3).integers(0, 5, size=n, dtype=np.uint32)
    elif kind == "allequal":
        v = np.full(n, 7, dtype=np.uint32)
    elif kind == "ascending":
        v = np.arange(n, dtype=np.uint32) // 3
    else:
        v = (n - np.arange(n, dtype=np.uint32)) // 3
    for k in (1, 3, 100, 4000, n):
        for threads in (1, 2, 7, 64):
            for largest in (True, False):
                want = oracle.topk_sort(v, k, "u32", largest)[1]
                got = oracle.topk_threaded(v, k, "u32", largest, threads=threads)[1]
                assert (got == want).all(), (kind, k, threads, largest)

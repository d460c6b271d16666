"""Checks that pin the oracle to facts outside itself.

Each ``pin_*`` takes the oracle function(s) under test and raises
AssertionError on disagreement, so the same checks run on the real oracle
(tests/test_oracle_definition.py) and on deliberately broken copies of it
(tests/test_oracle_mutations.py), which must fail at least one pin.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

ALPHABET = np.array([0, 1, 2, 0xFFFFFFFF], dtype=np.uint32)


def load_golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def brute_ranks(values: list, key_of) -> list:
    """Output order by the definition, via Python's own sort on (key desc, position asc)."""
    return sorted(range(len(values)), key=lambda i: (-key_of(values[i]), i))


def pin_exhaustive_u32(topk_fn, max_len: int = 5) -> None:
    """Every u32 array of length 1..max_len over {0, 1, 2, 2^32-1}, every k."""
    for n in range(1, max_len + 1):
        for combo in itertools.product(range(len(ALPHABET)), repeat=n):
            v = ALPHABET[list(combo)]
            want = brute_ranks([int(x) for x in v], int)
            for k in range(1, n + 1):
                vals, idx = topk_fn(v, k, "u32")
                assert list(map(int, idx)) == want[:k], (v.tolist(), k, list(idx), want[:k])
                assert (np.asarray(vals).view(np.uint32) == v[want[:k]]).all()


def pin_closed_forms_u32(topk_fn, seed: int = 7) -> None:
    """Special cases with answers fixed without any ranking code of ours."""
    rng = np.random.default_rng(seed)
    # k = 1: the first position of the maximum (numpy argmax returns the first).
    for n in (1, 2, 17, 1000):
        v = rng.integers(0, 50, size=n, dtype=np.uint32)
        _, idx = topk_fn(v, 1, "u32")
        assert int(idx[0]) == int(np.argmax(v))
    # k = n: a stable descending sort (numpy's stable argsort of the negated keys).
    for n in (1, 5, 300):
        v = rng.integers(0, 20, size=n, dtype=np.uint32)
        _, idx = topk_fn(v, n, "u32")
        assert (np.asarray(idx) == np.argsort(-v.astype(np.int64), kind="stable")).all()
    # all equal: positions 0..k-1.
    v = np.full(64, 99, dtype=np.uint32)
    for k in (1, 7, 64):
        _, idx = topk_fn(v, k, "u32")
        assert list(map(int, idx)) == list(range(k))
    # strictly descending: positions 0..k-1.
    v = np.arange(500, 0, -1).astype(np.uint32)
    _, idx = topk_fn(v, 123, "u32")
    assert list(map(int, idx)) == list(range(123))
    # strictly ascending: the last k positions, reversed.
    v = np.arange(10, 510).astype(np.uint32)
    _, idx = topk_fn(v, 50, "u32")
    assert list(map(int, idx)) == list(range(499, 449, -1))
    # heavy duplicates: walk the distinct values downwards, each in position order.
    v = rng.integers(0, 6, size=400, dtype=np.uint32)
    for k in (1, 30, 250, 400):
        want = []
        for val in sorted(set(v.tolist()), reverse=True):
            want.extend(np.flatnonzero(v == val).tolist())
        _, idx = topk_fn(v, k, "u32")
        assert list(map(int, idx)) == want[:k]
    # value multiset against numpy's sort.
    v = rng.integers(0, 2**32, size=5000, dtype=np.uint32)
    vals, _ = topk_fn(v, 777, "u32")
    assert (np.asarray(vals) == np.sort(v)[::-1][:777]).all()


def f32_chain() -> np.ndarray:
    """Bit patterns in ascending IEEE 754 totalOrder (Section 5.10 of the standard)."""
    pats = [
        0xFFFFFFFF,  # -NaN, largest payload
        0xFFC00001,  # -NaN, quiet, small payload
        0xFF800001,  # -NaN, signalling, smallest payload
        0xFF800000,  # -inf
        0xFF7FFFFF,  # -max finite
        0xBF800000,  # -1
        0x80800000,  # -min normal
        0x807FFFFF,  # -max subnormal
        0x80000001,  # -min subnormal
        0x80000000,  # -0
        0x00000000,  # +0
        0x00000001,  # +min subnormal
        0x007FFFFF,  # +max subnormal
        0x00800000,  # +min normal
        0x3F800000,  # +1
        0x7F7FFFFF,  # +max finite
        0x7F800000,  # +inf
        0x7F800001,  # +NaN, signalling, smallest payload
        0x7FC00000,  # +NaN, quiet
        0x7FFFFFFF,  # +NaN, largest payload
    ]
    return np.array(pats, dtype=np.uint32)


def pin_float_order(topk_fn, seed: int = 11) -> None:
    chain = f32_chain()
    rng = np.random.default_rng(seed)
    perm = rng.permutation(chain.shape[0])
    v = chain[perm].view(np.float32)
    vals, idx = topk_fn(v, chain.shape[0], "f32")
    got = np.asarray(vals).view(np.uint32)
    assert (got == chain[::-1]).all(), [hex(x) for x in got]
    # -0 below +0 regardless of position
    for pair in ([0x80000000, 0x00000000], [0x00000000, 0x80000000]):
        v = np.array(pair, dtype=np.uint32).view(np.float32)
        vals, _ = topk_fn(v, 1, "f32")
        assert int(np.asarray(vals).view(np.uint32)[0]) == 0
    # finite distinct floats: same order as Python's float comparison.
    x = rng.standard_normal(3000).astype(np.float32) * np.float32(1e3)
    x = np.unique(x)
    rng.shuffle(x)
    vals, _ = topk_fn(x, 100, "f32")
    want = sorted((float(a) for a in x), reverse=True)[:100]
    assert [float(a) for a in vals] == want


def pin_kth(kth_fn, seed: int = 5) -> None:
    rng = np.random.default_rng(seed)
    for n in (1, 9, 1000):
        v = rng.integers(0, 30, size=n, dtype=np.uint32)
        for k in sorted({1, n, max(1, n // 3)}):
            assert int(kth_fn(v, k, "u32")) == int(np.sort(v)[::-1][k - 1])


def pin_delegates_bruteforce(delegates_fn, seed: int = 3) -> None:
    """Each delegate row equals Python's sort of the subrange by (key desc, position asc)."""
    rng = np.random.default_rng(seed)
    for n in (1, 5, 16, 37, 64):
        v = rng.integers(0, 5, size=n, dtype=np.uint32)
        for alpha in (0, 1, 2, 3):
            L = 1 << alpha
            for beta in (1, 2, 3):
                dkey, didx = delegates_fn(v, "u32", alpha, beta)
                for s in range(-(-n // L)):
                    pos = list(range(s * L, min(n, (s + 1) * L)))
                    want = sorted(pos, key=lambda i: (-int(v[i]), i))[:beta]
                    got = [int(i) for i in didx[s] if int(i) != 0xFFFFFFFF]
                    assert got == want, (n, alpha, beta, s, got, want)
                    assert [int(x) for x in dkey[s][: len(want)]] == [int(v[i]) for i in want]


def pin_paper_example(stages_mod) -> None:
    """The worked example (Sections 2.2, 4.1-4.3, 5.3) from tests/golden."""
    g = load_golden("paper_example.json")
    V = np.array(g["V"], dtype=np.uint32)
    alpha = g["alpha"]
    bx = g["bucket_example"]
    assert int(V.min()) == bx["min"] and int(V.max()) == bx["max"]
    w = (bx["max"] - bx["min"]) / 4
    assert [bx["min"] + j * w for j in range(5)] == bx["bounds"]
    assert int((V >= bx["bounds"][3]).sum()) == bx["top_bucket_count"]
    for c in g["cases"]:
        beta, k = c["beta"], c["k"]
        dkey, didx = stages_mod.delegates(V, "u32", alpha, beta)
        if "delegate_keys" in c:
            assert dkey.tolist() == c["delegate_keys"], (c["name"], dkey.tolist())
        taken, t = stages_mod.first_topk(dkey, didx, k)
        assert sorted(dkey[taken].tolist(), reverse=True) == c["first_topk_keys"], c["name"]
        assert t[0] == c["threshold_key"], c["name"]
        qual = stages_mod.qualifying(taken, t)
        assert np.flatnonzero(qual).tolist() == c["qualifying_subranges"], c["name"]
        cand = stages_mod.concatenate(V, "u32", alpha, dkey, didx, taken, qual, t)
        assert sorted(V[cand].tolist()) == sorted(c["filtered_concatenation"]), c["name"]
        if "unfiltered_concatenation" in c:
            L = 1 << alpha
            unf = [int(V[i]) for s in np.flatnonzero(qual) for i in range(s * L, (s + 1) * L)]
            assert unf == c["unfiltered_concatenation"]
        vals, _, _ = stages_mod.method_topk(V, k, "u32", alpha, beta)
        assert vals.tolist() == c["topk_values"], c["name"]
    a = g["alpha_rule_instance"]
    assert stages_mod.alpha_rule(2 ** a["log2_n"], 2 ** a["log2_k"], a["const"]) == a["alpha"]


I32_ALPHABET = np.array([-2 ** 31, -1, 0, 1, 2 ** 31 - 1], dtype=np.int32)


def pin_smallest_and_i32(topk_fn, seed: int = 13) -> None:
    """The k smallest (largest=False) and signed int32 keys, against Python's
    own sort, numpy's argmin / stable argsort / sort, and hand-ordered lists."""
    rng = np.random.default_rng(seed)
    # exhaustive tiny arrays, k smallest: Python's sort on (key asc, position asc)
    for n in range(1, 5):
        for combo in itertools.product(range(len(ALPHABET)), repeat=n):
            v = ALPHABET[list(combo)]
            want = sorted(range(n), key=lambda i: (int(v[i]), i))
            for k in range(1, n + 1):
                vals, idx = topk_fn(v, k, "u32", largest=False)
                assert list(map(int, idx)) == want[:k], (v.tolist(), k, list(idx), want[:k])
                assert (np.asarray(vals).view(np.uint32) == v[want[:k]]).all()
    # exhaustive tiny int32 arrays over {-2^31, -1, 0, 1, 2^31-1}, both orders
    for n in range(1, 4):
        for combo in itertools.product(range(len(I32_ALPHABET)), repeat=n):
            v = I32_ALPHABET[list(combo)]
            up = sorted(range(n), key=lambda i: (int(v[i]), i))
            down = sorted(range(n), key=lambda i: (-int(v[i]), i))
            for k in range(1, n + 1):
                assert list(map(int, topk_fn(v, k, "i32", largest=False)[1])) == up[:k]
                assert list(map(int, topk_fn(v, k, "i32")[1])) == down[:k], (v.tolist(), k)
    # k = 1 smallest: numpy argmin (first position of the minimum)
    for n in (1, 2, 17, 1000):
        v = rng.integers(0, 50, size=n, dtype=np.uint32)
        assert int(topk_fn(v, 1, "u32", largest=False)[1][0]) == int(np.argmin(v))
        w = rng.integers(-25, 25, size=n).astype(np.int32)
        assert int(topk_fn(w, 1, "i32", largest=False)[1][0]) == int(np.argmin(w))
        assert int(topk_fn(w, 1, "i32")[1][0]) == int(np.argmax(w))
    # k = n: numpy's stable ascending argsort (and descending via the negation)
    for n in (1, 5, 300):
        v = rng.integers(0, 20, size=n, dtype=np.uint32)
        assert (np.asarray(topk_fn(v, n, "u32", largest=False)[1]) == np.argsort(v, kind="stable")).all()
        w = rng.integers(-10, 10, size=n).astype(np.int32)
        assert (np.asarray(topk_fn(w, n, "i32", largest=False)[1]) == np.argsort(w, kind="stable")).all()
        assert (np.asarray(topk_fn(w, n, "i32")[1]) ==
                np.argsort(-w.astype(np.int64), kind="stable")).all()
        # float32 without NaNs and without -0: numpy's value order is totalOrder there
        f = (rng.integers(-8, 8, size=n) * 0.5 + 0.25).astype(np.float32)
        assert (np.asarray(topk_fn(f, n, "f32", largest=False)[1]) == np.argsort(f, kind="stable")).all()
    # float32 totalOrder upwards: a hand-ordered chain, shuffled
    chain = f32_chain().view(np.float32)
    perm = rng.permutation(chain.shape[0])
    _, idx = topk_fn(chain[perm], chain.shape[0], "f32", largest=False)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    assert list(map(int, idx)) == [int(inv[j]) for j in range(chain.shape[0])]
    # heavy duplicates upwards, each value in position order
    v = rng.integers(0, 6, size=400, dtype=np.uint32)
    for k in (1, 30, 250, 400):
        want = []
        for val in sorted(set(v.tolist())):
            want.extend(np.flatnonzero(v == val).tolist())
        assert list(map(int, topk_fn(v, k, "u32", largest=False)[1])) == want[:k]
    # value multisets against numpy's sort
    v = rng.integers(0, 2 ** 32, size=5000, dtype=np.uint32)
    assert (np.asarray(topk_fn(v, 777, "u32", largest=False)[0]) == np.sort(v)[:777]).all()
    w = rng.integers(-2 ** 31, 2 ** 31, size=5000).astype(np.int32)
    assert (np.asarray(topk_fn(w, 777, "i32")[0]) == np.sort(w)[::-1][:777]).all()


def pin_kth_smallest(kth_fn, seed: int = 17) -> None:
    """k-th smallest (counting multiplicity) = numpy's ascending sort at k-1."""
    rng = np.random.default_rng(seed)
    for n in (1, 9, 1000):
        v = rng.integers(0, 30, size=n, dtype=np.uint32)
        w = rng.integers(-15, 15, size=n).astype(np.int32)
        for k in sorted({1, n, max(1, n // 3)}):
            assert int(kth_fn(v, k, "u32", largest=False)) == int(np.sort(v)[k - 1])
            assert int(kth_fn(w, k, "i32", largest=False)) == int(np.sort(w)[k - 1])
            assert int(kth_fn(w, k, "i32")) == int(np.sort(w)[::-1][k - 1])


U64_ALPHABET = np.array([0, 1, 1 << 63, (1 << 64) - 1], dtype=np.uint64)
I64_ALPHABET = np.array([-(1 << 63), -1, 0, 1, (1 << 63) - 1], dtype=np.int64)


def f64_chain() -> np.ndarray:
    """float64 bit patterns in ascending IEEE 754 totalOrder."""
    pats = [
        0xFFFFFFFFFFFFFFFF,  # -NaN, largest payload
        0xFFF8000000000001,  # -NaN, quiet, small payload
        0xFFF0000000000001,  # -NaN, signalling, smallest payload
        0xFFF0000000000000,  # -inf
        0xFFEFFFFFFFFFFFFF,  # -max finite
        0xBFF0000000000001,  # -(1 + 2^-52)
        0xBFF0000000000000,  # -1
        0x8010000000000000,  # -min normal
        0x800FFFFFFFFFFFFF,  # -max subnormal
        0x8000000000000001,  # -min subnormal
        0x8000000000000000,  # -0
        0x0000000000000000,  # +0
        0x0000000000000001,  # +min subnormal
        0x000FFFFFFFFFFFFF,  # +max subnormal
        0x0010000000000000,  # +min normal
        0x3FF0000000000000,  # +1
        0x3FF0000000000001,  # +(1 + 2^-52): differs from +1 in the lowest bit only
        0x7FEFFFFFFFFFFFFF,  # +max finite
        0x7FF0000000000000,  # +inf
        0x7FF0000000000001,  # +NaN, signalling, smallest payload
        0x7FF8000000000000,  # +NaN, quiet
        0x7FFFFFFFFFFFFFFF,  # +NaN, largest payload
    ]
    return np.array(pats, dtype=np.uint64)


def pin_wide(topk_fn, seed: int = 19) -> None:
    """64-bit keys (uint64, int64, float64), both orders, against Python's own
    sort of Python integers, numpy's argmax / argmin / stable argsort / sort,
    and the hand-ordered float64 totalOrder chain."""
    rng = np.random.default_rng(seed)
    for dt, alphabet, max_len in (("u64", U64_ALPHABET, 4), ("i64", I64_ALPHABET, 3)):
        for n in range(1, max_len + 1):
            for combo in itertools.product(range(len(alphabet)), repeat=n):
                v = alphabet[list(combo)]
                py = [int(x) for x in v]
                up = sorted(range(n), key=lambda i: (py[i], i))
                down = sorted(range(n), key=lambda i: (-py[i], i))
                for k in range(1, n + 1):
                    vals, idx = topk_fn(v, k, dt)
                    assert list(map(int, idx)) == down[:k], (dt, py, k, list(idx))
                    assert (np.asarray(vals).view(np.uint64) == v[down[:k]].view(np.uint64)).all()
                    assert list(map(int, topk_fn(v, k, dt, largest=False)[1])) == up[:k], (dt, py, k)
    # values above 2^53 that differ in their lowest bits (a float64 detour, or
    # the high 32 bits alone, would tie them)
    base = (1 << 60) + (7 << 32)
    v = np.array([base + 1, base, base + 2, base + (1 << 32), base - 1], dtype=np.uint64)
    assert list(map(int, topk_fn(v, 5, "u64")[1])) == [3, 2, 0, 1, 4]
    w = v.astype(np.int64) * -1
    assert list(map(int, topk_fn(w, 5, "i64")[1])) == [4, 1, 0, 2, 3]
    # k = 1: numpy's first argmax / argmin
    for n in (1, 2, 17, 1000):
        u = rng.integers(0, 50, size=n).astype(np.uint64) << np.uint64(58)
        assert int(topk_fn(u, 1, "u64")[1][0]) == int(np.argmax(u))
        assert int(topk_fn(u, 1, "u64", largest=False)[1][0]) == int(np.argmin(u))
        s = rng.integers(-25, 25, size=n).astype(np.int64) << np.int64(50)
        assert int(topk_fn(s, 1, "i64")[1][0]) == int(np.argmax(s))
        assert int(topk_fn(s, 1, "i64", largest=False)[1][0]) == int(np.argmin(s))
        f = rng.integers(-8, 8, size=n) * 0.5 + 0.25
        assert int(topk_fn(f, 1, "f64")[1][0]) == int(np.argmax(f))
        assert int(topk_fn(f, 1, "f64", largest=False)[1][0]) == int(np.argmin(f))
    # k = n, the k smallest: numpy's stable ascending argsort (ties in position order)
    for n in (1, 5, 300):
        u = rng.integers(0, 20, size=n).astype(np.uint64) * np.uint64(0x0F00000000000001)
        assert (np.asarray(topk_fn(u, n, "u64", largest=False)[1]) == np.argsort(u, kind="stable")).all()
        s = rng.integers(-10, 10, size=n).astype(np.int64) * np.int64(0x0300000000000001)
        assert (np.asarray(topk_fn(s, n, "i64", largest=False)[1]) == np.argsort(s, kind="stable")).all()
        f = rng.integers(-8, 8, size=n) * 0.5 + 0.25  # no NaN, no -0: value order is totalOrder
        assert (np.asarray(topk_fn(f, n, "f64", largest=False)[1]) == np.argsort(f, kind="stable")).all()
    # distinct values, largest first: numpy's ascending argsort reversed
    u = rng.permutation(np.arange(1000, dtype=np.uint64) * np.uint64(0x00FF00FF00FF00FF))
    assert (np.asarray(topk_fn(u, 1000, "u64")[1]) == np.argsort(u)[::-1]).all()
    # float64 totalOrder both ways: the hand-ordered chain, shuffled
    chain = f64_chain()
    perm = rng.permutation(chain.shape[0])
    vals, _ = topk_fn(chain[perm].view(np.float64), chain.shape[0], "f64")
    assert (np.asarray(vals).view(np.uint64) == chain[::-1]).all(), [hex(x) for x in np.asarray(vals).view(np.uint64)]
    vals, _ = topk_fn(chain[perm].view(np.float64), chain.shape[0], "f64", largest=False)
    assert (np.asarray(vals).view(np.uint64) == chain).all()
    # value multisets against numpy's sort
    u = rng.integers(0, 2 ** 63, size=5000, dtype=np.int64).view(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=5000).astype(np.uint64)
    assert (np.asarray(topk_fn(u, 777, "u64")[0]) == np.sort(u)[::-1][:777]).all()
    s = rng.integers(-2 ** 63, 2 ** 63 - 1, size=5000, dtype=np.int64)
    assert (np.asarray(topk_fn(s, 777, "i64", largest=False)[0]) == np.sort(s)[:777]).all()
    f = rng.standard_normal(5000) * 1e300
    assert (np.asarray(topk_fn(f, 777, "f64")[0]) == np.sort(f)[::-1][:777]).all()


def pin_kth_wide(kth_fn, seed: int = 23) -> None:
    """k-th largest / smallest of 64-bit keys = numpy's sort at k-1."""
    rng = np.random.default_rng(seed)
    for n in (1, 9, 1000):
        u = rng.integers(0, 30, size=n).astype(np.uint64) << np.uint64(59)
        s = rng.integers(-15, 15, size=n).astype(np.int64) << np.int64(58)
        f = rng.integers(-15, 15, size=n) * 0.125
        for k in sorted({1, n, max(1, n // 3)}):
            assert int(kth_fn(u, k, "u64")) == int(np.sort(u)[::-1][k - 1])
            assert int(kth_fn(u, k, "u64", largest=False)) == int(np.sort(u)[k - 1])
            assert int(kth_fn(s, k, "i64")) == int(np.sort(s)[::-1][k - 1])
            assert int(kth_fn(s, k, "i64", largest=False)) == int(np.sort(s)[k - 1])
            assert float(kth_fn(f, k, "f64")) == float(np.sort(f)[::-1][k - 1])

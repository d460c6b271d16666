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

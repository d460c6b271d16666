"""Exactness checks of GPU results against the oracle.

``check_exact`` compares element by element with the oracle's answer.
``check_invariants`` verifies, at any size, properties that together fix the
answer uniquely (so passing them is exact agreement too):
  I1 k outputs, distinct positions in range;
  I2 out_vals[r] is bit-identical to keys[out_idx[r]];
  I3 outputs strictly ordered by (key desc, position asc);
(largest=False: the k smallest, every "desc" / "above" read in reverse order).
  I4 fewer than k keys rank strictly above the k-th, at least k at or above;
  I5 the k-th value appears k - #{key > kth} times in the output;
  I6 those tied outputs are the lowest positions holding the k-th value.
"""
from __future__ import annotations

import numpy as np

import oracle


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def check_exact(keys: np.ndarray, k: int, dtype: str, got_vals: np.ndarray, got_idx: np.ndarray, tag="",
                largest: bool = True):
    want_vals, want_idx = oracle.topk_reference(keys, k, dtype, largest)
    gi = np.asarray(got_idx).view(np.uint32).astype(np.int64)
    assert gi.shape == (k,), (tag, gi.shape)
    bad = np.flatnonzero(gi != want_idx)
    assert bad.size == 0, f"{tag}: {bad.size} index mismatches, first at slot {bad[0]}: got {gi[bad[0]]} want {want_idx[bad[0]]}"
    gv = oracle.order.bits(got_vals)
    wv = oracle.order.bits(want_vals)
    assert (gv == wv).all(), f"{tag}: values differ"


def check_invariants(keys: np.ndarray, k: int, dtype: str, got_vals: np.ndarray, got_idx: np.ndarray, tag="",
                     largest: bool = True):
    def order_key(v):  # larger ranks first; ~ reverses the order without overflow
        rk = oracle.rank_key(v, dtype)
        return rk if largest else ~rk

    n = keys.shape[0]
    gi = np.asarray(got_idx).view(np.uint32).astype(np.int64)
    gv = oracle.order.bits(got_vals)
    assert gi.shape == (k,), tag
    assert (gi >= 0).all() and (gi < n).all(), f"{tag}: position out of range"
    assert np.unique(gi).shape[0] == k, f"{tag}: repeated positions"  # I1
    kb = oracle.order.bits(keys)
    assert (kb[gi] == gv).all(), f"{tag}: values are not the keys at the positions"  # I2
    rk = order_key(keys[gi])
    ok = (rk[:-1] > rk[1:]) | ((rk[:-1] == rk[1:]) & (gi[:-1] < gi[1:]))
    assert ok.all(), f"{tag}: outputs not in (key desc, position asc) order"  # I3
    kth = rk[-1]
    full = order_key(keys)
    greater = int(np.count_nonzero(full > kth))
    at_least = greater + int(np.count_nonzero(full == kth))
    assert greater < k <= at_least, f"{tag}: k-th value wrong ({greater}, {k}, {at_least})"  # I4
    tied = gi[rk == kth]
    assert tied.shape[0] == k - greater, f"{tag}: tie multiplicity"  # I5
    first = np.flatnonzero(full == kth)[: k - greater]
    assert (np.sort(tied) == first).all(), f"{tag}: tied positions are not the lowest"  # I6

"""Planted mistakes in copies of the oracle must trip at least one pin.

Each mutant is a plausible slip (a wrong sign, a dropped term, an off-by-one,
a reversed tie rule, a transposed operand).  The mutants live here, on the
CPU; the oracle itself is never modified.
"""
import numpy as np
import pytest

import oracle
from oracle import order, stages, topk as T
import oracle_pins as pins


def _key_float_value(values, dtype):
    # mistake: compare floats by value (loses -0 < +0 and the NaN places)
    if dtype == "f32":
        return np.asarray(values).astype(np.float64)
    return order.rank_key(values, dtype)


def _key_no_flip(values, dtype):
    # mistake: signed view without reflecting negative magnitudes
    if dtype == "f32":
        return np.asarray(values).view(np.int32).astype(np.int64)
    return order.rank_key(values, dtype)


def _sort_ties_desc(values, k, dtype):
    # mistake: ties in descending position
    n = values.shape[0]
    key = order.rank_key(values, dtype)
    o = np.lexsort((-np.arange(n), -key))[:k]
    return values[o], o


def _select_off_by_one(values, k, dtype):
    # mistake: partition index n-k+1 instead of n-k
    n = values.shape[0]
    key = order.rank_key(values, dtype)
    T_ = np.partition(key, min(n - 1, n - k + 1))[min(n - 1, n - k + 1)]
    above = np.flatnonzero(key > T_)
    ties = np.flatnonzero(key == T_)[: max(0, k - above.shape[0])]
    idx = np.concatenate([above, ties])
    o = np.lexsort((idx, -key[idx]))
    return values[idx[o]], idx[o]


def _heap_wrong_tiebreak(values, k, dtype):
    # mistake: heap items (key, index) instead of (key, -index)
    import heapq
    key = [int(x) for x in order.rank_key(values, dtype)]
    h = []
    for i in range(len(key)):
        it = (key[i], i)
        if len(h) < k:
            heapq.heappush(h, it)
        elif it > h[0]:
            heapq.heapreplace(h, it)
    idx = np.array([i for _, i in sorted(h, reverse=True)])
    return values[idx], idx


def _smallest_ties_desc(values, k, dtype, largest=True):
    # mistake: for the k smallest, ties in descending position (negating the
    # whole (key, position) order instead of the key alone)
    n = values.shape[0]
    key = order.rank_key(values, dtype)
    o = np.lexsort((np.arange(n), -key))[::-1][:k] if not largest else np.lexsort((np.arange(n), -key))[:k]
    return values[o], o


def _i32_unsigned(values, k, dtype, largest=True):
    # mistake: int32 ranked by its unsigned bit pattern
    v = np.asarray(values)
    key = v.view(np.uint32).astype(np.int64) if dtype == "i32" else order.rank_key(v, dtype)
    key = key if largest else -key
    o = np.lexsort((np.arange(v.shape[0]), -key))[:k]
    return v[o], o


def _threaded_part_share(values, k, dtype):
    # mistake: each of three parts contributes only its share ceil(k / 3) of
    # candidates instead of its own top k
    v = np.asarray(values)
    n = v.shape[0]
    bounds = [n * i // 3 for i in range(4)]
    parts = []
    for i in range(3):
        lo, hi = bounds[i], bounds[i + 1]
        if hi > lo:
            parts.append(T.topk_select(v[lo:hi], min(-(-k // 3), hi - lo), dtype)[1] + lo)
    cand = np.concatenate(parts)
    key = order.rank_key(v[cand], dtype)
    idx = cand[np.lexsort((cand, -key))[:k]]
    return v[idx], idx


def _with_key(fn_key):
    def f(values, k, dtype):
        n = values.shape[0]
        key = fn_key(values, dtype)
        o = np.lexsort((np.arange(n), -key))[:k]
        return values[o], o
    return f


def _with_key_both(fn_key, flip=lambda k: ~k):
    """A sort-and-choose route on a (possibly broken) rank key, both orders."""
    def f(values, k, dtype, largest=True):
        n = values.shape[0]
        key = fn_key(values, dtype)
        key = key if largest else flip(key)
        o = np.lexsort((np.arange(n), ~key))[:k]
        return values[o], o
    return f


def _key_u64_signed(values, dtype):
    # mistake: uint64 ranked by its signed view (2^63 and above rank below 0)
    if dtype == "u64":
        return np.asarray(values).view(np.int64)
    return order.rank_key(values, dtype)


def _key_f64_value(values, dtype):
    # mistake: float64 compared by value (loses -0 < +0 and the NaN places)
    if dtype == "f64":
        return np.asarray(values).astype(np.float64)
    return order.rank_key(values, dtype)


def _key_high_word(values, dtype):
    # mistake: 64-bit keys ranked by their high 32 bits only
    key = order.rank_key(values, dtype)
    return key >> 32 if dtype in ("u64", "i64", "f64") else key


MUTANTS = {
    "float_by_value": (_with_key(_key_float_value), pins.pin_float_order),
    "no_negative_flip": (_with_key(_key_no_flip), pins.pin_float_order),
    "ties_descending": (_sort_ties_desc, pins.pin_closed_forms_u32),
    "select_off_by_one": (_select_off_by_one, pins.pin_exhaustive_u32),
    "heap_tiebreak": (_heap_wrong_tiebreak, pins.pin_exhaustive_u32),
    "smallest_ties_descending": (_smallest_ties_desc, pins.pin_smallest_and_i32),
    "i32_unsigned_order": (_i32_unsigned, pins.pin_smallest_and_i32),
    "threaded_part_share": (_threaded_part_share, pins.pin_exhaustive_u32),
    "u64_signed_view": (_with_key_both(_key_u64_signed), pins.pin_wide),
    "f64_by_value": (_with_key_both(_key_f64_value, flip=lambda k: -k), pins.pin_wide),
    "wide_high_word_only": (_with_key_both(_key_high_word), pins.pin_wide),
    # mistake: the k smallest by negating the key (-(-2^63) wraps to -2^63)
    "i64_negated_smallest": (_with_key_both(order.rank_key, flip=lambda k: -k), pins.pin_wide),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_definition_mutant_caught(name):
    fn, pin = MUTANTS[name]
    with pytest.raises(AssertionError):
        pin(fn)


def test_real_oracle_passes_same_pins():
    for fn, pin in MUTANTS.values():
        pin(oracle.topk_sort)


class _StagesMutant:
    """stages module with one function swapped for a broken one."""

    def __init__(self, **over):
        self.__dict__.update({k: getattr(stages, k) for k in
                              ("delegates", "first_topk", "qualifying", "concatenate",
                               "alpha_rule", "at_or_above")})
        self.__dict__.update(over)

    def method_topk(self, values, k, dtype, alpha, beta):
        dkey, didx = self.delegates(values, dtype, alpha, beta)
        taken, t = self.first_topk(dkey, didx, k)
        qual = self.qualifying(taken, t)
        cand = self.concatenate(values, dtype, alpha, dkey, didx, taken, qual, t)
        sub = np.asarray(values)[cand]
        _, j = oracle.topk_sort(sub, min(k, sub.shape[0]), dtype)
        return np.asarray(values)[cand[j]], cand[j], {}


def _delegates_last_max(values, dtype, alpha, beta):
    # mistake: keep the last (not first) position among equal keys
    key = order.rank_key(values, dtype)
    n = key.shape[0]
    L = 1 << alpha
    S = -(-n // L)
    dk = np.full((S, beta), stages.PAD_KEY, dtype=np.int64)
    di = np.full((S, beta), order.INVALID_INDEX, dtype=np.int64)
    for s in range(S):
        pos = list(range(s * L, min(n, (s + 1) * L)))
        best = sorted(pos, key=lambda i: (-key[i], -i))[:beta]
        for j, i in enumerate(best):
            dk[s, j], di[s, j] = key[i], i
    return dk, di


def _qualifying_any(taken, t):
    # mistake: Rule 3 with "any" delegate taken instead of all of them
    return taken.any(axis=1) if t is not None else np.ones(taken.shape[0], bool)


def _concat_strict(values, dtype, alpha, dkey, didx, taken, qual, t):
    # mistake: filter strictly above t (drops t itself)
    key = order.rank_key(values, dtype)
    n = key.shape[0]
    L = 1 << alpha
    parts = []
    for s in np.flatnonzero(qual):
        pos = np.arange(s * L, min(n, (s + 1) * L))
        kk = key[pos]
        parts.append(pos[(kk > t[0]) | ((kk == t[0]) & (pos < t[1]))])
    parts.append(didx[taken & ~qual[:, None]].astype(np.int64))
    return np.unique(np.concatenate(parts))


def _alpha_ceil(n, k, const=3.0):
    import math
    return int(math.ceil(0.5 * (math.log2(n) - math.log2(k) + const)))


def _first_topk_kplus1(dkey, didx, k):
    # mistake: threshold taken at the (k+1)-th delegate
    return stages.first_topk(dkey, didx, k + 1)


@pytest.mark.parametrize("name,mut,pin", [
    ("delegate_last_max", dict(delegates=_delegates_last_max), pins.pin_delegates_bruteforce),
    ("qualify_any", dict(qualifying=_qualifying_any), pins.pin_paper_example),
    ("filter_strict", dict(concatenate=_concat_strict), pins.pin_paper_example),
    ("alpha_ceil", dict(alpha_rule=_alpha_ceil), pins.pin_paper_example),
    ("threshold_k_plus_1", dict(first_topk=_first_topk_kplus1), pins.pin_paper_example),
])
def test_stage_mutant_caught(name, mut, pin):
    m = _StagesMutant(**mut)
    with pytest.raises(AssertionError):
        if pin is pins.pin_delegates_bruteforce:
            pin(m.delegates)
        else:
            pin(m)

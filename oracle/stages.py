"""The delegate-centric method step by step (oracle; test infrastructure only).

This is the paper's pipeline (Sections 3-5) written plainly, in its order, so
that each stage of the GPU path can be compared with it:

1. delegate vector (Section 5.1; Rule 1 for the maximum delegate, Rule 3 for
   beta delegates): V is cut into subranges of 2^alpha consecutive elements;
   each contributes its beta highest-ranked elements as (key, position);
2. first top-k (Rule 2): the k highest-ranked delegates; their lowest member
   t is the least value the final k-th element can take;
3. qualifying subranges (Rules 1 and 3): a subrange is concatenated only when
   all of its beta delegates are among the first top-k;
4. filtered concatenation (Section 4.2): elements of qualifying subranges
   that rank at or above t, together with the taken delegates of the other
   subranges (the beta = 2, top-3 worked example keeps such a delegate);
5. second top-k on the concatenated vector.

Readings where the paper is silent or loose (each listed in the design notes):
* order and ties: ``rank_key`` order, equal keys ranked by ascending
  position, applied everywhere -- inside a subrange, in the delegate vector
  and in the threshold, which is therefore a (key, position) pair;
* "larger than min(topk(D))": kept inclusive (rank >= t), as the worked
  example keeps 3012 = t itself;
* a last subrange shorter than 2^alpha is allowed; a subrange with fewer than
  beta elements pads its delegate list with (lowest key, INVALID_INDEX);
* fewer than k real delegates: no threshold, every subrange qualifies.

The padding key below is below every rank key of the 32-bit key types; the
stage model serves those (64-bit keys are checked on final results).
"""
from __future__ import annotations

import math

import numpy as np

from .order import rank_key, INVALID_INDEX
from .topk import topk_sort

PAD_KEY = -(1 << 40)  # below every rank key of every dtype


def alpha_rule(n: int, k: int, const: float = 3.0) -> int:
    """Rule 4 (equation for the tuned alpha): alpha = 1/2 [log2|V| - log2 k + const],
    rounded down (the paper's worked instance |V| = 2^30, k = 2^24 gives 4),
    with const = 3 from the paper's tuning; never below 0."""
    a = 0.5 * (math.log2(n) - math.log2(k) + const)
    return max(0, int(math.floor(a)))


def delegates(values: np.ndarray, dtype: str, alpha: int, beta: int):
    """Delegate vector: per subrange of 2^alpha elements, its top-beta (key, position).

    Returns ``(dkey, didx)`` of shape (S, beta), S = ceil(n / 2^alpha), each row
    in rank order; padding rows use (PAD_KEY, INVALID_INDEX).
    """
    key = rank_key(values, dtype)
    n = key.shape[0]
    L = 1 << alpha
    S = -(-n // L)
    kp = np.full(S * L, PAD_KEY, dtype=np.int64)
    kp[:n] = key
    rows = kp.reshape(S, L)
    if beta == 1:
        col = np.argmax(rows, axis=1)[:, None]  # first (lowest-position) maximum
    else:
        col = np.argsort(-rows, axis=1, kind="stable")[:, :beta]
        if col.shape[1] < beta:  # 2^alpha < beta: every element is a delegate
            col = np.concatenate([col, np.full((S, beta - col.shape[1]), -1)], axis=1)
    dkey = np.full((S, beta), PAD_KEY, dtype=np.int64)
    didx = np.full((S, beta), INVALID_INDEX, dtype=np.int64)
    base = (np.arange(S, dtype=np.int64) * L)[:, None]
    pos = base + col
    ok = (col >= 0) & (pos < n)
    dkey[ok] = kp[pos[ok]]
    didx[ok] = pos[ok]
    return dkey, didx


def first_topk(dkey: np.ndarray, didx: np.ndarray, k: int):
    """Rule 2: the k highest-ranked real delegates and their lowest one, t.

    Returns ``(taken, t)``: ``taken`` is a boolean (S, beta) mask of delegates in
    top-k(D); ``t`` is the (key, position) of the k-th, or None when D holds
    fewer than k real delegates.
    """
    valid = didx != INVALID_INDEX
    fk, fi = dkey[valid], didx[valid]
    if fk.shape[0] < k:
        return valid.copy(), None
    order = np.lexsort((fi, -fk))
    t = (int(fk[order[k - 1]]), int(fi[order[k - 1]]))
    return at_or_above(dkey, didx, t) & valid, t


def at_or_above(key: np.ndarray, idx: np.ndarray, t) -> np.ndarray:
    """Rank >= t in the (key desc, position asc) order: key > tk, or key == tk and pos <= ti."""
    tk, ti = t
    return (key > tk) | ((key == tk) & (idx <= ti))


def qualifying(taken: np.ndarray, t) -> np.ndarray:
    """Rules 1 and 3: subrange s is concatenated iff all beta of its delegates are taken."""
    if t is None:
        return np.ones(taken.shape[0], dtype=bool)
    return taken.all(axis=1)


def concatenate(values: np.ndarray, dtype: str, alpha: int, dkey, didx, taken, qual, t):
    """Filtered concatenation: positions of qualifying subranges ranked >= t,
    plus the taken delegates of non-qualifying subranges.  Ascending positions."""
    key = rank_key(values, dtype)
    n = key.shape[0]
    L = 1 << alpha
    if t is None:
        return np.arange(n, dtype=np.int64)
    parts = []
    for s in np.flatnonzero(qual):
        lo, hi = s * L, min(n, (s + 1) * L)
        pos = np.arange(lo, hi, dtype=np.int64)
        parts.append(pos[at_or_above(key[lo:hi], pos, t)])
    other = taken & ~qual[:, None]
    parts.append(didx[other].astype(np.int64))
    return np.unique(np.concatenate(parts)) if parts else np.zeros(0, dtype=np.int64)


def scanned_threshold_form(dkey, didx, t) -> np.ndarray:
    """The equivalent per-subrange test the GPU path uses: scan s iff its beta-th
    delegate ranks strictly above t (Rule 3 with the beta-th delegate compared to t)."""
    if t is None:
        return np.ones(dkey.shape[0], dtype=bool)
    tk, ti = t
    k_b, i_b = dkey[:, -1], didx[:, -1]
    return (k_b > tk) | ((k_b == tk) & (i_b < ti))


def method_topk(values: np.ndarray, k: int, dtype: str, alpha: int, beta: int):
    """All five steps; returns (values, indices, info) where info holds each stage."""
    dkey, didx = delegates(values, dtype, alpha, beta)
    taken, t = first_topk(dkey, didx, k)
    qual = qualifying(taken, t)
    cand = concatenate(values, dtype, alpha, dkey, didx, taken, qual, t)
    sub = np.asarray(values)[cand]
    _, j = topk_sort(sub, k, dtype)
    idx = cand[j]
    info = dict(dkey=dkey, didx=didx, taken=taken, t=t, qualifying=qual, candidates=cand)
    return np.asarray(values)[idx], idx, info

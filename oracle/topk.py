"""Top-k and k-selection by definition (oracle; test infrastructure only).

Problem statement (Section 1): top-k returns the k largest elements of V,
k-selection the k-th largest.  This project fixes what the paper leaves open:

* order: ``rank_key`` (unsigned and signed integers in their own order; floats
  by IEEE totalOrder; 32- and 64-bit keys);
* ties: among equal keys the lower position ranks first, so position i
  precedes j iff key[i] > key[j] or (key[i] == key[j] and i < j);
* output: the k first positions in that order, i.e. values sorted by key
  descending with ties in ascending position; the k-th value counts
  multiplicity (the value at output slot k-1).

``largest=False`` asks for the k smallest instead (the nearest-neighbour and
least-score uses of the real-world datasets, Section 6): the same definition
with the key order reversed and the same tie rule, i.e. i precedes j iff
key[i] < key[j] or (key[i] == key[j] and i < j); values come out ascending.

Every function returns ``(values, indices)`` with ``values`` the input's own
bit patterns at ``indices``.
"""
from __future__ import annotations

import heapq
import os
import threading

import numpy as np

from .order import rank_key


def _key(values: np.ndarray, dtype: str, largest: bool) -> np.ndarray:
    """Ranking key: a larger number ranks first (for the k smallest, the
    complemented order key: ~x = -1 - x reverses the order like a negation
    but cannot overflow at the int64 minimum)."""
    key = rank_key(values, dtype)
    return key if largest else ~key


def _check(values: np.ndarray, k: int) -> int:
    n = int(np.asarray(values).shape[0])
    if not (1 <= k <= n):
        raise ValueError(f"need 1 <= k <= n, got k={k}, n={n}")
    return n


def topk_bruteforce(values: np.ndarray, k: int, dtype: str, largest: bool = True):
    """O(n^2) ranks straight from the definition (pure Python; n <= a few thousand).

    rank(i) = #{j : key[j] > key[i]} + #{j < i : key[j] == key[i]}; the output
    slot r holds the unique i with rank(i) == r.
    """
    n = _check(values, k)
    key = [int(x) for x in _key(values, dtype, largest)]
    out = [None] * n
    for i in range(n):
        r = 0
        for j in range(n):
            if key[j] > key[i] or (key[j] == key[i] and j < i):
                r += 1
        out[r] = i
    idx = np.array(out[:k], dtype=np.int64)
    return np.asarray(values)[idx], idx


def topk_sort(values: np.ndarray, k: int, dtype: str, largest: bool = True):
    """Sort-and-choose (Section 2.2): sort every position by (key desc, index asc), keep k."""
    n = _check(values, k)
    key = _key(values, dtype, largest)
    order = np.lexsort((np.arange(n, dtype=np.int64), ~key))
    idx = order[:k].astype(np.int64)
    return np.asarray(values)[idx], idx


def topk_select(values: np.ndarray, k: int, dtype: str, largest: bool = True):
    """k-selection first, then extraction (the selection route the paper's
    top-k algorithms follow, Section 2.2):

    1. T = the k-th largest key (numpy introselect on the rank keys);
    2. g = #{key > T};
    3. take every position with key > T, and the k - g lowest positions with
       key == T, in one ascending pass;
    4. order those k by (key desc, index asc).
    """
    n = _check(values, k)
    key = _key(values, dtype, largest)
    T = np.partition(key, n - k)[n - k]
    above = np.flatnonzero(key > T)
    g = above.shape[0]
    ties = np.flatnonzero(key == T)[: k - g]
    idx = np.concatenate([above, ties]).astype(np.int64)
    order = np.lexsort((idx, ~key[idx]))
    idx = idx[order]
    return np.asarray(values)[idx], idx


def topk_heap(values: np.ndarray, k: int, dtype: str, largest: bool = True):
    """The textbook priority-queue top-k (Section 1): a size-k min-heap slides
    over V; an element replaces the heap minimum when it ranks higher.

    Heap items are (key, -index) so the heap root is the lowest-ranked kept
    element (smallest key; among equal keys, the largest index).  Pure Python.
    """
    n = _check(values, k)
    key = [int(x) for x in _key(values, dtype, largest)]
    heap = []
    for i in range(n):
        item = (key[i], -i)
        if len(heap) < k:
            heapq.heappush(heap, item)
        elif item > heap[0]:
            heapq.heapreplace(heap, item)
    kept = sorted(heap, reverse=True)
    idx = np.array([-m for _, m in kept], dtype=np.int64)
    return np.asarray(values)[idx], idx


def topk_threaded(values: np.ndarray, k: int, dtype: str, largest: bool = True, threads: int | None = None):
    """The selection route on every host core: split, select per part, merge.

    Positions [0, n) are cut into ``threads`` contiguous parts (default: the
    OMP_NUM_THREADS share, else every core); a thread takes its part's
    min(k, part) highest-ranked positions by ``topk_select``.  Every member of
    the answer is among its own part's top k (fewer than k elements rank above
    it anywhere, so also inside its part), so the answer is the first k of the
    union of the part lists in the (key desc, position asc) order.  numpy's
    selection and sorting release the interpreter lock, so the parts run in
    parallel.
    """
    n = _check(values, k)
    values = np.asarray(values)
    T = threads or int(os.environ.get("OMP_NUM_THREADS") or 0) or os.cpu_count() or 1
    T = max(1, min(int(T), n))
    bounds = [n * i // T for i in range(T + 1)]
    parts: list = [None] * T
    errors: list = []

    def work(i: int) -> None:
        try:
            lo, hi = bounds[i], bounds[i + 1]
            _, idx = topk_select(values[lo:hi], min(k, hi - lo), dtype, largest)
            parts[i] = idx + lo
        except BaseException as e:  # re-raised in the caller
            errors.append(e)

    pool = [threading.Thread(target=work, args=(i,)) for i in range(T)]
    for t in pool:
        t.start()
    for t in pool:
        t.join()
    if errors:
        raise errors[0]
    cand = np.concatenate(parts)
    key = _key(values[cand], dtype, largest)
    idx = cand[np.lexsort((cand, ~key))[:k]].astype(np.int64)
    return values[idx], idx


def topk(values: np.ndarray, k: int, dtype: str, largest: bool = True):
    """Reference answer at any size: the selection route (fast, numpy)."""
    return topk_select(values, k, dtype, largest)


def kth_value(values: np.ndarray, k: int, dtype: str, largest: bool = True):
    """k-selection (Section 1): the k-th largest value (or k-th smallest),
    counting multiplicity."""
    n = _check(values, k)
    key = _key(values, dtype, largest)
    T = np.partition(key, n - k)[n - k]
    i = int(np.flatnonzero(key == T)[0])
    return np.asarray(values)[i]

"""Independent numpy derivations used to pin the oracle and to check the GPU.

Nothing here implements the sampling method: these are the plain definitions
of the problem (section 2 of the paper, with the implicit tags of section
6.1) written with numpy's stable sort, plus the invariants a correct run must
satisfy.
"""
from __future__ import annotations

import numpy as np

NONE = (1 << 64) - 1


def seg_bounds(n: int, p: int) -> np.ndarray:
    """Segment boundaries floor(s N / p), s = 0..p, exact."""
    return np.array([(s * n) // p for s in range(p + 1)], dtype=np.int64)


def ideal(n: int, p: int) -> np.ndarray:
    return np.array([(i * n) // p for i in range(p + 1)], dtype=object)


def local_order(keys: np.ndarray, p: int) -> np.ndarray:
    """Original index of the element that ends up at tag g after the local sort."""
    n = len(keys)
    sb = seg_bounds(n, p)
    out = np.empty(n, dtype=np.int64)
    for s in range(p):
        a, b = sb[s], sb[s + 1]
        out[a:b] = a + np.argsort(keys[a:b], kind="stable")
    return out


def global_rank_of_index(keys: np.ndarray) -> np.ndarray:
    """Rank of every original index in the order (key, index) = the stable sort."""
    order = np.argsort(keys, kind="stable")
    rank = np.empty(len(keys), dtype=np.int64)
    rank[order] = np.arange(len(keys))
    return rank


def tag_rank(keys: np.ndarray, p: int) -> np.ndarray:
    """Global rank of the element with tag g (position in the locally sorted buffer)."""
    return global_rank_of_index(keys)[local_order(keys, p)]


def brute_counts(keys: np.ndarray, p: int, g: int) -> np.ndarray:
    """c_s for the element with tag g, by direct comparison with every element."""
    n = len(keys)
    sb = seg_bounds(n, p)
    lo = local_order(keys, p)
    x = lo[g]
    kx = keys[x]
    res = np.zeros(p, dtype=np.int64)
    for s in range(p):
        seg = keys[sb[s]:sb[s + 1]]
        idx = np.arange(sb[s], sb[s + 1])
        # (key, original index) order == (key, segment, local index) order
        res[s] = int(np.sum((seg < kx) | ((seg == kx) & (idx < x))))
    return res


def expected_partition(keys, vals, p, chi):
    """Partition output implied by splitter ranks chi: bucket-major, then
    source segment, then local sorted order."""
    n = len(keys)
    lo = local_order(keys, p)              # tag -> original index
    rank_of_tag = global_rank_of_index(keys)[lo]
    sb = seg_bounds(n, p)
    seg_of_tag = np.searchsorted(sb, np.arange(n), side="right") - 1
    chi = np.asarray([int(c) for c in chi], dtype=np.int64)
    bucket = np.searchsorted(chi, rank_of_tag, side="right") - 1
    order = np.lexsort((np.arange(n), seg_of_tag, bucket))
    src = lo[order]
    return keys[src], (None if vals is None else vals[src])


def check_balance(chi, n: int, p: int, tol: int):
    """Section 2 invariants: each splitter rank inside its target range, ranks
    non-decreasing, every bucket at most ceil(N/p) + 2 tol keys."""
    chi = [int(c) for c in chi]
    idl = ideal(n, p)
    assert chi[0] == 0 and chi[p] == n
    for i in range(1, p):
        assert abs(chi[i] - idl[i]) <= tol, (i, chi[i], idl[i], tol)
    for i in range(p):
        assert chi[i] <= chi[i + 1]
        assert chi[i + 1] - chi[i] <= -(-n // p) + 2 * tol

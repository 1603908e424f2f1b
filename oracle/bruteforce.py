"""O(n^2) brute-force re-indexer for tiny meshes — TEST INFRASTRUCTURE.

Independent of the std::map oracle (no sorting, no maps): duplicates are found
by comparing record bytes pairwise, a value's new id is the number of used
distinct values whose word tuple is smaller (counted pairwise), and the
representative is the smallest original id among all bitwise-equal copies.
Pure-Python loops; keep n to a few hundred.
"""
from __future__ import annotations

import numpy as np


def _less(a, b) -> bool:
    """Word tuples compared unsigned, word 0 first."""
    for x, y in zip(a, b):
        if x != y:
            return x < y
    return False


def reindex(vtx: np.ndarray, idx: np.ndarray):
    v = np.ascontiguousarray(vtx)
    n = v.shape[0]
    recs = [v[i].tobytes() for i in range(n)]
    words = [tuple(int(w) for w in v[i].view(np.uint32)) for i in range(n)]
    flat = [int(x) for x in np.asarray(idx).reshape(-1)]
    for k, x in enumerate(flat):
        if x < 0 or x >= n:
            raise IndexError(k)
    # first copy of each value (smallest id with identical bytes)
    first = [min(j for j in range(n) if recs[j] == recs[i]) for i in range(n)]
    used_heads = sorted(set(first[x] for x in flat))
    # new id of a used head = number of used heads with a smaller word tuple
    new_of_head = {}
    for h in used_heads:
        new_of_head[h] = sum(1 for g in used_heads if _less(words[g], words[h]))
    u = len(used_heads)
    out_vtx = np.zeros((u, v.view(np.uint32).shape[1] if n else 0), dtype=np.uint32)
    new2old = np.zeros(u, dtype=np.int32)
    for h, j in new_of_head.items():
        out_vtx[j] = v[h].view(np.uint32)
        new2old[j] = h
    old2new = np.array([new_of_head.get(first[i], -1) for i in range(n)], dtype=np.int32)
    out_idx = np.array([old2new[x] for x in flat], dtype=np.int32).reshape(np.asarray(idx).shape)
    return out_vtx, out_idx, old2new, new2old

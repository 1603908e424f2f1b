"""Re-enactment of the method's Steps 1-4 (Section 2) in the paper's order and
notation — TEST INFRASTRUCTURE.

It exists to pin the std::map oracle: it follows the paper's own sequence
(mark used, overwrite unused, key-value sort with orgID, nodup flags, postfix
sum minus one, scatter to newVtx, inverse permutation ``perm``, index remap)
and exposes every intermediate array so that the tests can compare them with
the arrays the paper prints for its worked example.

Readings taken where the text is loose:
* vertices compare as tuples of unsigned 32-bit words, word 0 most
  significant; equality is bitwise;
* the "postfix sum" of Step 2 is an inclusive prefix sum (the paper names
  ``thrust::inclusive_scan``), followed by subtracting one;
* Step 3 reads the *sorted* array at sorted positions (as its pseudocode
  does);
* the sort is a stable key-value sort unless the caller passes another
  ordering of equal keys (``sort_order``), which lets a test reproduce the
  tie order the paper happened to print.
"""
from __future__ import annotations

import numpy as np


def _as_words(vtx: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(vtx)
    return v.view(np.uint32).reshape(v.shape[0], -1)


def step1_mark_used(num_vtx: int, idx: np.ndarray) -> np.ndarray:
    """isUsed[vtxID] = true for every vertex index of every element."""
    is_used = np.zeros(num_vtx, dtype=bool)
    for vtx_id in np.asarray(idx).reshape(-1):
        is_used[vtx_id] = True
    return is_used


def step1_overwrite_unused(words: np.ndarray, idx: np.ndarray, is_used: np.ndarray) -> np.ndarray:
    """vtx[i] = vtx[first vertex of first element] for every unused i."""
    out = words.copy()
    first = int(np.asarray(idx).reshape(-1)[0])
    for i in range(out.shape[0]):
        if not is_used[i]:
            out[i] = words[first]
    return out


def step2_sort(words: np.ndarray, sort_order=None):
    """Key-value sort of (vtx, orgID). Stable unless ``sort_order`` is given."""
    org_id = np.arange(words.shape[0], dtype=np.int64)
    if sort_order is None:
        # np.lexsort sorts by the last key first; pass w{K-1} .. w0 so that w0
        # is the primary key. It is stable.
        order = np.lexsort(tuple(words[:, w] for w in range(words.shape[1] - 1, -1, -1)))
    else:
        order = np.asarray(sort_order, dtype=np.int64)
    return words[order], org_id[order]


def step2_nodup(sorted_words: np.ndarray) -> np.ndarray:
    """nodup[i] = (i == 0) || (vtx[i] != vtx[i-1])."""
    n = sorted_words.shape[0]
    nodup = np.zeros(n, dtype=np.int64)
    for i in range(n):
        nodup[i] = 1 if i == 0 or not np.array_equal(sorted_words[i], sorted_words[i - 1]) else 0
    return nodup


def step2_new_idx(nodup: np.ndarray):
    """Postfix (inclusive) sum over nodup, then subtract one."""
    inclusive = np.cumsum(nodup)
    return inclusive, inclusive - 1


def step3_new_vtx(sorted_words: np.ndarray, nodup: np.ndarray, new_idx: np.ndarray):
    """newN = newIdx.back() + 1; newVtx[newIdx[i]] = vtx[i] at run heads."""
    new_n = int(new_idx[-1]) + 1
    new_vtx = np.zeros((new_n, sorted_words.shape[1]), dtype=np.uint32)
    for i in range(sorted_words.shape[0]):
        if nodup[i]:
            new_vtx[new_idx[i]] = sorted_words[i]
    return new_n, new_vtx


def step4_perm(org_id: np.ndarray) -> np.ndarray:
    """perm[orgID[i]] = i."""
    perm = np.empty(org_id.shape[0], dtype=np.int64)
    for i in range(org_id.shape[0]):
        perm[org_id[i]] = i
    return perm


def step4_remap(idx: np.ndarray, perm: np.ndarray, new_idx: np.ndarray) -> np.ndarray:
    """Every old index i becomes newIdx[perm[i]]."""
    flat = np.asarray(idx).reshape(-1)
    out = np.array([new_idx[perm[i]] for i in flat], dtype=np.int64)
    return out.reshape(np.asarray(idx).shape)


def run(vtx: np.ndarray, idx: np.ndarray, sort_order=None) -> dict:
    """All four steps; returns every intermediate array by its paper name."""
    words = _as_words(vtx)
    is_used = step1_mark_used(words.shape[0], idx)
    cleaned = step1_overwrite_unused(words, idx, is_used)
    sorted_words, org_id = step2_sort(cleaned, sort_order)
    nodup = step2_nodup(sorted_words)
    postfix, new_idx = step2_new_idx(nodup)
    new_n, new_vtx = step3_new_vtx(sorted_words, nodup, new_idx)
    perm = step4_perm(org_id)
    new_elems = step4_remap(idx, perm, new_idx)
    return dict(isUsed=is_used, vtx_cleaned=cleaned, vtx_sorted=sorted_words,
                orgID=org_id, nodup=nodup, newIdx_postfix=postfix, newIdx=new_idx,
                newN=new_n, newVtx=new_vtx, perm=perm, idx_new=new_elems,
                old2new=new_idx[perm])

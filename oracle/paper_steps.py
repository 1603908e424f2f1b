"""Re-enactment of the method's four steps (Section 2) in the paper's order and
with its array names — TEST INFRASTRUCTURE.

It exists to pin the std::map oracle. Each function states what its step
produces and computes it with whole-array numpy operations; every
intermediate array is returned under the paper's name, so the tests can hold
it against the arrays the paper prints for its worked example.

Readings taken where the text is loose:
* records compare as tuples of unsigned 32-bit words, word 0 most
  significant; equality is bitwise;
* the running sum of Step 2 is inclusive (the library routine the paper
  names is an inclusive scan), and one is subtracted afterwards;
* Step 3 reads the *sorted* array at sorted positions (its pseudocode does;
  its prose says otherwise);
* the sort is stable unless the caller supplies another order of equal keys
  (``sort_order``), which lets a test reproduce the tie order the paper
  happened to print.
"""
from __future__ import annotations

import numpy as np


def _as_words(vtx: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(vtx)
    return v.view(np.uint32).reshape(v.shape[0], -1)


def step1_mark_used(num_vtx: int, idx: np.ndarray) -> np.ndarray:
    """Step 1 (isUsed): True exactly for the vertices some element refers to."""
    is_used = np.zeros(num_vtx, dtype=bool)
    is_used[np.asarray(idx, dtype=np.int64).reshape(-1)] = True
    return is_used


def step1_overwrite_unused(words: np.ndarray, idx: np.ndarray, is_used: np.ndarray) -> np.ndarray:
    """Step 1, second half: every vertex nobody refers to takes over the
    record of the vertex that the very first index entry names, so that it
    becomes a duplicate of a used vertex and vanishes in the later steps."""
    out = words.copy()
    donor = int(np.asarray(idx).reshape(-1)[0])
    out[~is_used] = words[donor]
    return out


def step2_sort(words: np.ndarray, sort_order=None):
    """Step 2: sort the records together with their original ids (orgID);
    stable unless ``sort_order`` is given."""
    org_id = np.arange(words.shape[0], dtype=np.int64)
    if sort_order is None:
        # np.lexsort's last key is the primary one: hand it w{K-1} .. w0
        order = np.lexsort(tuple(words[:, w] for w in range(words.shape[1] - 1, -1, -1)))
    else:
        order = np.asarray(sort_order, dtype=np.int64)
    return words[order], org_id[order]


def step2_nodup(sorted_words: np.ndarray) -> np.ndarray:
    """Step 2 (nodup): 1 where a sorted record starts a run of equal records
    (the first record always does), 0 inside a run."""
    n = sorted_words.shape[0]
    flags = np.ones(n, dtype=np.int64)
    if n > 1:
        flags[1:] = np.any(sorted_words[1:] != sorted_words[:-1], axis=1)
    return flags


def step2_new_idx(nodup: np.ndarray):
    """Step 2 (newIdx): the running count of run starts up to and including
    each position, and that count less one, which numbers the runs from 0."""
    inclusive = np.cumsum(nodup)
    return inclusive, inclusive - 1


def step3_new_vtx(sorted_words: np.ndarray, nodup: np.ndarray, new_idx: np.ndarray):
    """Step 3 (newN, newVtx): the number of runs, and one record per run
    (the record at the run's start), in sorted order."""
    new_n = int(new_idx[-1]) + 1
    heads = np.flatnonzero(nodup)
    new_vtx = np.zeros((new_n, sorted_words.shape[1]), dtype=np.uint32)
    new_vtx[new_idx[heads]] = sorted_words[heads]
    return new_n, new_vtx


def step4_perm(org_id: np.ndarray) -> np.ndarray:
    """Step 4 (perm): the inverse of the sort's permutation, i.e. where each
    original vertex ended up in the sorted array."""
    perm = np.empty(org_id.shape[0], dtype=np.int64)
    perm[org_id] = np.arange(org_id.shape[0], dtype=np.int64)
    return perm


def step4_remap(idx: np.ndarray, perm: np.ndarray, new_idx: np.ndarray) -> np.ndarray:
    """Step 4: an old index is replaced by the run number of the sorted
    position its vertex moved to."""
    idx = np.asarray(idx)
    return new_idx[perm[idx.reshape(-1).astype(np.int64)]].reshape(idx.shape)


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

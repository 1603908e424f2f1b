"""Shared test helpers: full-size property checks (no oracle call needed)."""
import numpy as np


def words(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32).reshape(a.shape[0], -1)


def _void(w):
    w = np.ascontiguousarray(w)
    return w.view(np.dtype((np.void, w.dtype.itemsize * w.shape[1]))).reshape(-1)


def check_properties(vtx, idx, out_vtx, out_idx, old2new, new2old, expected_unique=None):
    """Properties that determine the re-index result at any size:
    * out_vtx is strictly ascending (unsigned word tuples) => distinct;
    * out_vtx[out_idx[k]] == vtx[idx[k]] bitwise (Section 2, 'Checking our Example');
    * every output vertex is referenced;
    * new2old[j] holds out_vtx[j] and is the smallest original id with that value;
    * old2new[i] is the new id of vtx[i]'s value, or exactly -1 iff that
      value is unused.
    """
    w = words(vtx)
    ow = words(out_vtx)
    u = ow.shape[0]
    if expected_unique is not None:
        assert u == expected_unique
    flat_idx = idx.reshape(-1)
    flat_out = out_idx.reshape(-1)
    assert flat_out.min(initial=0) >= 0 and flat_out.max(initial=-1) < u
    assert np.array_equal(ow[flat_out], w[flat_idx])
    if u > 1:
        # strictly ascending, lexicographic with word 0 most significant
        order = np.lexsort(tuple(ow[:, c] for c in range(ow.shape[1] - 1, -1, -1)))
        assert np.array_equal(order, np.arange(u))
        assert not np.any(np.all(ow[1:] == ow[:-1], axis=1))
    ref = np.zeros(u, dtype=bool)
    ref[flat_out] = True
    assert ref.all()
    assert new2old.shape[0] == u
    assert np.array_equal(w[new2old], ow)
    assert np.array_equal(old2new[new2old], np.arange(u))
    mapped = old2new >= 0
    # the only negative value old2new may hold is -1 (value not used)
    assert np.all(old2new[~mapped] == -1)
    assert old2new.max(initial=-1) < u
    assert np.array_equal(w[mapped], ow[old2new[mapped]])
    # unmapped vertices hold values that are not among the outputs
    vo = _void(ow)
    vu = _void(w[~mapped])
    if vu.size and u:
        srt = np.sort(vo)
        pos = np.searchsorted(srt, vu)
        pos = np.minimum(pos, u - 1)
        assert not np.any(srt[pos] == vu)
    # representative = smallest original id with that value
    first = np.full(u, np.iinfo(np.int64).max, dtype=np.int64)
    ids = np.nonzero(mapped)[0]
    np.minimum.at(first, old2new[mapped], ids)
    assert np.array_equal(first, new2old)

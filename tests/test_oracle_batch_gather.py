"""Pins for the batched and attribute-gather parts of the CPU oracle (no GPU).

``oracle.reindex_batched`` is checked against the brute-force re-indexer run on
each mesh built on its own (so a wrong slice or a wrong offset accumulation in
the packing shows), against a closed form for the output count of every
patch mesh of the batched workload, and on copies of one mesh that must not
merge across meshes.

``oracle.gather_attrs`` / ``gather_attrs_backward`` are checked against
explicit row loops, against the closed form of the gradient of a weighted sum
through an injective map, and on a map with repeated entries whose gradient
rows must accumulate.
"""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from oracle import bruteforce


def _pack(meshes, words, arity):
    vo = np.concatenate([[0], np.cumsum([m[0].shape[0] for m in meshes])]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum([m[1].shape[0] for m in meshes])]).astype(np.int64)
    vtx = np.concatenate([m[0].reshape(-1, words) for m in meshes]).reshape(-1, words)
    idx = np.concatenate([m[1].reshape(-1, arity) for m in meshes]).reshape(-1, arity)
    return vtx, idx, vo, eo


def _tiny_batches(count, seed=31):
    """Batches of tiny meshes (some with no vertices, some with no elements)
    built one by one."""
    rng = np.random.default_rng(seed)
    for c in range(count):
        words = int(rng.integers(1, 4))
        arity = int(rng.integers(1, 4))
        meshes = []
        for _ in range(int(rng.integers(1, 6))):
            n = int(rng.integers(0, 30))
            if n == 0:
                meshes.append((np.zeros((0, words), np.uint32), np.zeros((0, arity), np.int32)))
                continue
            e = int(rng.integers(0, 12))
            v, i = meshgen.random_mesh(n, max(e, 1), arity, words, int(rng.integers(1, n + 1)),
                                       4000 + 10 * c + len(meshes), 0.7)
            if e == 0:
                i = np.zeros((0, arity), np.int32)
            meshes.append((np.ascontiguousarray(v).view(np.uint32).reshape(n, words), i))
        yield meshes, words, arity


def test_batched_matches_bruteforce_of_each_mesh():
    for meshes, words, arity in _tiny_batches(80):
        vtx, idx, vo, eo = _pack(meshes, words, arity)
        ov, offs, oi, o2n, n2o = oracle.reindex_batched(vtx, idx, vo, eo)
        assert offs[0] == 0 and offs.shape[0] == len(meshes) + 1
        for b, (v, i) in enumerate(meshes):
            ev, ei, eo2n, en2o = bruteforce.reindex(v, i)
            assert offs[b + 1] - offs[b] == ev.shape[0]
            if ev.shape[0]:
                assert np.array_equal(ov[offs[b]:offs[b + 1]], ev)
            assert np.array_equal(n2o[offs[b]:offs[b + 1]], en2o)
            assert np.array_equal(oi[eo[b]:eo[b + 1]], ei)
            assert np.array_equal(o2n[vo[b]:vo[b + 1]], eo2n)
        assert ov.shape[0] == offs[-1] and n2o.shape[0] == offs[-1]
        assert oi.shape == idx.shape and o2n.shape[0] == vtx.shape[0]


def _patch_points_touched(w: int, t: int) -> int:
    """Distinct grid points used by the first t triangles, row-major, of a
    quad patch w quads wide (quad (i, j) = triangles (v00, v10, v11) and
    (v00, v11, v01)), counted by rows rather than by listing them."""
    q, half = divmod(t, 2)
    rows, c = divmod(q, w)
    pts = (rows + 1) * (w + 1) if rows else 0
    if c:
        pts += (c + 1) if rows else 2 * (c + 1)
    if half:
        pts += 1 if rows else (2 if c else 3)
    return pts


def test_patch_count_closed_form_by_listing():
    # 2 quads wide: 1 triangle -> 3 points, then 4, 6, 6, 7 (the second row starts)
    assert [_patch_points_touched(2, t) for t in range(1, 6)] == [3, 4, 6, 6, 7]
    for w in range(1, 6):
        for t in range(1, 40):
            pts = set()
            for k in range(t):
                i, j = (k // 2) % w, (k // 2) // w
                tri = [(i, j), (i + 1, j), (i + 1, j + 1)] if k % 2 == 0 else \
                      [(i, j), (i + 1, j + 1), (i, j + 1)]
                pts.update(tri)
            assert _patch_points_touched(w, t) == len(pts), (w, t)


def test_batched_closed_form_counts():
    b = meshgen.batched(24, 100, 4000, 0.05, 2109_09812 + 41, "small_batch")
    t, w, h, _ = meshgen.batch_sizes(24, 100, 4000, 2109_09812 + 41)
    closed = np.array([_patch_points_touched(int(w[i]), int(t[i])) for i in range(24)])
    assert np.array_equal(closed, b.expected_unique)
    ov, offs, oi, o2n, n2o = oracle.reindex_batched(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    assert np.array_equal(np.diff(offs), closed)
    # E is unchanged and every id is local to its mesh
    assert oi.shape == b.idx.shape
    for i in range(24):
        u = offs[i + 1] - offs[i]
        local = oi[b.elem_offsets[i]:b.elem_offsets[i + 1]]
        assert local.min() >= 0 and local.max() < u
        seg = o2n[b.vtx_offsets[i]:b.vtx_offsets[i + 1]]
        assert seg.max() == u - 1 and seg.min() == -1    # 5% unused vertices per mesh
        assert n2o[offs[i]:offs[i + 1]].max() < b.vtx_offsets[i + 1] - b.vtx_offsets[i]


def test_batched_copies_never_merge():
    m = meshgen.grid_soup(20, 0.1, 17, "copies")
    single = oracle.reindex(m.vtx, m.idx)
    u = single[0].shape[0]
    copies = 3
    meshes = [(m.vtx.view(np.uint32), m.idx)] * copies
    vtx, idx, vo, eo = _pack(meshes, 3, 3)
    ov, offs, oi, o2n, n2o = oracle.reindex_batched(vtx, idx, vo, eo)
    assert list(offs) == [c * u for c in range(copies + 1)]
    for c in range(copies):
        assert np.array_equal(ov[c * u:(c + 1) * u], single[0])
        assert np.array_equal(oi[eo[c]:eo[c + 1]], single[1])
        assert np.array_equal(o2n[vo[c]:vo[c + 1]], single[2])
        assert np.array_equal(n2o[c * u:(c + 1) * u], single[3])
    # the same packed arrays merged as one mesh collapse to one copy
    assert oracle.merge(vtx, idx, vo, eo)[0].shape[0] == u


def test_batched_reports_local_range_errors():
    a = meshgen.grid_soup(6, 0.0, 1, "a")
    b = meshgen.grid_soup(6, 0.0, 2, "b")
    idx = np.concatenate([a.idx, b.idx]).copy()
    idx[a.idx.shape[0] + 1, 0] = b.vtx.shape[0]   # one past mesh b's last vertex
    vtx, _, vo, eo = _pack([(a.vtx, a.idx), (b.vtx, b.idx)], 3, 3)
    with pytest.raises(oracle.OracleIndexError):
        oracle.reindex_batched(vtx, idx, vo, eo)


# ----------------------------------------------------------------- attribute gather

@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_gather_matches_row_loop(dtype):
    g = torch.Generator().manual_seed(3)
    attrs = torch.randn(50, 7, generator=g, dtype=dtype)
    for new2old in (np.array([4, 0, 49, 17, 17, 3], np.int32), np.arange(50, dtype=np.int32)[::-1].copy(),
                    np.zeros(0, np.int32)):
        got = oracle.gather_attrs(attrs, new2old)
        assert got.shape == (new2old.shape[0], 7) and got.dtype == dtype
        for j, i in enumerate(new2old.tolist()):
            for c in range(7):
                assert got[j, c].item() == attrs[i, c].item()


def test_gather_backward_injective_closed_form():
    """d/d attrs of sum(w * attrs[new2old]) is w[j] in row new2old[j], zero
    in every other row; with an injective map every row gets one term."""
    g = torch.Generator().manual_seed(4)
    n, c = 40, 5
    new2old = np.random.default_rng(4).permutation(n)[:23].astype(np.int32)
    w = torch.randn(23, c, generator=g)
    grad = oracle.gather_attrs_backward(w, new2old, n)
    expected = torch.zeros(n, c)
    for j, i in enumerate(new2old.tolist()):
        expected[i] = w[j]
    assert torch.equal(grad, expected)
    untouched = np.setdiff1d(np.arange(n), new2old)
    assert torch.count_nonzero(grad[torch.from_numpy(untouched)]) == 0


def test_gather_backward_repeated_rows_accumulate():
    """A map with repeated entries: every row's gradient is the sum of the
    output rows that read it. Small integer weights keep every sum exact,
    whatever the order of the additions."""
    rng = np.random.default_rng(5)
    n, c = 12, 3
    new2old = rng.integers(0, n, size=40).astype(np.int32)
    w_int = rng.integers(-8, 9, size=(40, c))
    for dtype in (torch.float32, torch.float64):
        grad = oracle.gather_attrs_backward(torch.tensor(w_int, dtype=dtype), new2old, n)
        sums = [[0] * c for _ in range(n)]
        for j, i in enumerate(new2old.tolist()):
            for k in range(c):
                sums[i][k] += int(w_int[j, k])
        assert torch.equal(grad, torch.tensor(sums, dtype=dtype))


def test_gather_gradcheck_fp64():
    g = torch.Generator().manual_seed(6)
    attrs = torch.randn(9, 4, generator=g, dtype=torch.float64, requires_grad=True)
    new2old = np.array([8, 1, 1, 0, 5], np.int32)
    assert torch.autograd.gradcheck(lambda a: oracle.gather_attrs(a, new2old), (attrs,))

"""GPU parity of the Section 3 mesh edits that feed the re-index: merging the
meshes of a packed batch into one mesh, and extracting the sub-mesh of
selected elements. Both are compared bit for bit with the oracle."""
import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _dev_batch(b: meshgen.Batch):
    return (torch.from_numpy(np.ascontiguousarray(b.vtx).view(np.int32)).to(DEV),
            torch.from_numpy(b.vtx_offsets).to(DEV),
            torch.from_numpy(np.ascontiguousarray(b.idx, dtype=np.int32)).to(DEV),
            torch.from_numpy(b.elem_offsets).to(DEV))


def _host(r):
    return (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(), r.old2new.cpu().numpy(),
            r.new2old.cpu().numpy())


def _same(got, exp, name):
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
        assert g.shape == e.shape, (name, label, g.shape, e.shape)
        assert np.array_equal(g, e), f"{name}: {label} differs at {np.argwhere(g != e)[:5].tolist()}"


# ------------------------------------------------------------------ merge

@pytest.mark.parametrize("meshes,hi,seed", [(1, 2000, 1), (7, 3000, 2), (64, 20_000, 3), (300, 4_000, 4)])
def test_merge_matches_oracle(meshes, hi, seed):
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(meshes, 100, hi, 0.05, 1300 + seed)
    _say("merge", meshes, "meshes", b.vtx.shape[0], "vertices")
    got = _host(mrx.merge_meshes(*_dev_batch(b)))
    exp = oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    _same(got, exp, f"merge{meshes}")
    # patches overlap in [0,1]^2, so merging must join vertices across meshes
    if meshes > 1:
        assert got[0].shape[0] < int(b.expected_unique.sum())


def test_merge_of_copies_and_in_place():
    import paper_2109_09812_amd as mrx
    m = meshgen.grid_soup(120, 0.05, 21, "copies")
    n, e = m.vtx.shape[0], m.idx.shape[0]
    b = meshgen.Batch(np.concatenate([m.vtx] * 3), np.concatenate([m.idx] * 3),
                      np.arange(4, dtype=np.int64) * n, np.arange(4, dtype=np.int64) * e,
                      np.full(3, m.expected_unique), "copies")
    vtx, vo, idx, eo = _dev_batch(b)
    _say("merge copies in place")
    r = mrx.merge_meshes(vtx, vo, idx, eo, in_place=True)
    assert r.out_idx.data_ptr() == idx.data_ptr()
    got = _host(r)
    _same(got, oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets), "copies")
    assert got[0].shape[0] == m.expected_unique


def test_merge_with_empty_meshes():
    import paper_2109_09812_amd as mrx
    parts = [meshgen.batched(1, 200, 201, 0.05, 70 + s).mesh(0) for s in range(2)]
    empty_v = np.zeros((0, 3), np.float32)
    empty_i = np.zeros((0, 3), np.int32)
    vs = [empty_v, parts[0].vtx, empty_v, parts[1].vtx, parts[0].vtx]
    is_ = [empty_i, parts[0].idx, empty_i, empty_i, parts[0].idx]
    vo = np.concatenate([[0], np.cumsum([v.shape[0] for v in vs])]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum([i.shape[0] for i in is_])]).astype(np.int64)
    b = meshgen.Batch(np.concatenate(vs), np.concatenate(is_), vo, eo, np.zeros(5, np.int64), "holes")
    _say("merge with empty meshes")
    got = _host(mrx.merge_meshes(*_dev_batch(b)))
    _same(got, oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets), "holes")


def test_merge_local_index_out_of_range():
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(4, 100, 500, 0.05, 88)
    idx = b.idx.copy()
    e2 = int(b.elem_offsets[2])
    idx[e2, 1] = int(b.vtx_offsets[3] - b.vtx_offsets[2])   # valid packed id, outside mesh 2
    bb = meshgen.Batch(b.vtx, idx, b.vtx_offsets, b.elem_offsets, b.expected_unique, "bad")
    _say("merge out of range")
    with pytest.raises(IndexError):
        mrx.merge_meshes(*_dev_batch(bb))


def test_merge_all_tunings_and_flags():
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(40, 100, 6000, 0.05, 99)
    exp = oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    tensors = _dev_batch(b)
    for t in mrx.tunings(12):
        for fl in (0, mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES, mrx.MRX_TUNING_BANDS):
            _say("merge tuning", t.as_tuple(), fl)
            _same(_host(mrx.merge_meshes(*tensors, tuning=(*t.as_tuple(), fl))), exp, "merge tuning")


# ------------------------------------------------------------------ extract

def _extract(vtx_np, idx_np, keep_np, tuning=None):
    import paper_2109_09812_amd as mrx
    v = torch.from_numpy(np.ascontiguousarray(vtx_np).view(np.int32)).to(DEV)
    i = torch.from_numpy(np.ascontiguousarray(idx_np, dtype=np.int32)).to(DEV)
    k = torch.from_numpy(np.ascontiguousarray(keep_np, dtype=bool)).to(DEV)
    r = mrx.extract_submesh(v, i, k, tuning=tuning)
    assert r.num_elems_out == int(np.count_nonzero(keep_np))
    return _host(r)


@pytest.mark.parametrize("frac,seed", [(0.5, 1), (0.05, 2), (0.95, 3), (0.3, 4)])
def test_extract_matches_oracle(frac, seed):
    m = meshgen.grid_soup(400, 0.05, 500 + seed, "ext")
    keep = np.random.default_rng(seed).random(m.idx.shape[0]) < frac
    _say("extract", frac, m.idx.shape[0], "elements")
    _same(_extract(m.vtx, m.idx, keep), oracle.extract(m.vtx, m.idx, keep), f"extract{frac}")


def test_extract_tet_material_and_edge_cases():
    m = meshgen.tet_mesh(16, 0.03, 31)
    for mat in range(3):
        keep = (np.arange(m.idx.shape[0]) % 3) == mat       # three "materials"
        _say("tets material", mat)
        _same(_extract(m.vtx, m.idx, keep), oracle.extract(m.vtx, m.idx, keep), f"material{mat}")
    _say("keep all / none")
    _same(_extract(m.vtx, m.idx, np.ones(m.idx.shape[0], bool)), oracle.reindex(m.vtx, m.idx), "all")
    got = _extract(m.vtx, m.idx, np.zeros(m.idx.shape[0], bool))
    assert got[0].shape[0] == 0 and got[1].shape == (0, 4) and np.all(got[2] == -1)


@pytest.mark.parametrize("n", [64, 1000])
def test_extract_even_quad_rows_closed_form(n):
    m = meshgen.paper_quads(n)
    keep = (np.arange(n * n) // n) % 2 == 0
    _say("quads rows", n)
    got = _extract(m.vtx, m.idx, keep)
    assert got[0].shape[0] == n * (n + 1)
    _same(got, oracle.extract(m.vtx, m.idx, keep), f"quads{n}")


def test_extract_range_errors_only_in_kept_elements():
    m = meshgen.grid_soup(50, 0.0, 3, "bad")
    idx = m.idx.copy()
    idx[10, 0] = m.vtx.shape[0]           # out of range
    keep = np.ones(idx.shape[0], bool)
    keep[10] = False
    _say("extract drops the bad element")
    _same(_extract(m.vtx, idx, keep), oracle.extract(m.vtx, idx, keep), "dropped bad")
    keep[10] = True
    _say("extract keeps the bad element")
    with pytest.raises(IndexError):
        _extract(m.vtx, idx, keep)


def test_extract_all_tunings_and_flags():
    import paper_2109_09812_amd as mrx
    m = meshgen.grid_soup(200, 0.05, 808, "ext tune")
    keep = np.random.default_rng(8).random(m.idx.shape[0]) < 0.6
    exp = oracle.extract(m.vtx, m.idx, keep)
    for t in mrx.tunings(12):
        for fl in (0, mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES, mrx.MRX_TUNING_BANDS,
                   mrx.MRX_TUNING_BANDS | mrx.MRX_TUNING_CLAIMED_TILES):
            _say("extract tuning", t.as_tuple(), fl)
            _same(_extract(m.vtx, m.idx, keep, tuning=(*t.as_tuple(), fl)), exp, "extract tuning")


def test_preallocated_merger_and_extractor_relaunch():
    """The preallocated classes launch repeatedly; the extractor's keep flags
    are refilled in place between launches."""
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(30, 100, 3000, 0.05, 444)
    mg = mrx.MeshMerger(*_dev_batch(b))
    exp = oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    for rep in range(2):
        _say("merger launch", rep)
        mg.launch()
        _same(_host(mg.result()), exp, "merger")
    m = meshgen.grid_soup(150, 0.05, 45, "relaunch")
    v = torch.from_numpy(np.ascontiguousarray(m.vtx).view(np.int32)).to(DEV)
    i = torch.from_numpy(m.idx).to(DEV)
    keep = torch.zeros(m.idx.shape[0], dtype=torch.bool, device=DEV)
    x = mrx.SubmeshExtractor(v, i, keep)
    rng = np.random.default_rng(46)
    for rep, frac in enumerate((0.7, 0.2, 0.0)):
        k = rng.random(m.idx.shape[0]) < frac
        keep.copy_(torch.from_numpy(k))
        _say("extractor launch", rep, frac)
        x.launch()
        r = x.result()
        assert r.num_elems_out == int(k.sum())
        _same(_host(r), oracle.extract(m.vtx, m.idx, k), f"extractor{rep}")


def _capture(launch):
    """Capture one launch into a graph (after an eager warm-up on a side stream)."""
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=DEV)
    side.wait_stream(torch.cuda.current_stream(DEV))
    with torch.cuda.stream(side):
        launch()
    torch.cuda.current_stream(DEV).wait_stream(side)
    with torch.cuda.graph(g):
        launch()
    return g


def test_graph_replays_single_merge_extract():
    """Reindexer, MeshMerger and SubmeshExtractor captured once and replayed
    on refilled inputs, with eager work between replays; every replay must
    match the oracle."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(123)
    # single mesh: same shape, new vertex order each replay
    m = meshgen.grid_soup(120, 0.05, 77, "graph")
    v = torch.from_numpy(np.ascontiguousarray(m.vtx).view(np.int32)).to(DEV)
    i = torch.from_numpy(m.idx).to(DEV)
    rx = mrx.Reindexer(v, i)
    g = _capture(rx.launch)
    for rep in range(3):
        p = rng.permutation(m.vtx.shape[0])
        inv = np.empty_like(p)
        inv[p] = np.arange(p.size)
        vtx_r, idx_r = m.vtx[p], inv[m.idx].astype(np.int32)
        v.copy_(torch.from_numpy(np.ascontiguousarray(vtx_r).view(np.int32)))
        i.copy_(torch.from_numpy(idx_r))
        _say("graph single replay", rep)
        g.replay()
        _same(_host(rx.result()), oracle.reindex(vtx_r, idx_r), f"graph single {rep}")
        _ = (v.float() * 2).sum().item()
    # merge
    b = meshgen.batched(20, 100, 2000, 0.05, 78)
    tensors = _dev_batch(b)
    mg = mrx.MeshMerger(*tensors)
    g = _capture(mg.launch)
    exp = oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    for rep in range(2):
        _say("graph merge replay", rep)
        g.replay()
        _same(_host(mg.result()), exp, f"graph merge {rep}")
        _ = (tensors[0].float() * 2).sum().item()
    # extract: new keep flags each replay
    keep = torch.zeros(m.idx.shape[0], dtype=torch.bool, device=DEV)
    x = mrx.SubmeshExtractor(v, i, keep)
    g = _capture(x.launch)
    for rep, frac in enumerate((0.5, 0.1, 0.9)):
        k = rng.random(m.idx.shape[0]) < frac
        keep.copy_(torch.from_numpy(k))
        _say("graph extract replay", rep)
        g.replay()
        r = x.result()
        assert r.num_elems_out == int(k.sum())
        _same(_host(r), oracle.extract(vtx_r, idx_r, k), f"graph extract {rep}")
        _ = (v.float() * 2).sum().item()

"""GPU parity of the batched (segmented) re-index: one launch sequence for
many independent meshes must equal the per-mesh oracle, never merge equal
vertices of different meshes, and replay correctly from a HIP graph."""
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


def to_dev(b: meshgen.Batch):
    return (torch.from_numpy(np.ascontiguousarray(b.vtx).view(np.int32)).to(DEV),
            torch.from_numpy(b.vtx_offsets).to(DEV),
            torch.from_numpy(b.idx).to(DEV),
            torch.from_numpy(b.elem_offsets).to(DEV))


def check_batch(b: meshgen.Batch, res):
    ov, ooff, oi, o2n, n2o = oracle.reindex_batched(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    assert np.array_equal(res.out_vtx_offsets.cpu().numpy(), ooff)
    assert np.array_equal(res.out_vtx.cpu().numpy().view(np.uint32), ov)
    assert np.array_equal(res.out_idx.cpu().numpy(), oi)
    assert np.array_equal(res.old2new.cpu().numpy(), o2n)
    assert np.array_equal(res.new2old.cpu().numpy(), n2o)
    assert np.array_equal(np.diff(ooff), b.expected_unique)


SORT_ALL = 4  # MRX_TUNING_SORT_ALL; without it batches of 2^16 vertices and more use hash grouping


@pytest.mark.parametrize("strategy", [None, (0, 0, 0, SORT_ALL)])
@pytest.mark.parametrize("meshes,hi,seed", [(1, 3000, 1), (7, 3000, 2), (64, 20_000, 3), (300, 5_000, 4)])
def test_batched_matches_per_mesh_oracle(meshes, hi, seed, strategy):
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(meshes, 100, hi, 0.05, 900 + seed)
    _say("batch", meshes, "meshes", b.vtx.shape[0], "vertices", strategy)
    res = mrx.reindex_mesh_batched(*to_dev(b), tuning=strategy)
    check_batch(b, res)


def test_batched_with_skipped_passes():
    """Key passes whose digit is the same in every mesh are skipped in a
    batch too (the mesh-id passes never are here: 5 meshes)."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(78)
    sizes = [3_001, 0, 17_000, 5, 40_000]
    n = sum(sizes)
    vtx = np.full((n, 3), 0x3F000000, np.uint32)
    vtx[:, 1] = rng.integers(0, 9, n).astype(np.uint32) << np.uint32(16)   # one live key pass
    vo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    idx_parts, eo = [], [0]
    for sz in sizes:
        e = sz // 3
        idx_parts.append(rng.integers(0, max(sz, 1), size=(e, 3)).astype(np.int32))
        eo.append(eo[-1] + e)
    idx = np.concatenate(idx_parts)
    eo = np.array(eo, np.int64)
    _say("batch with skipped passes", n, "vertices")
    for t in (None, (0, 0, 0, mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES), (0, 0, 0, SORT_ALL),
              (0, 0, 0, SORT_ALL | mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES)):
        res = mrx.reindex_mesh_batched(torch.from_numpy(vtx.view(np.int32)).to(DEV), torch.from_numpy(vo).to(DEV),
                                       torch.from_numpy(idx).to(DEV), torch.from_numpy(eo).to(DEV), tuning=t)
        ov, ooff, oi, o2n, n2o = oracle.reindex_batched(vtx, idx, vo, eo)
        assert np.array_equal(res.out_vtx_offsets.cpu().numpy(), ooff)
        assert np.array_equal(res.out_vtx.cpu().numpy().view(np.uint32), ov)
        assert np.array_equal(res.out_idx.cpu().numpy(), oi)
        assert np.array_equal(res.old2new.cpu().numpy(), o2n)
        assert np.array_equal(res.new2old.cpu().numpy(), n2o)


def test_cross_mesh_vertices_never_merge():
    import paper_2109_09812_amd as mrx
    one = meshgen.batched(1, 500, 501, 0.05, 31)
    m = one.mesh(0)
    # the same mesh three times: bitwise-equal vertices in every mesh
    vtx = np.concatenate([m.vtx] * 3)
    idx = np.concatenate([m.idx] * 3)
    n, e = m.num_vtx, m.idx.shape[0]
    b = meshgen.Batch(vtx, idx, np.arange(4, dtype=np.int64) * n, np.arange(4, dtype=np.int64) * e,
                      np.full(3, m.expected_unique), "triplicate")
    _say("triplicate batch")
    res = mrx.reindex_mesh_batched(*to_dev(b))
    check_batch(b, res)
    assert int(res.out_vtx_offsets[-1]) == 3 * m.expected_unique


def test_empty_meshes_inside_batch():
    import paper_2109_09812_amd as mrx
    parts = [meshgen.batched(1, 200, 201, 0.05, 40 + s).mesh(0) for s in range(3)]
    empty_v = np.zeros((0, 3), np.float32)
    empty_i = np.zeros((0, 3), np.int32)
    # meshes: [p0, empty, p1 with vertices but no elements, empty, p2]
    vs = [parts[0].vtx, empty_v, parts[1].vtx, empty_v, parts[2].vtx]
    is_ = [parts[0].idx, empty_i, empty_i, empty_i, parts[2].idx]
    vo = np.concatenate([[0], np.cumsum([v.shape[0] for v in vs])]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum([i.shape[0] for i in is_])]).astype(np.int64)
    exp = np.array([parts[0].expected_unique, 0, 0, 0, parts[2].expected_unique])
    b = meshgen.Batch(np.concatenate(vs), np.concatenate(is_), vo, eo, exp, "holes")
    _say("batch with empty meshes")
    res = mrx.reindex_mesh_batched(*to_dev(b))
    check_batch(b, res)


def test_batched_index_out_of_range():
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(5, 100, 1000, 0.05, 61)
    idx = b.idx.copy()
    # a local index equal to its own mesh's vertex count is out of range even
    # though it is a valid id of the packed array
    m2 = int(b.elem_offsets[2])
    idx[m2, 0] = int(b.vtx_offsets[3] - b.vtx_offsets[2])
    bb = meshgen.Batch(b.vtx, idx, b.vtx_offsets, b.elem_offsets, b.expected_unique, "bad")
    _say("batch out of range")
    with pytest.raises(IndexError):
        mrx.reindex_mesh_batched(*to_dev(bb))


@pytest.mark.parametrize("strategy", [None, (0, 0, 0, SORT_ALL)])
def test_graph_replays_with_new_contents(strategy):
    """Capture once, refill the inputs in place, replay; every replay must be
    exact (the per-call state is cleared by a kernel inside the graph)."""
    import paper_2109_09812_amd as mrx
    batches = [meshgen.batched(40, 100, 8000, 0.05, 70 + s) for s in range(3)]
    # same shapes: take the shape of the first batch and regenerate contents
    # by permuting each mesh's vertices (indices follow), mesh sizes unchanged
    base = batches[0]
    rng = np.random.default_rng(5)
    variants = [base]
    for _ in range(2):
        vtx = base.vtx.copy()
        idx = base.idx.copy()
        for m in range(base.num_meshes):
            v0, v1 = base.vtx_offsets[m], base.vtx_offsets[m + 1]
            e0, e1 = base.elem_offsets[m], base.elem_offsets[m + 1]
            p = rng.permutation(v1 - v0)
            inv = np.empty_like(p)
            inv[p] = np.arange(p.size)
            vtx[v0:v1] = base.vtx[v0:v1][p]
            idx[e0:e1] = inv[base.idx[e0:e1]]
        variants.append(meshgen.Batch(vtx, idx, base.vtx_offsets, base.elem_offsets,
                                      base.expected_unique, "perm"))
    tensors = to_dev(base)
    _say("capture graph", strategy)
    gr = mrx.GraphedBatchedReindexer(*tensors, tuning=strategy)
    for rep, b in enumerate(variants + [variants[1]]):
        _say("replay", rep)
        tensors[0].copy_(torch.from_numpy(np.ascontiguousarray(b.vtx).view(np.int32)))
        tensors[2].copy_(torch.from_numpy(b.idx))
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        check_batch(b, gr.result())
        # eager work between replays
        _ = (tensors[0].float() * 2).sum().item()


@pytest.mark.parametrize("strategy", [None, (0, 0, 0, SORT_ALL)])
def test_graph_replays_with_changing_skipped_passes(strategy):
    """The pass plan is worked out on the device in every replay: contents
    that alternate between records with several single-digit passes and
    records with none must all come out exact."""
    import paper_2109_09812_amd as mrx
    base = meshgen.batched(30, 100, 6000, 0.05, 88)
    rng = np.random.default_rng(9)
    n = base.vtx.shape[0]
    flat = np.full((n, 3), 0x3F000000, np.uint32)
    flat[:, 1] = rng.integers(0, 5, n).astype(np.uint32) << np.uint32(8)     # one live key pass
    few = meshgen.Batch(flat.view(np.float32), base.idx, base.vtx_offsets, base.elem_offsets, None, "few")
    tensors = to_dev(base)
    _say("capture graph (skipped passes)", strategy)
    gr = mrx.GraphedBatchedReindexer(*tensors, tuning=strategy)
    for rep, b in enumerate([few, base, few, base]):
        _say("replay", rep, b.name)
        tensors[0].copy_(torch.from_numpy(np.ascontiguousarray(b.vtx).view(np.int32)))
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        res = gr.result()
        ov, ooff, oi, o2n, n2o = oracle.reindex_batched(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
        assert np.array_equal(res.out_vtx_offsets.cpu().numpy(), ooff)
        assert np.array_equal(res.out_vtx.cpu().numpy().view(np.uint32), ov)
        assert np.array_equal(res.out_idx.cpu().numpy(), oi)
        assert np.array_equal(res.old2new.cpu().numpy(), o2n)
        assert np.array_equal(res.new2old.cpu().numpy(), n2o)
        _ = (tensors[0].float() * 2).sum().item()


def test_batched_tuning_flags():
    import paper_2109_09812_amd as mrx
    b = meshgen.batched(300, 100, 5000, 0.05, 616)
    for fl in (mrx.MRX_TUNING_WIDE_LOOKBACK, mrx.MRX_TUNING_CLAIMED_TILES,
               mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES):
        for strategy in (0, SORT_ALL):
            _say("batched flags", fl | strategy)
            check_batch(b, mrx.reindex_mesh_batched(*to_dev(b), tuning=(0, 0, 0, fl | strategy)))


def test_batched_all_tunings_and_autotune(tmp_path):
    import paper_2109_09812_amd as mrx
    from paper_2109_09812_amd import autotune
    b = meshgen.batched(50, 100, 6000, 0.05, 515)
    tensors = to_dev(b)
    for t in mrx.tunings(12):
        _say("batched tuning", t.as_tuple(), "sort all")
        check_batch(b, mrx.reindex_mesh_batched(*tensors, tuning=(*t.as_tuple(), SORT_ALL)))
    t, report = autotune.autotune(tensors[0], tensors[2], tensors[1], tensors[3], reps=2,
                                  path=str(tmp_path / "t.json"))
    check_batch(b, mrx.reindex_mesh_batched(*tensors, tuning=t))


def test_cfg4_full_batch():
    """The full 4096-mesh batch (~328M vertices) in one launch sequence:
    every mesh's output count matches its closed form, and every mesh
    matches the per-mesh oracle bit for bit (oracle calls spread over host
    threads; each call releases the interpreter lock). The default (hash
    grouping) is compared with the oracle, the sort-all path with it."""
    import concurrent.futures as cf
    import os
    import paper_2109_09812_amd as mrx
    _say("batch4096: generate")
    b = meshgen.cfg4()
    _say("batch4096: re-index", b.vtx.shape[0], "vertices")
    tensors = to_dev(b)
    res = mrx.reindex_mesh_batched(*tensors)
    _say("batch4096: re-index, sort all")
    other = mrx.reindex_mesh_batched(*tensors, tuning=(0, 0, 0, SORT_ALL))
    for name in ("out_vtx_offsets", "out_vtx", "out_idx", "old2new", "new2old"):
        assert torch.equal(getattr(res, name), getattr(other, name)), name
    del other, tensors
    offs = res.out_vtx_offsets.cpu().numpy()
    assert np.array_equal(np.diff(offs), b.expected_unique)
    ov_all = res.out_vtx.cpu().numpy().view(np.uint32)
    oi_all = res.out_idx.cpu().numpy()
    o2n_all = res.old2new.cpu().numpy()
    n2o_all = res.new2old.cpu().numpy()

    def one(mi):
        v0, v1 = int(b.vtx_offsets[mi]), int(b.vtx_offsets[mi + 1])
        e0, e1 = int(b.elem_offsets[mi]), int(b.elem_offsets[mi + 1])
        ov, oi, o2n, n2o = oracle.reindex(b.vtx[v0:v1], b.idx[e0:e1])
        return (np.array_equal(ov_all[offs[mi]:offs[mi + 1]], ov) and np.array_equal(oi_all[e0:e1], oi)
                and np.array_equal(o2n_all[v0:v1], o2n) and np.array_equal(n2o_all[offs[mi]:offs[mi + 1]], n2o))

    workers = max(1, min(16, os.cpu_count() or 1))
    _say("batch4096: per-mesh oracle on", workers, "threads")
    bad = []
    # largest meshes first so the pool drains evenly
    order = np.argsort(-np.diff(b.vtx_offsets), kind="stable")
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for done, (mi, ok) in enumerate(zip(order, ex.map(one, order.tolist())), 1):
            if not ok:
                bad.append(int(mi))
            if done % 512 == 0:
                _say("batch4096: oracle meshes checked", done)
    assert not bad, f"meshes differing from the oracle: {bad[:10]}"

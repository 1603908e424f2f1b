"""GPU parity of the hash-grouping path (records sorted by a few hash
digits, equal records grouped in on-chip memory, only the used values sorted
by their full key) against the oracle, bit for bit, next to the sort-all
path: small and ragged sizes, every record width, the flags, meshes whose
heavy duplicates overflow a hash bucket (the device falls back to sorting
everything), and the full-size workloads."""
import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
HASH = 8       # MRX_TUNING_HASH_GROUPS
SORT_ALL = 4   # MRX_TUNING_SORT_ALL
BANDS = 16     # MRX_TUNING_BANDS: Steps 1 and 4 by vertex bands at any size


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(vtx_np, idx_np, flags, tuning=(0, 0, 0)):
    import paper_2109_09812_amd as mrx
    v = torch.from_numpy(np.ascontiguousarray(vtx_np).view(np.int32)).to(DEV)
    i = torch.from_numpy(np.ascontiguousarray(idx_np, dtype=np.int32)).to(DEV)
    r = mrx.reindex_mesh(v, i, tuning=(*tuning, flags))
    torch.cuda.synchronize()
    return (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(), r.old2new.cpu().numpy(),
            r.new2old.cpu().numpy())


def check(vtx_np, idx_np, name, flags=HASH, tuning=(0, 0, 0)):
    _say(name, "N=%d E=%d A=%d flags=%d tuning=%s" % (vtx_np.shape[0], idx_np.shape[0], idx_np.shape[1], flags,
                                                      tuning))
    got = _run(vtx_np, idx_np, flags, tuning)
    exp = oracle.reindex(vtx_np, idx_np)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
        assert g.shape == e.shape, (name, label, g.shape, e.shape)
        assert np.array_equal(g, e), f"{name}: {label} differs at {np.argwhere(g != e)[:5].tolist()}"
    return got


def test_worked_example_and_tiny():
    x = np.array([1.0, 2.0, 3.0, 7.5, 4.0, 3.0, 5.0, 6.0, 8.5, 4.0], np.float32)
    vtx = np.stack([x, np.zeros_like(x)], 1)
    idx = np.array([[0, 1, 2], [0, 2, 4], [5, 6, 7], [5, 7, 9]], np.int32)
    ov, oi, o2n, n2o = check(vtx, idx, "worked example")
    assert o2n.tolist() == [0, 1, 2, -1, 3, 2, 4, 5, -1, 3]
    assert n2o.tolist() == [0, 1, 2, 4, 6, 7]
    for n in (1, 2, 3, 63, 64, 65, 511, 1365, 2047, 2048, 2049, 3071, 3072, 3073, 6145):
        vtx, idx = meshgen.random_mesh(n, max(1, n // 2), 3, 3, max(1, n // 3), 500 + n, 0.8)
        check(vtx, idx, f"tiny{n}")


def test_no_elements_and_all_unused():
    vtx = np.random.default_rng(0).random((70_000, 3), dtype=np.float32)
    got = check(vtx, np.zeros((0, 3), np.int32), "no elements")
    assert got[0].shape[0] == 0 and np.all(got[2] == -1)


FUZZ = [
    # n, words, arity, distinct, used_frac, seed
    (4095, 3, 3, 900, 0.9, 6), (4097, 3, 3, 4097, 0.6, 8), (8191, 2, 4, 3000, 0.9, 9),
    (8193, 5, 3, 2000, 0.9, 10), (12289, 8, 4, 5000, 0.97, 11), (20000, 12, 3, 700, 0.9, 12),
    (30001, 16, 2, 9000, 0.8, 13), (100_000, 3, 3, 30_000, 0.95, 14), (300_001, 3, 3, 60_000, 0.9, 15),
    (250_000, 1, 1, 1_000, 0.5, 16), (150_000, 2, 4, 150_000, 1.0, 17), (99_999, 7, 3, 20_000, 0.9, 18),
    (1_000_003, 3, 3, 170_000, 0.95, 19), (700_000, 4, 3, 700_000, 0.9, 20), (400_000, 6, 4, 90_000, 0.9, 21),
]


@pytest.mark.parametrize("n,k,a,d,u,seed", FUZZ)
def test_fuzz(n, k, a, d, u, seed):
    e = max(1, (n * 2) // (3 * a))
    vtx, idx = meshgen.random_mesh(n, e, a, k, d, 7000 + seed, u)
    check(vtx, idx, f"fuzz{seed}")


def test_every_record_width():
    rng = np.random.default_rng(17)
    for k in range(1, 17):
        n = int(rng.integers(60_000, 140_000))
        vtx, idx = meshgen.random_mesh(n, n // 3, 3, k, n // 5, 800 + k, 0.9)
        check(vtx, idx, f"width{k}")


def test_flags_and_tunings():
    import paper_2109_09812_amd as mrx
    m = meshgen.grid_soup(300, 0.05, 4321, "hashflags")
    for fl in (HASH | 1, HASH | 2, HASH | 3):
        check(m.vtx, m.idx, "soup300 flags", flags=fl)
    for t in mrx.tunings(12):
        check(m.vtx, m.idx, "soup300 tuning", flags=HASH, tuning=t.as_tuple())


def test_heavy_duplicates_fall_back():
    """A value with thousands of copies overflows its hash bucket's window:
    the device takes the sort-all path, with the identical result."""
    rng = np.random.default_rng(31)
    n = 200_000
    vtx = rng.random((n, 3), dtype=np.float32)
    heavy = rng.choice(n, 6000, replace=False)
    vtx[heavy] = vtx[heavy[0]]
    idx = rng.integers(0, n, size=(n // 3, 3)).astype(np.int32)
    check(vtx, idx, "heavy duplicates")
    check(np.ones((90_000, 3), np.float32), np.array([[5, 8000, 17]], np.int32), "identical")
    # an unreferenced heavy value among used ones
    vtx2 = vtx.copy()
    idx2 = idx.copy()
    idx2[np.isin(idx2, heavy)] = 7
    check(vtx2, idx2, "heavy unused")


def test_paper_quads_and_soups():
    for q in (256, 300):
        m = meshgen.paper_quads(q)
        got = check(m.vtx, m.idx, f"quads{q}")
        assert got[0].shape[0] == (q + 1) ** 2
    m = meshgen.cfg1()
    check(m.vtx, m.idx, "soup256")


def test_full_size_workloads():
    for name, make, u in (("tets64", meshgen.cfg3, 65 ** 3), ("soup10M", meshgen.cfg5_mesh, 1251 * 1281)):
        m = make()
        got = check(m.vtx, m.idx, name)
        assert got[0].shape[0] == u


def test_hash_and_sort_all_agree_on_soup2048():
    m = meshgen.cfg2()
    _say("soup2048 hash vs sort-all")
    a = _run(m.vtx, m.idx, HASH)
    b = _run(m.vtx, m.idx, SORT_ALL)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert a[0].shape[0] == 2048 * 2048


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


def test_graph_replays_switch_between_grouping_and_fallback():
    """One captured hash-grouping launch sequence replayed on contents that
    alternately group in LDS and overflow a bucket (a value with 6,000
    copies): the device picks the path on every replay, and every replay
    equals the oracle."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(4040)
    n = 120_000
    base = rng.random((n, 3), dtype=np.float32)
    idx_np = rng.integers(0, n, size=(n // 3, 3)).astype(np.int32)
    v = torch.from_numpy(base.view(np.int32).copy()).to(DEV)
    i = torch.from_numpy(idx_np).to(DEV)
    rx = mrx.Reindexer(v, i, tuning=(0, 0, 0, HASH))
    g = _capture(rx.launch)
    for rep in range(4):
        vtx = base.copy()
        if rep % 2:
            heavy = rng.choice(n, 6000, replace=False)
            vtx[heavy] = vtx[heavy[0]]
        else:
            vtx[rng.choice(n, n // 4, replace=False)] = vtx[rng.choice(n, n // 4)]
        v.copy_(torch.from_numpy(vtx.view(np.int32)))
        _say("graph replay", rep, "heavy" if rep % 2 else "grouped")
        g.replay()
        r = rx.result()
        got = (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(), r.old2new.cpu().numpy(),
               r.new2old.cpu().numpy())
        exp = oracle.reindex(vtx, idx_np)
        for label, gg, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
            assert np.array_equal(gg, e), f"replay {rep}: {label}"
        _ = (v.float() * 2).sum().item()


def test_band_marking_shapes():
    """Steps 1 and 4 by vertex bands (asked for at these sizes): ragged
    vertex counts around the band-size steps, entries crowded
    into one band (slices longer than a wave), an index array that is only
    4-byte aligned, a vertex that is never referenced at each band edge."""
    rng = np.random.default_rng(77)
    for n, m, lo_hi, name in ((70_000, 3 * 65_536, (0, 4096), "one band"),
                              (1_048_577, 3 * 400_000, None, "shift 13, ragged last band"),
                              (300_001, 3 * 30_000, None, "few entries per band"),
                              (262_144, 3 * 87_381 + 3, None, "ragged last tile")):
        vtx = rng.integers(0, 1 << 20, (n, 3), dtype=np.uint32).view(np.float32)
        vtx[rng.integers(0, n, n // 3)] = vtx[rng.integers(0, n, n // 3)]  # duplicates
        if lo_hi is None:
            idx = rng.integers(0, n, m, dtype=np.int64)
        else:
            idx = rng.integers(*lo_hi, m, dtype=np.int64)
        idx = idx.astype(np.int32)
        edges = np.arange(0, n, 4096)          # first vertex of each 4096-band: unused
        idx[np.isin(idx, edges)] = 1
        check(vtx, idx.reshape(-1, 3), name, flags=HASH | BANDS)
    # index array at a 4-byte (not 16-byte) offset
    n, m = 150_000, 3 * 40_000
    vtx = rng.random((n, 3), dtype=np.float32)
    flat = torch.from_numpy(rng.integers(0, n, m + 1, dtype=np.int64).astype(np.int32)).to(DEV)
    idx_dev = flat[1:].view(-1, 3)
    assert idx_dev.data_ptr() % 16 != 0
    import paper_2109_09812_amd as mrx
    _say("unaligned index array")
    r = mrx.reindex_mesh(torch.from_numpy(vtx.view(np.int32)).to(DEV), idx_dev, tuning=(0, 0, 0, HASH | BANDS))
    exp = oracle.reindex(vtx, flat[1:].cpu().numpy().reshape(-1, 3))
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"),
                           (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(),
                            r.old2new.cpu().numpy(), r.new2old.cpu().numpy()), exp):
        assert np.array_equal(g, e), label


@pytest.mark.parametrize("pos", [0, 8191, 8192, 3 * 70_000 - 1])
def test_band_marking_reports_bad_index(pos):
    """An out-of-range entry anywhere in a band-marked call (first and last
    entry of a tile, last entry) raises; a following call is unaffected."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(pos)
    n = 100_000
    vtx = rng.random((n, 3), dtype=np.float32)
    for bad in (-1, n, 2**31 - 1):
        idx = rng.integers(0, n, 3 * 70_000).astype(np.int32)
        idx[pos] = bad
        _say("bad index", bad, "at", pos)
        with pytest.raises(IndexError):
            mrx.reindex_mesh(torch.from_numpy(vtx.view(np.int32)).to(DEV),
                             torch.from_numpy(idx.reshape(-1, 3)).to(DEV), tuning=(0, 0, 0, HASH | BANDS))
    check(vtx, rng.integers(0, n, (70_000, 3)).astype(np.int32), "after the error", flags=HASH | BANDS)


def test_band_map_in_place_and_unaligned_old2new():
    """Step 4 by vertex bands writes out_idx over the index partition it kept
    there: in place (idx is out_idx) and into an old2new that is only 4-byte
    aligned (the band slices are then stored word by word)."""
    import ctypes

    import paper_2109_09812_amd as mrx
    from paper_2109_09812_amd import _lib
    m = meshgen.grid_soup(300, 0.05, 4242, "band-inplace")
    _say("band map in place", m.vtx.shape[0])
    v = torch.from_numpy(m.vtx.view(np.int32)).to(DEV)
    i = torch.from_numpy(m.idx).to(DEV)
    r = mrx.reindex_mesh(v, i.clone(), tuning=(0, 0, 0, HASH | BANDS), in_place=True)
    exp = oracle.reindex(m.vtx, m.idx)
    got = (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(), r.old2new.cpu().numpy(),
           r.new2old.cpu().numpy())
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
        assert np.array_equal(g, e), label
    _say("band map, old2new at a 4-byte offset")
    n, k = m.vtx.shape
    lib = _lib.load()
    out_vtx = torch.empty_like(v)
    out_idx = torch.empty_like(i)
    o2n_buf = torch.full((n + 4,), -7, dtype=torch.int32, device=DEV)
    n2o = torch.empty(n, dtype=torch.int32, device=DEV)
    meta = torch.zeros(2, dtype=torch.int64, device=DEV)
    tun = _lib.make_tuning((0, 0, 0, HASH | BANDS))
    wsb = mrx.workspace_size(n, 4 * k, i.numel(), 1, (0, 0, 0, HASH | BANDS))
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    o2n_ptr = o2n_buf.data_ptr() + 4
    assert o2n_ptr % 16 != 0
    st = lib.mrx_reindex_mesh(
        ctypes.c_void_p(v.data_ptr()), n, 4 * k, ctypes.c_void_p(i.data_ptr()), i.shape[0], i.shape[1],
        ctypes.c_void_p(out_vtx.data_ptr()), ctypes.c_void_p(out_idx.data_ptr()), ctypes.c_void_p(o2n_ptr),
        ctypes.c_void_p(n2o.data_ptr()), ctypes.c_void_p(meta.data_ptr()),
        ctypes.c_void_p(meta.data_ptr() + 8), ctypes.c_void_p(ws.data_ptr()), wsb, tun,
        ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    _lib.check(st, "mrx_reindex_mesh")
    torch.cuda.synchronize()
    assert int(meta[1]) == 0
    o2n = o2n_buf.cpu().numpy()
    assert o2n[0] == -7 and np.all(o2n[n + 1:] == -7)
    assert np.array_equal(o2n[1:n + 1], exp[2])
    assert np.array_equal(out_idx.cpu().numpy(), exp[1])


def test_band_marking_only_beyond_map_bands():
    """More than 2^25 vertices: the old2new slices of 2^15 vertices would
    need more bands than one table holds, so only the marking goes by
    (larger) bands and Step 4 scatters; compared with the parallel CPU
    re-indexer (itself pinned to the oracle) and with the sort-all path."""
    rng = np.random.default_rng(2025)
    n = 2**25 + 4099
    vtx = rng.integers(0, 1 << 22, (n, 1), dtype=np.uint32).view(np.float32)
    idx = rng.integers(0, n, (n - 12345, 1)).astype(np.int32)
    _say("band marking only, N =", n)
    got = _run(vtx, idx, HASH)
    exp = oracle.reindex_parallel(vtx, idx, threads=16)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
        assert np.array_equal(g, e), label
    other = _run(vtx, idx, SORT_ALL)
    for g, o in zip(got, other):
        assert np.array_equal(g, o)


def test_sort_all_path_by_bands():
    """Steps 1 and 4 by vertex bands on the sort-all path (asked for at these
    sizes): the pairs come from the flag scan's spare buffer, the partitions
    and new ids go into the sort buffers the plan leaves free; ragged band
    and tile edges, in place, extraction and merging."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(31)
    for n, m, name in ((70_000, 3 * 65_536, "sort-all bands, few vertices"),
                       (1_048_577, 3 * 400_000, "sort-all bands, shift 13"),
                       (262_144, 3 * 87_381 + 3, "sort-all bands, ragged last tile")):
        vtx = rng.integers(0, 1 << 20, (n, 3), dtype=np.uint32).view(np.float32)
        vtx[rng.integers(0, n, n // 3)] = vtx[rng.integers(0, n, n // 3)]
        idx = rng.integers(0, n, m).astype(np.int32).reshape(-1, 3)
        check(vtx, idx, name, flags=SORT_ALL | BANDS)
    m = meshgen.grid_soup(300, 0.05, 77, "sa-inplace")
    _say("sort-all bands in place")
    r = mrx.reindex_mesh(torch.from_numpy(m.vtx.view(np.int32)).to(DEV), torch.from_numpy(m.idx).to(DEV),
                         tuning=(0, 0, 0, SORT_ALL | BANDS), in_place=True)
    exp = oracle.reindex(m.vtx, m.idx)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"),
                           (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(),
                            r.old2new.cpu().numpy(), r.new2old.cpu().numpy()), exp):
        assert np.array_equal(g, e), label
    keep = rng.random(m.idx.shape[0]) < 0.4
    _say("sort-all bands extract")
    x = mrx.extract_submesh(torch.from_numpy(m.vtx.view(np.int32)).to(DEV), torch.from_numpy(m.idx).to(DEV),
                            torch.from_numpy(keep).to(DEV), tuning=(0, 0, 0, SORT_ALL | BANDS))
    ex = oracle.extract(m.vtx, m.idx, keep)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"),
                           (x.out_vtx.cpu().numpy().view(np.uint32), x.out_idx.cpu().numpy(),
                            x.old2new.cpu().numpy(), x.new2old.cpu().numpy()), ex):
        assert np.array_equal(g, e), label
    b = meshgen.batched(30, 100, 8000, 0.05, 4040)
    _say("sort-all bands merge")
    got = mrx.merge_meshes(torch.from_numpy(np.ascontiguousarray(b.vtx).view(np.int32)).to(DEV),
                           torch.from_numpy(b.vtx_offsets).to(DEV),
                           torch.from_numpy(np.ascontiguousarray(b.idx, dtype=np.int32)).to(DEV),
                           torch.from_numpy(b.elem_offsets).to(DEV), tuning=(0, 0, 0, SORT_ALL | BANDS))
    me = oracle.merge(b.vtx, b.idx, b.vtx_offsets, b.elem_offsets)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"),
                           (got.out_vtx.cpu().numpy().view(np.uint32), got.out_idx.cpu().numpy(),
                            got.old2new.cpu().numpy(), got.new2old.cpu().numpy()), me):
        assert np.array_equal(g, e), label

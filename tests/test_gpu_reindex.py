"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, bit for bit."""
import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle
from helpers import check_properties, words

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def to_dev(vtx_np, idx_np):
    v = torch.from_numpy(np.ascontiguousarray(vtx_np).view(np.int32)).to(DEV)
    i = torch.from_numpy(np.ascontiguousarray(idx_np, dtype=np.int32)).to(DEV)
    return v, i


def gpu(vtx_np, idx_np, tuning=None, in_place=False):
    import paper_2109_09812_amd as mrx
    v, i = to_dev(vtx_np, idx_np)
    r = mrx.reindex_mesh(v, i, tuning=tuning, in_place=in_place)
    torch.cuda.synchronize()
    return (r.out_vtx.cpu().numpy().view(np.uint32), r.out_idx.cpu().numpy(), r.old2new.cpu().numpy(),
            r.new2old.cpu().numpy())


def assert_parity(vtx_np, idx_np, tuning=None, name=""):
    _say(name, "N=%d K=%d E=%d A=%d" % (vtx_np.shape[0], words(vtx_np).shape[1] if vtx_np.size else 0,
                                        idx_np.shape[0], idx_np.shape[1]), "tuning", tuning)
    got = gpu(vtx_np, idx_np, tuning)
    exp = oracle.reindex(vtx_np, idx_np)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
        assert g.shape == e.shape, (label, g.shape, e.shape)
        assert np.array_equal(g, e), f"{name}: {label} differs at {np.argwhere(g != e)[:5].tolist()}"
    return got


def test_worked_example():
    x = np.array([1.0, 2.0, 3.0, 7.5, 4.0, 3.0, 5.0, 6.0, 8.5, 4.0], np.float32)
    vtx = np.stack([x, np.zeros_like(x)], 1)
    idx = np.array([[0, 1, 2], [0, 2, 4], [5, 6, 7], [5, 7, 9]], np.int32)
    ov, oi, o2n, n2o = assert_parity(vtx, idx, name="worked example")
    assert oi.tolist() == [[0, 1, 2], [0, 2, 3], [2, 4, 5], [2, 5, 3]]
    assert o2n.tolist() == [0, 1, 2, -1, 3, 2, 4, 5, -1, 3]
    assert n2o.tolist() == [0, 1, 2, 4, 6, 7]


def test_cfg1_soup256():
    m = meshgen.cfg1()
    got = assert_parity(m.vtx, m.idx, name="soup256")
    assert got[0].shape[0] == 65536


FUZZ = [
    # n, words, arity, distinct, used_frac, seed
    (1, 3, 3, 1, 1.0, 1), (2, 3, 1, 2, 1.0, 2), (63, 2, 3, 20, 0.8, 3), (64, 1, 2, 64, 0.5, 4),
    (65, 4, 4, 10, 1.0, 5), (4095, 3, 3, 900, 0.9, 6), (4096, 3, 3, 1000, 0.7, 7),
    (4097, 3, 3, 4097, 0.6, 8), (8191, 2, 4, 3000, 0.9, 9), (8193, 5, 3, 2000, 0.9, 10),
    (12289, 8, 4, 5000, 0.97, 11), (20000, 12, 3, 700, 0.9, 12), (30001, 16, 2, 9000, 0.8, 13),
    (100_000, 3, 3, 30_000, 0.95, 14), (300_001, 3, 3, 60_000, 0.9, 15), (250_000, 1, 1, 1_000, 0.5, 16),
    (150_000, 2, 4, 150_000, 1.0, 17), (99_999, 7, 3, 20_000, 0.9, 18),
]


@pytest.mark.parametrize("n,k,a,d,u,seed", FUZZ)
def test_fuzz_parity(n, k, a, d, u, seed):
    e = max(1, (n * 2) // (3 * a))
    vtx, idx = meshgen.random_mesh(n, e, a, k, d, 7000 + seed, u)
    assert_parity(vtx, idx, name=f"fuzz{seed}")


def test_empty_and_degenerate():
    import paper_2109_09812_amd as mrx
    _say("empty mesh")
    v, i = to_dev(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    r = mrx.reindex_mesh(v, i)
    assert r.num_out == 0 and r.out_vtx.shape == (0, 3) and r.old2new.numel() == 0
    # vertices but no elements: nothing is used
    vtx = np.random.default_rng(0).random((5000, 3), dtype=np.float32)
    got = assert_parity(vtx, np.zeros((0, 3), np.int32), name="no elements")
    assert got[0].shape[0] == 0 and np.all(got[2] == -1)
    # all vertices identical
    assert_parity(np.ones((9000, 3), np.float32), np.array([[5, 8000, 17]], np.int32), name="identical")
    # signed zeros and NaN payloads
    w = np.array([[0x80000000], [0], [0x7FC00000], [0x7FC00001], [0x7FC00000], [0x80000000]], np.uint32)
    got = assert_parity(w, np.arange(6, dtype=np.int32).reshape(6, 1), name="zeros/nan")
    assert got[0].reshape(-1).tolist() == [0, 0x7FC00000, 0x7FC00001, 0x80000000]


def test_sorted_reverse_and_single_digit_inputs():
    n = 70_000
    k = np.arange(n, dtype=np.uint32)
    asc = np.stack([k // 7, k % 7, k], 1).astype(np.uint32)
    idx = np.arange(n, dtype=np.int32).reshape(-1, 1)
    assert_parity(asc, idx, name="ascending")
    assert_parity(asc[::-1].copy(), idx, name="descending")
    # keys that differ only in one byte of one word: every other digit pass sees one bucket
    one = np.zeros((n, 3), np.uint32)
    one[:, 1] = (np.random.default_rng(3).integers(0, 256, n).astype(np.uint32) << 16)
    assert_parity(one, (np.arange(n, dtype=np.int32) % n).reshape(-1, 2)[: n // 2], name="one byte")


def test_out_of_range_index_reported():
    import paper_2109_09812_amd as mrx
    vtx = np.random.default_rng(1).random((1000, 3), dtype=np.float32)
    for bad in (-1, 1000, 2**31 - 1):
        idx = np.arange(300, dtype=np.int32).reshape(100, 3)
        idx[57, 1] = bad
        _say("out of range", bad)
        v, i = to_dev(vtx, idx)
        with pytest.raises(IndexError):
            mrx.reindex_mesh(v, i)
    _say("no vertices, one element")
    v, i = to_dev(np.zeros((0, 3), np.float32), np.zeros((1, 3), np.int32))
    with pytest.raises(IndexError):
        mrx.reindex_mesh(v, i)
    # a later valid call on fresh outputs is unaffected
    assert_parity(vtx, np.arange(300, dtype=np.int32).reshape(100, 3), name="after error")


def test_in_place_remap():
    m = meshgen.grid_soup(100, 0.05, 99, "inplace")
    _say("in place")
    got = gpu(m.vtx, m.idx, in_place=True)
    exp = oracle.reindex(m.vtx, m.idx)
    for g, e in zip(got, exp):
        assert np.array_equal(g, e)


def test_repeat_determinism_and_all_tunings():
    import paper_2109_09812_amd as mrx
    m = meshgen.grid_soup(300, 0.07, 1234, "tune")
    exp = oracle.reindex(m.vtx, m.idx)
    for t in mrx.tunings(12):
        for rep in range(2):
            _say("tuning", t.as_tuple(), "rep", rep)
            got = gpu(m.vtx, m.idx, tuning=t)
            for g, e in zip(got, exp):
                assert np.array_equal(g, e)


def test_wide_records_all_tunings():
    import paper_2109_09812_amd as mrx
    m = meshgen.tet_mesh(12, 0.03, 55)
    exp = oracle.reindex(m.vtx, m.idx)
    assert exp[0].shape[0] == 13 ** 3
    for t in mrx.tunings(32):
        _say("tets tuning", t.as_tuple())
        got = gpu(m.vtx, m.idx, tuning=t)
        for g, e in zip(got, exp):
            assert np.array_equal(g, e)


def test_every_record_width_every_tuning():
    """Records of 1-16 words, every compiled variant of each width, on meshes
    of several tiles with a ragged tail, sorting all and with hash grouping.
    Narrow records (up to 4 words) run the used marking and digit histograms
    as one launch, wider ones as two; the lopsided shapes give that launch
    almost only histogram tiles, or almost only marking tiles."""
    import paper_2109_09812_amd as mrx
    for k in range(1, 17):
        vtx, idx = meshgen.random_mesh(20_011 + 97 * k, 7_001, 3, k, 2_500, 4_700 + k, 0.9)
        for t in mrx.tunings(4 * k):
            for strategy in (mrx.MRX_TUNING_SORT_ALL, mrx.MRX_TUNING_HASH_GROUPS):
                assert_parity(vtx, idx, tuning=(*t.as_tuple(), strategy), name=f"width {k}")
    for k in (2, 3, 5):
        assert_parity(*meshgen.random_mesh(300_007, 1, 3, k, 40_000, 4_800 + k), name=f"one element {k}")
        assert_parity(*meshgen.random_mesh(37, 200_003, 3, k, 20, 4_900 + k), name=f"many elements {k}")


def _few_live_bytes(n, live, rng):
    """Records of three words, all equal except the byte of each LSD pass in
    ``live`` (pass p = byte p % 4 of word 2 - p // 4), which takes 7 values."""
    vtx = np.full((n, 3), 0x3F000000, np.uint32)
    for p in live:
        word, shift = 2 - p // 4, 8 * (p % 4)
        vtx[:, word] &= np.uint32(~(0xFF << shift) & 0xFFFFFFFF)
        vtx[:, word] |= rng.integers(0, 7, n).astype(np.uint32) << np.uint32(shift)
    return vtx


def test_single_digit_passes_are_skipped():
    """A pass whose digit is the same for every record moves nothing; the
    element buffers then alternate on the device. One, two and three live
    passes (odd and even numbers skipped), the last pass alone, only the
    first, every record equal; each under every look-back and tile-order
    flag."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(77)
    n = 50_003
    idx = rng.integers(0, n, size=(20_000, 3)).astype(np.int32)
    both = mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES
    flag_sets = (0, mrx.MRX_TUNING_WIDE_LOOKBACK, mrx.MRX_TUNING_CLAIMED_TILES, both)
    for live in ([6], [2, 9], [1, 5, 10], [11], [0], []):
        vtx = _few_live_bytes(n, live, rng)
        for fl in flag_sets:
            assert_parity(vtx, idx, tuning=(0, 0, 0, fl), name=f"live passes {live} flags {fl}")


def test_tuning_flags_match():
    """64-bit look-back words (forced here; automatic from 2^30 vertices on),
    counter-claimed tiles and Steps 1 and 4 by vertex bands (forced here;
    automatic from 2^20 index entries on) give the same result as the
    defaults, in every variant."""
    import paper_2109_09812_amd as mrx
    m = meshgen.grid_soup(300, 0.07, 4321, "wide")
    exp = oracle.reindex(m.vtx, m.idx)
    flag_sets = (mrx.MRX_TUNING_WIDE_LOOKBACK, mrx.MRX_TUNING_CLAIMED_TILES,
                 mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES,
                 mrx.MRX_TUNING_BANDS | mrx.MRX_TUNING_WIDE_LOOKBACK | mrx.MRX_TUNING_CLAIMED_TILES)
    for t in mrx.tunings(12):
        for fl in flag_sets:
            shape = t.as_tuple()
            _say("flags", fl, shape)
            got = gpu(m.vtx, m.idx, tuning=(*shape, fl))
            for g, e in zip(got, exp):
                assert np.array_equal(g, e)
    for fl in flag_sets:
        assert_parity(*meshgen.random_mesh(70_001, 30_000, 3, 8, 9_000, 9191, 0.9),
                      tuning=(0, 0, 0, fl), name=f"flags {fl} K=8")


def test_tet_seam_does_not_merge():
    m = meshgen.tet_mesh(16, 0.03, 77, seam=True)
    got = assert_parity(m.vtx, m.idx, name="seam")
    assert got[0].shape[0] == m.expected_unique


def test_paper_quads():
    # 256 (a power of two: the low byte of every coordinate is zero, a pass is
    # skipped) and 300 (no such byte)
    for q in (256, 300):
        m = meshgen.paper_quads(q)
        got = assert_parity(m.vtx, m.idx, name=f"quads{q}")
        assert got[0].shape[0] == (q + 1) ** 2


SORT_ALL = (0, 0, 0, 4)   # MRX_TUNING_SORT_ALL: Section 2's sort of every vertex


def test_cfg3_tets_full():
    m = meshgen.cfg3()
    for t in (None, SORT_ALL):
        got = assert_parity(m.vtx, m.idx, tuning=t, name="tets64")
        assert got[0].shape[0] == 65 ** 3


def test_cfg5_soup10m_full():
    m = meshgen.cfg5_mesh()
    for t in (None, SORT_ALL):
        got = assert_parity(m.vtx, m.idx, tuning=t, name="soup10M")
        assert got[0].shape[0] == 1251 * 1281


def test_cfg2_soup2048_full():
    """The 26.4M-vertex soup at full size, in the default launch
    configuration: all four outputs equal the oracle's element by element,
    and the properties that fix the result hold."""
    m = meshgen.cfg2()
    _say("soup2048 full size: GPU")
    got = gpu(m.vtx, m.idx)
    _say("soup2048 full size: properties")
    check_properties(m.vtx, m.idx, *got, expected_unique=2048 * 2048)
    _say("soup2048 full size: oracle (about a minute on one host core)")
    exp = oracle.reindex(m.vtx, m.idx)
    for label, g, e in zip(("out_vtx", "out_idx", "old2new", "new2old"), got, exp):
        assert g.shape == e.shape, (label, g.shape, e.shape)
        assert np.array_equal(g, e), f"soup2048: {label} differs at {np.argwhere(g != e)[:5].tolist()}"


def test_autotune_picks_a_verified_variant(tmp_path):
    """The tuner runs every compiled variant, checks each against variant 0
    bit for bit, and its choice reproduces the oracle's result."""
    import paper_2109_09812_amd as mrx
    from paper_2109_09812_amd import autotune
    m = meshgen.grid_soup(400, 0.05, 4242, "tune")
    v, i = to_dev(m.vtx, m.idx)
    _say("autotune")
    t, report = autotune.autotune(v, i, reps=2, path=str(tmp_path / "t.json"))
    assert t.as_key() in report and len(report) == 2 * len(mrx.tunings(12))
    t2, rep2 = autotune.autotune(v, i, reps=2, path=str(tmp_path / "t.json"))
    assert t2.as_key() == t.as_key() and "cached" in rep2
    got = gpu(m.vtx, m.idx, tuning=t)
    exp = oracle.reindex(m.vtx, m.idx)
    for g, e in zip(got, exp):
        assert np.array_equal(g, e)

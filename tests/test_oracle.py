"""Pins for the CPU oracle (no GPU).

Each check ties the std::map oracle to something other than itself: the
arrays the paper prints for its worked example, a re-enactment of the paper's
Steps 1-4, an O(n^2) brute force, numpy.unique, closed-form vertex counts and
invariants. ``test_oracle_mutants`` plants plausible mistakes in a copy of
the oracle and checks that these pins catch every one.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import meshgen
import oracle
from oracle import bruteforce, paper_steps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
LETTER_X = {"A": 1.0, "B": 2.0, "C": 3.0, "D": 4.0, "E": 5.0, "F": 6.0, "X": 7.5, "Y": 8.5}


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _example():
    g = _golden()
    x = np.array(g["x"], dtype=np.float32)
    vtx = np.stack([x, np.zeros_like(x)], axis=1)
    idx = np.array(g["idx"], dtype=np.int32)
    return vtx, idx, g


def _letters_to_words(letters):
    x = np.array([LETTER_X[c] for c in letters], dtype=np.float32)
    return np.stack([x, np.zeros_like(x)], axis=1).view(np.uint32)


# ----------------------------------------------------------------- worked example

def test_worked_example_oracle_golden():
    vtx, idx, g = _example()
    ov, oi, o2n, n2o = oracle.reindex(vtx, idx)
    exp = g["expected_oracle"]
    assert ov.shape[0] == exp["num_out"] == g["printed"]["newN"]["value"]
    assert np.array_equal(ov.view(np.float32)[:, 0], np.array(exp["out_x"], np.float32))
    assert np.array_equal(oi, np.array(exp["out_idx"]))
    assert np.array_equal(oi, np.array(g["printed"]["idx_new"]["value"]))
    assert np.array_equal(o2n, np.array(exp["old2new"]))
    assert np.array_equal(n2o, np.array(exp["new2old"]))
    assert np.array_equal(ov, _letters_to_words(g["printed"]["newVtx"]["value"]))


def test_worked_example_paper_steps_reproduce_printed_arrays():
    vtx, idx, g = _example()
    p = g["printed"]
    r = paper_steps.run(vtx, idx)
    assert np.array_equal(r["isUsed"].astype(int), p["isUsed"]["value"])
    assert np.array_equal(r["vtx_cleaned"], _letters_to_words(p["vtx_after_overwrite"]["value"]))
    assert np.array_equal(r["vtx_sorted"], _letters_to_words(p["vtx_sorted"]["value"]))
    assert np.array_equal(r["nodup"], p["nodup"]["value"])
    assert np.array_equal(r["newIdx_postfix"], p["newIdx_postfix"]["value"])
    assert np.array_equal(r["newIdx"], p["newIdx"]["value"])
    assert r["newN"] == p["newN"]["value"]
    assert np.array_equal(r["newVtx"], _letters_to_words(p["newVtx"]["value"]))
    assert np.array_equal(r["idx_new"], p["idx_new"]["value"])
    # a stable sort keeps equal keys in original-id order
    assert list(r["orgID"]) == [0, 3, 8, 1, 2, 5, 4, 9, 6, 7]


def test_worked_example_paper_tie_order_gives_printed_perm():
    vtx, idx, g = _example()
    p = g["printed"]
    order = p["orgID_sorted_corrected"]["value"]
    r = paper_steps.run(vtx, idx, sort_order=order)
    assert np.array_equal(r["perm"], p["perm"]["value"])
    # the printed perm is exactly the inverse of the corrected sorted orgID
    perm = np.array(p["perm"]["value"])
    assert np.array_equal(perm[np.array(order)], np.arange(10))
    assert np.array_equal(r["idx_new"], p["idx_new"]["value"])


# ----------------------------------------------------------------- cross-checks

def _fuzz_cases(count, max_n=120):
    rng = np.random.default_rng(7)
    for s in range(count):
        n = int(rng.integers(1, max_n))
        words = int(rng.integers(1, 6))
        arity = int(rng.integers(1, 5))
        e = int(rng.integers(1, max(2, n // 2)))
        distinct = int(rng.integers(1, max(2, n)))
        used = float(rng.uniform(0.2, 1.0))
        vtx, idx = meshgen.random_mesh(n, e, arity, words, distinct, 1000 + s, used)
        yield vtx, idx


def test_oracle_matches_bruteforce_on_tiny_meshes():
    for vtx, idx in _fuzz_cases(250):
        a = oracle.reindex(vtx, idx)
        b = bruteforce.reindex(vtx, idx)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_oracle_matches_paper_steps_on_tiny_meshes():
    """The paper's Steps 1-4 give the same compact vertices and the same new
    indices; they differ only where the paper leaves the choice open (which
    copy represents a value, and where unreferenced vertices point)."""
    for vtx, idx in _fuzz_cases(120, max_n=80):
        ov, oi, o2n, n2o = oracle.reindex(vtx, idx)
        r = paper_steps.run(vtx, idx)
        assert np.array_equal(ov, r["newVtx"])
        assert np.array_equal(oi, r["idx_new"])
        # Step 1 overwrites every unreferenced vertex, so only referenced
        # vertices keep their own value in the paper's walk-through.
        ref = r["isUsed"]
        assert np.array_equal(o2n[ref], r["old2new"][ref])


def _numpy_reindex(vtx, idx):
    """Sorted unique rows with first-occurrence index and inverse, then a
    used filter: the library special case of the sort/flag/scan steps."""
    w = np.ascontiguousarray(vtx).view(np.uint32)
    uniq, first, inv = np.unique(w, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    used_g = np.zeros(uniq.shape[0], dtype=bool)
    used_g[inv[idx.reshape(-1)]] = True
    cid = np.cumsum(used_g) - 1
    gmap = np.where(used_g, cid, -1)
    old2new = gmap[inv].astype(np.int32)
    return uniq[used_g], old2new[idx].astype(np.int32), old2new, first[used_g].astype(np.int32)


def test_oracle_matches_numpy_unique():
    for s, (n, k, e, a, d) in enumerate([(20000, 3, 6000, 3, 5000), (50000, 2, 10000, 4, 40000),
                                         (30000, 8, 7000, 4, 3000), (10000, 1, 9000, 1, 100),
                                         (5000, 16, 1000, 3, 2000)]):
        vtx, idx = meshgen.random_mesh(n, e, a, k, d, 500 + s, 0.7)
        got = oracle.reindex(vtx, idx)
        exp = _numpy_reindex(vtx, idx)
        for x, y in zip(got, exp):
            assert np.array_equal(x, y)


# ----------------------------------------------------------------- closed forms & invariants

def check_invariants(vtx, idx, out_vtx, out_idx, old2new, new2old):
    """Properties that hold at any size (Section 2, 'Checking our Example')."""
    w = np.ascontiguousarray(vtx).view(np.uint32).reshape(vtx.shape[0], -1)
    ow = np.ascontiguousarray(out_vtx).view(np.uint32).reshape(out_vtx.shape[0], -1)
    u = ow.shape[0]
    # same elements, bitwise
    assert np.array_equal(ow[out_idx.reshape(-1)], w[idx.reshape(-1)])
    # strictly ascending output (unsigned word tuples)
    if u > 1:
        order = np.lexsort(tuple(ow[:, c] for c in range(ow.shape[1] - 1, -1, -1)))
        assert np.array_equal(order, np.arange(u))
        assert not np.any(np.all(ow[1:] == ow[:-1], axis=1))
    # every output vertex referenced
    ref = np.zeros(u, dtype=bool)
    ref[out_idx.reshape(-1)] = True
    assert ref.all()
    # maps are consistent
    assert np.array_equal(old2new[new2old], np.arange(u))
    assert np.array_equal(ow, w[new2old])
    mapped = old2new >= 0
    assert np.array_equal(w[mapped], ow[old2new[mapped]])


def test_cfg1_closed_form_and_invariants():
    m = meshgen.cfg1()
    res = oracle.reindex(m.vtx, m.idx)
    assert res[0].shape[0] == m.expected_unique == 256 * 256
    check_invariants(m.vtx, m.idx, *res)
    # the representative is the smallest original id among equal copies
    w = m.vtx.view(np.uint32)
    _, first, inv = np.unique(w, axis=0, return_index=True, return_inverse=True)
    assert np.array_equal(res[3], first[inv.reshape(-1)[res[3]]])
    # unused copies of used values map to their value; others to -1
    assert (res[2] == -1).sum() == m.num_vtx - 3 * m.idx.shape[0]


@pytest.mark.parametrize("n,expected", [(7, 64), (8, 81), (64, 4225), (100, 10201)])
def test_paper_quads_closed_form(n, expected):
    """Table 1: out = (N+1)^2 for the N x N quad generator."""
    m = meshgen.paper_quads(n)
    assert m.num_vtx == 5 * n * n
    res = oracle.reindex(m.vtx, m.idx)
    assert res[0].shape[0] == expected == (n + 1) ** 2
    check_invariants(m.vtx, m.idx, *res)


def test_tets_closed_form_and_seam():
    m = meshgen.tet_mesh(8, 0.03, 11)
    res = oracle.reindex(m.vtx, m.idx)
    assert res[0].shape[0] == 9 ** 3
    check_invariants(m.vtx, m.idx, *res)
    s = meshgen.tet_mesh(8, 0.03, 12, seam=True)
    res = oracle.reindex(s.vtx, s.idx)
    # positions on the seam plane appear twice (different normals): they must not merge
    assert res[0].shape[0] == s.expected_unique == 9 ** 3 + 9 * 9


# ----------------------------------------------------------------- edge cases

def test_empty_inputs():
    ov, oi, o2n, n2o = oracle.reindex(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32))
    assert ov.shape == (0, 3) and oi.shape == (0, 3) and o2n.shape == (0,) and n2o.shape == (0,)
    vtx = np.arange(12, dtype=np.float32).reshape(4, 3)
    ov, oi, o2n, n2o = oracle.reindex(vtx, np.zeros((0, 3), np.int32))
    assert ov.shape[0] == 0 and np.all(o2n == -1)
    with pytest.raises(oracle.OracleIndexError):
        oracle.reindex(np.zeros((0, 3), np.float32), np.zeros((1, 3), np.int32))


def test_out_of_range_reports_first_position():
    vtx = np.arange(12, dtype=np.float32).reshape(4, 3)
    idx = np.array([[0, 1, 2], [3, 4, 1], [-1, 0, 0]], dtype=np.int32)
    with pytest.raises(oracle.OracleIndexError) as e:
        oracle.reindex(vtx, idx)
    assert e.value.pos == 4
    with pytest.raises(oracle.OracleIndexError) as e:
        oracle.reindex(vtx, np.array([[0], [-1]], np.int32))
    assert e.value.pos == 1


def test_all_identical_and_signed_zero_and_nan_payloads():
    vtx = np.ones((50, 3), np.float32)
    ov, oi, o2n, n2o = oracle.reindex(vtx, np.array([[7, 3, 49]], np.int32))
    assert ov.shape[0] == 1 and np.all(o2n == 0) and list(n2o) == [0] and np.all(oi == 0)
    words = np.array([[0x80000000], [0x00000000], [0x7FC00000], [0x7FC00001], [0x7FC00000],
                      [0x80000000]], dtype=np.uint32)
    ov, oi, o2n, n2o = oracle.reindex(words, np.arange(6, dtype=np.int32).reshape(6, 1))
    # +0 < NaN(0x7FC00000) < NaN(0x7FC00001) < -0 as unsigned words; equal payloads merge
    assert list(ov.reshape(-1)) == [0x00000000, 0x7FC00000, 0x7FC00001, 0x80000000]
    assert list(o2n) == [3, 0, 1, 2, 1, 3]
    assert list(n2o) == [1, 2, 3, 0]


def test_word_order_is_unsigned_lexicographic():
    words = np.array([[1, 0xFFFFFFFF], [2, 0], [1, 0], [0xFFFFFFFF, 5]], dtype=np.uint32)
    ov, oi, o2n, n2o = oracle.reindex(words, np.arange(4, dtype=np.int32).reshape(2, 2))
    assert [tuple(r) for r in ov] == [(1, 0), (1, 0xFFFFFFFF), (2, 0), (0xFFFFFFFF, 5)]


@pytest.mark.parametrize("k", list(range(1, 17)))
def test_all_record_widths(k):
    vtx, idx = meshgen.random_mesh(300, 80, 3, k, 60, 90 + k, 0.6)
    got = oracle.reindex(vtx, idx)
    exp = bruteforce.reindex(vtx, idx)
    for x, y in zip(got, exp):
        assert np.array_equal(x, y)


# ----------------------------------------------------------------- mutation check

MUTANTS = {
    "last copy represents": ("groups.emplace(key_of(vtx, i, words), Group{(int32_t)i, false, -1});",
                             "groups[key_of(vtx, i, words)] = Group{(int32_t)i, false, -1};"),
    "signed word compare": ("using Key = std::array<uint32_t, kMaxWords>;",
                            "using Key = std::array<int32_t, kMaxWords>;"),
    "word 0 least significant": ("k[w] = vtx[i * words + w];",
                                 "k[words - 1 - w] = vtx[i * words + w];"),
    "unused values kept": ("if (!g.used) continue;", ""),
    "only the representative maps": ("old2new[i] = groups.at(key_of(vtx, i, words)).new_id;",
                                     "old2new[i] = groups.at(key_of(vtx, i, words)).rep == (int32_t)i"
                                     " ? groups.at(key_of(vtx, i, words)).new_id : -1;"),
    "index bound off by one": ("idx[k] >= num_vtx", "idx[k] > num_vtx"),
    "new ids off by one": ("g.new_id = (int32_t)u;", "g.new_id = (int32_t)u + (u > 0);"),
}


def _pins_pass(lib_path):
    saved = oracle._lib
    oracle._lib = None
    real_path = oracle._LIB_PATH
    try:
        oracle._LIB_PATH = lib_path
        for t in (test_worked_example_oracle_golden, test_word_order_is_unsigned_lexicographic,
                  test_all_identical_and_signed_zero_and_nan_payloads, test_out_of_range_reports_first_position):
            t()
        for vtx, idx in _fuzz_cases(40, max_n=60):
            a = oracle.reindex(vtx, idx)
            b = bruteforce.reindex(vtx, idx)
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        m = meshgen.paper_quads(8)
        assert oracle.reindex(m.vtx, m.idx)[0].shape[0] == 81
        return True
    except (AssertionError, IndexError, ValueError):
        return False
    finally:
        oracle._LIB_PATH = real_path
        oracle._lib = saved


# ----------------------------------------------------------------- merge (Section 3)

def _merge_cases(count, seed=77):
    """Tiny packed batches whose meshes draw records from one shared pool, so
    equal vertices occur inside and across meshes."""
    rng = np.random.default_rng(seed)
    for c in range(count):
        words = int(rng.integers(1, 4))
        pool = rng.integers(0, 6, size=(int(rng.integers(1, 12)), words)).astype(np.uint32)
        meshes = []
        for _ in range(int(rng.integers(1, 5))):
            n = int(rng.integers(0, 25))
            e = int(rng.integers(0, 12)) if n else 0
            v = pool[rng.integers(0, pool.shape[0], size=n)] if n else np.zeros((0, words), np.uint32)
            i = rng.integers(0, n, size=(e, 3)).astype(np.int32) if e else np.zeros((0, 3), np.int32)
            meshes.append((v, i))
        vo = np.concatenate([[0], np.cumsum([m[0].shape[0] for m in meshes])]).astype(np.int64)
        eo = np.concatenate([[0], np.cumsum([m[1].shape[0] for m in meshes])]).astype(np.int64)
        vtx = np.concatenate([m[0] for m in meshes]).reshape(-1, words)
        idx = np.concatenate([m[1] for m in meshes]).reshape(-1, 3)
        yield meshes, vtx, idx, vo, eo


def test_merge_matches_bruteforce_of_the_concatenation():
    for meshes, vtx, idx, vo, eo in _merge_cases(120):
        # global indices built element by element, independently of merge()
        glob = []
        base = 0
        for v, i in meshes:
            for row in i.tolist():
                glob.append([x + base for x in row])
            base += v.shape[0]
        gidx = np.array(glob, dtype=np.int32).reshape(-1, 3)
        got = oracle.merge(vtx, idx, vo, eo)
        exp = bruteforce.reindex(vtx, gidx)
        for x, y in zip(got, exp):
            assert np.array_equal(x, y)


def test_merge_of_copies_collapses_to_one_mesh():
    m = meshgen.grid_soup(30, 0.1, 5, "copies")
    single = oracle.reindex(m.vtx, m.idx)
    b = 3
    n, e = m.vtx.shape[0], m.idx.shape[0]
    vtx = np.concatenate([m.vtx] * b)
    idx = np.concatenate([m.idx] * b)
    vo = np.arange(b + 1, dtype=np.int64) * n
    eo = np.arange(b + 1, dtype=np.int64) * e
    ov, oi, o2n, n2o = oracle.merge(vtx, idx, vo, eo)
    assert np.array_equal(ov, single[0])
    assert np.array_equal(n2o, single[3])           # representatives stay in copy 0
    for c in range(b):
        assert np.array_equal(oi[c * e:(c + 1) * e], single[1])
        assert np.array_equal(o2n[c * n:(c + 1) * n], single[2])


def test_merge_of_disjoint_meshes_adds_up():
    parts = [meshgen.grid_soup(20 + 5 * s, 0.05, 60 + s, "part") for s in range(3)]
    vs = []
    for s, p in enumerate(parts):
        v = p.vtx.copy()
        v[:, 0] += np.float32(2 * s + 2)              # disjoint x ranges
        vs.append(v)
    vo = np.concatenate([[0], np.cumsum([v.shape[0] for v in vs])]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum([p.idx.shape[0] for p in parts])]).astype(np.int64)
    ov, oi, o2n, n2o = oracle.merge(np.concatenate(vs), np.concatenate([p.idx for p in parts]), vo, eo)
    assert ov.shape[0] == sum(p.expected_unique for p in parts)


def test_merge_checks_local_indices_per_mesh():
    a = meshgen.grid_soup(10, 0.0, 1, "a")
    b = meshgen.grid_soup(10, 0.0, 2, "b")
    idx = np.concatenate([a.idx, b.idx]).copy()
    e = a.idx.shape[0]
    idx[e + 4, 2] = b.vtx.shape[0]            # a valid packed id, but outside mesh b
    vo = np.array([0, a.vtx.shape[0], a.vtx.shape[0] + b.vtx.shape[0]], np.int64)
    eo = np.array([0, e, e + b.idx.shape[0]], np.int64)
    with pytest.raises(oracle.OracleIndexError) as ex:
        oracle.merge(np.concatenate([a.vtx, b.vtx]), idx, vo, eo)
    assert ex.value.pos == (e + 4) * 3 + 2
    idx[e + 4, 2] = -1
    with pytest.raises(oracle.OracleIndexError):
        oracle.merge(np.concatenate([a.vtx, b.vtx]), idx, vo, eo)


# ----------------------------------------------------------------- extract (Section 3)

def test_extract_matches_bruteforce_of_kept_elements():
    rng = np.random.default_rng(91)
    for vtx, idx in _fuzz_cases(150):
        keep = rng.random(idx.shape[0]) < rng.uniform(0, 1)
        rows = [idx[r] for r in range(idx.shape[0]) if keep[r]]
        kept = np.array(rows, dtype=np.int32).reshape(-1, idx.shape[1])
        got = oracle.extract(vtx, idx, keep)
        exp = bruteforce.reindex(vtx, kept)
        for x, y in zip(got, exp):
            assert np.array_equal(x, y)


def test_extract_all_and_nothing():
    m = meshgen.grid_soup(25, 0.1, 9, "ext")
    full = oracle.reindex(m.vtx, m.idx)
    got = oracle.extract(m.vtx, m.idx, np.ones(m.idx.shape[0], bool))
    for x, y in zip(got, full):
        assert np.array_equal(x, y)
    ov, oi, o2n, n2o = oracle.extract(m.vtx, m.idx, np.zeros(m.idx.shape[0], bool))
    assert ov.shape[0] == 0 and oi.shape == (0, 3) and n2o.size == 0 and np.all(o2n == -1)


@pytest.mark.parametrize("n", [2, 8, 64])
def test_extract_even_quad_rows_closed_form(n):
    # quad e covers grid cells (e % n, e // n); rows 0, 2, .. n-2 use point rows 0 .. n-1
    m = meshgen.paper_quads(n)
    keep = (np.arange(n * n) // n) % 2 == 0
    ov, oi, o2n, n2o = oracle.extract(m.vtx, m.idx, keep)
    assert ov.shape[0] == n * (n + 1)
    assert oi.shape == (n * n // 2, 4)
    # copies of used values map, kept or not: all corners of kept rows and of
    # the dropped rows between them, half the corners of the last (dropped) row
    assert int((o2n >= 0).sum()) == 4 * n * n - 2 * n


# ----------------------------------------------------------------- parallel CPU baseline

@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_cpu_baseline_matches_oracle(threads):
    cases = list(_fuzz_cases(60))
    cases.append((meshgen.cfg1().vtx, meshgen.cfg1().idx))
    cases.append((meshgen.tet_mesh(8, 0.03, 5).vtx, meshgen.tet_mesh(8, 0.03, 5).idx))
    cases.append((np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32)))
    for vtx, idx in cases:
        exp = oracle.reindex(vtx, idx)
        got = oracle.reindex_parallel(vtx, idx, threads)
        for x, y in zip(got, exp):
            assert np.array_equal(x, y)
    vtx = np.zeros((10, 2), np.float32)
    with pytest.raises(oracle.OracleIndexError) as e:
        oracle.reindex_parallel(vtx, np.array([[1, 2], [3, 10], [-1, 0]], np.int32), threads)
    assert e.value.pos == 3


def test_oracle_mutants_are_caught(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    oracle._load()
    src = open(oracle._SRC).read()
    for name, (old, new) in MUTANTS.items():
        assert old in src, name
        path = tmp_path / (name.replace(" ", "_") + ".cpp")
        path.write_text(src.replace(old, new))
        so = str(path) + ".so"
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", so, str(path)])
        assert not _pins_pass(so), f"mutant '{name}' slipped through the pins"

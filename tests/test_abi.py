"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments before enqueuing anything."""
import ctypes
import os
import re

import pytest

from paper_2109_09812_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "meshrx.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrx_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = declared_symbols()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_status_strings():
    lib = _lib.load()
    assert lib.mrx_abi_version() == 6
    for code, name in [(0, "MRX_OK"), (1, "MRX_ERR_INVALID_ARGUMENT"), (2, "MRX_ERR_WORKSPACE_TOO_SMALL"),
                       (3, "MRX_ERR_INDEX_OUT_OF_RANGE"), (4, "MRX_ERR_TOO_LARGE"), (5, "MRX_ERR_HIP"),
                       (6, "MRX_ERR_UNSUPPORTED"), (7, "MRX_ERR_INTERNAL")]:
        assert _lib.status_string(code) == name
    assert _lib.status_string(99) == "MRX_UNKNOWN_STATUS"


def test_tuning_enumeration():
    lib = _lib.load()
    for vb in range(4, 65, 4):
        ts = _lib.tunings(vb)
        assert len(ts) >= 1
        assert ts[0].digit_bits >= 8 and ts[0].block_threads % 64 == 0
        assert len({t.as_tuple() for t in ts}) == len(ts)
    for bad in (0, 2, 6, 68, -4):
        assert lib.mrx_tuning_count(bad) == 0
    t = _lib.Tuning()
    assert lib.mrx_tuning_get(12, 99, ctypes.byref(t)) == _lib.MRX_ERR_INVALID_ARGUMENT


def _ws(n, vb, m, meshes=1, tuning=None):
    out = ctypes.c_size_t(0)
    st = _lib.load().mrx_reindex_workspace_size(n, vb, m, meshes, _lib.make_tuning(tuning),
                                                ctypes.byref(out))
    return st, out.value


def test_workspace_size():
    st, small = _ws(1000, 12, 3000)
    assert st == 0 and small > 0 and small % 256 == 0
    st, big = _ws(26_398_316, 12, 25_141_254)
    assert st == 0 and big > 2 * 26_398_316 * 16
    st, batched = _ws(1000, 12, 3000, 4096)
    assert st == 0 and batched >= small
    assert _ws(-1, 12, 0)[0] == _lib.MRX_ERR_INVALID_ARGUMENT
    assert _ws(10, 6, 0)[0] == _lib.MRX_ERR_INVALID_ARGUMENT
    assert _ws(10, 12, 0, 0)[0] == _lib.MRX_ERR_INVALID_ARGUMENT
    assert _ws(2**31, 12, 0)[0] == _lib.MRX_ERR_TOO_LARGE
    assert _ws(10, 12, 0, 1, (7, 256, 16))[0] == _lib.MRX_ERR_UNSUPPORTED


# Fake, never-dereferenced device addresses: every call below must be
# rejected by host-side validation before anything is enqueued.
A = 0x10000000
B = 0x20000000
C = 0x30000000
D = 0x40000000
E = 0x50000000
F = 0x60000000
W = 0x70000000


def _call(**kw):
    args = dict(vtx=A, n=100, vb=12, idx=B, ne=10, arity=3, out_vtx=C, out_idx=D, old2new=E,
                new2old=F, out_num=0x7F000000, status=0x7F000100, ws=W, wsb=1 << 30, tuning=None,
                stream=None)
    args.update(kw)
    return _lib.load().mrx_reindex_mesh(
        args["vtx"], args["n"], args["vb"], args["idx"], args["ne"], args["arity"], args["out_vtx"],
        args["out_idx"], args["old2new"], args["new2old"], args["out_num"], args["status"], args["ws"],
        args["wsb"], _lib.make_tuning(args["tuning"]), args["stream"])


@pytest.mark.parametrize("kw,expected", [
    (dict(vb=6), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(vb=0), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(vb=68), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(arity=0), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(n=-1), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(ne=-1), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(n=2**31), _lib.MRX_ERR_TOO_LARGE),
    (dict(ne=2**30, arity=3), _lib.MRX_ERR_TOO_LARGE),
    (dict(vtx=None), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(out_vtx=None), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(old2new=None), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(idx=None), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(out_idx=None), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(out_num=None), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(vtx=A + 2), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(ws=W + 64), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(out_num=0x7F000004), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(wsb=1024), _lib.MRX_ERR_WORKSPACE_TOO_SMALL),
    (dict(ws=None, wsb=0), _lib.MRX_ERR_WORKSPACE_TOO_SMALL),
    (dict(out_vtx=A + 4), _lib.MRX_ERR_INVALID_ARGUMENT),      # overlaps vtx
    (dict(old2new=C + 8), _lib.MRX_ERR_INVALID_ARGUMENT),      # overlaps out_vtx
    (dict(out_idx=E), _lib.MRX_ERR_INVALID_ARGUMENT),          # out_idx == old2new
    (dict(new2old=W + 4096), _lib.MRX_ERR_INVALID_ARGUMENT),   # inside the workspace
    (dict(out_idx=B + 4), _lib.MRX_ERR_INVALID_ARGUMENT),        # overlaps idx without being it
    (dict(tuning=(7, 256, 16)), _lib.MRX_ERR_UNSUPPORTED),
    (dict(status=None), _lib.MRX_ERR_INVALID_ARGUMENT),              # the status word is required
    (dict(status=0x7F000102), _lib.MRX_ERR_INVALID_ARGUMENT),
    (dict(tuning=(0, 0, 0, 32)), _lib.MRX_ERR_UNSUPPORTED),         # unknown flag bit
    (dict(tuning=(8, 256, 16, 1 | 64)), _lib.MRX_ERR_UNSUPPORTED),
    (dict(tuning=(0, 0, 0, 4 | 8)), _lib.MRX_ERR_UNSUPPORTED),      # sort-all and hash grouping at once
])
def test_reindex_rejects_bad_arguments(kw, expected):
    assert _call(**kw) == expected


def test_tuning_flags():
    # the flags are accepted with the default or any compiled shape and
    # leave the workspace size unchanged
    st0, need0 = _ws(5000, 12, 3000)
    st1, need1 = _ws(5000, 12, 3000, tuning=(0, 0, 0, _lib.MRX_TUNING_WIDE_LOOKBACK))
    assert st0 == st1 == 0 and need0 == need1
    both = _lib.MRX_TUNING_WIDE_LOOKBACK | _lib.MRX_TUNING_CLAIMED_TILES
    for t in _lib.tunings(12):
        for fl in (_lib.MRX_TUNING_WIDE_LOOKBACK, _lib.MRX_TUNING_CLAIMED_TILES, both):
            st, need = _ws(5000, 12, 3000, tuning=(*t.as_tuple(), fl))
            assert st == 0, (t.as_tuple(), fl)
    assert _ws(5000, 12, 3000, tuning=(0, 0, 0, 32))[0] == _lib.MRX_ERR_UNSUPPORTED
    assert _ws(5000, 12, 3000, tuning=(0, 0, 0, both | 64))[0] == _lib.MRX_ERR_UNSUPPORTED
    sort_all, hashed = _lib.MRX_TUNING_SORT_ALL, _lib.MRX_TUNING_HASH_GROUPS
    assert _ws(5000, 12, 3000, tuning=(0, 0, 0, sort_all | hashed))[0] == _lib.MRX_ERR_UNSUPPORTED
    # the hash grouping needs a third element buffer
    st_s, need_s = _ws(100_000, 12, 90_000, tuning=(0, 0, 0, sort_all))
    st_h, need_h = _ws(100_000, 12, 90_000, tuning=(0, 0, 0, hashed))
    st_d, need_d = _ws(100_000, 12, 90_000)
    assert st_s == st_h == st_d == 0 and need_h >= need_s + 100_000 * 16 and need_d == need_h
    # vertex bands: band tables on top (single meshes, any size and either
    # strategy with the flag; without it only with hash grouping, from 2^20
    # index entries)
    bands = _lib.MRX_TUNING_BANDS
    st_b, need_b = _ws(100_000, 12, 90_000, tuning=(0, 0, 0, hashed | bands))
    assert st_b == 0 and need_b > need_h
    st_sb, need_sb = _ws(100_000, 12, 90_000, tuning=(0, 0, 0, sort_all | bands))
    assert st_sb == 0 and need_sb > need_s
    assert _ws(100_000, 12, 90_000, 7, (0, 0, 0, bands)) == _ws(100_000, 12, 90_000, 7)   # batches: none
    big = (2_000_000, 12, 1_500_000)
    assert _ws(*big, tuning=(0, 0, 0, sort_all))[1] < _ws(*big, tuning=(0, 0, 0, sort_all | bands))[1]
    assert _ws(2_000_000, 12, 1_500_000)[1] == _ws(2_000_000, 12, 1_500_000, tuning=(0, 0, 0, bands))[1]
    # more index entries than the element buffer holds: no bands
    assert _ws(1000, 4, 10_000, tuning=(0, 0, 0, hashed | bands))[1] == _ws(1000, 4, 10_000, tuning=(0, 0, 0, hashed))[1]
    # batches: hash grouping by (mesh id, record) needs the third buffer and
    # the meshes' bucket table; the default from 2^16 vertices in all
    st_b, need_b = _ws(100_000, 12, 90_000, 2, tuning=(0, 0, 0, hashed))
    st_bs, need_bs = _ws(100_000, 12, 90_000, 2, tuning=(0, 0, 0, sort_all))
    assert st_b == st_bs == 0 and need_b >= need_bs + 100_000 * 16
    assert _ws(100_000, 12, 90_000, 2) == (0, need_b)
    assert _ws(60_000, 12, 50_000, 2) == _ws(60_000, 12, 50_000, 2, tuning=(0, 0, 0, sort_all))
    assert (_ws(100_000, 64, 90_000, 2, tuning=(0, 0, 0, hashed))[1] >
            _ws(100_000, 64, 90_000, 2, tuning=(0, 0, 0, sort_all))[1])
    # a batch needing more than 2^24 hash buckets (at least one per mesh)
    # sorts all whatever the flags say
    many = (1 << 26, 12, 1 << 25, 20_000_000)
    assert _ws(*many, tuning=(0, 0, 0, hashed)) == _ws(*many, tuning=(0, 0, 0, sort_all))
    few = (1 << 26, 12, 1 << 25, 1_000_000)
    assert _ws(*few, tuning=(0, 0, 0, hashed))[1] > _ws(*few, tuning=(0, 0, 0, sort_all))[1]


def test_workspace_one_byte_short():
    st, need = _ws(100, 12, 30)
    assert st == 0
    assert _call(wsb=need - 1) == _lib.MRX_ERR_WORKSPACE_TOO_SMALL


def test_batched_rejects_bad_arguments():
    lib = _lib.load()
    f = lib.mrx_reindex_mesh_batched
    base = [A, 0x7E000000, 100, 12, B, 0x7E100000, 10, 3, 4, C, 0x7E200000, D, E, F, 0x7F000100, W, 1 << 30,
            None, None]
    assert f(*base[:8], 0, *base[9:]) == _lib.MRX_ERR_INVALID_ARGUMENT          # no meshes
    bad = list(base); bad[1] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no vtx_offsets
    bad = list(base); bad[10] = 0x7E200004
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # misaligned offsets
    bad = list(base); bad[16] = 256
    assert f(*bad) == _lib.MRX_ERR_WORKSPACE_TOO_SMALL
    bad = list(base); bad[11] = B + 4
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # out_idx overlaps idx
    bad = list(base); bad[14] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no status word


def test_merge_rejects_bad_arguments():
    f = _lib.load().mrx_merge_meshes
    # vtx, vtx_off, total_vtx, vb, idx, elem_off, total_elems, arity, meshes, out_vtx, out_idx,
    # old2new, new2old, out_num, status, ws, wsb, tuning, stream
    base = [A, 0x7E000000, 100, 12, B, 0x7E100000, 10, 3, 4, C, D, E, F, 0x7F000000, 0x7F000100, W,
            1 << 30, None, None]
    assert f(*base[:8], 0, *base[9:]) == _lib.MRX_ERR_INVALID_ARGUMENT          # no meshes
    bad = list(base); bad[5] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no elem_offsets
    bad = list(base); bad[5] = 0x7E000008
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # offsets overlap
    bad = list(base); bad[13] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no out_num_vtx
    bad = list(base); bad[16] = 256
    assert f(*bad) == _lib.MRX_ERR_WORKSPACE_TOO_SMALL
    bad = list(base); bad[17] = _lib.make_tuning((0, 0, 0, 32))
    assert f(*bad) == _lib.MRX_ERR_UNSUPPORTED
    bad = list(base); bad[14] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no status word


def test_extract_rejects_bad_arguments():
    f = _lib.load().mrx_extract_submesh
    # vtx, n, vb, idx, ne, arity, keep, out_vtx, out_idx, out_num_elems, old2new, new2old, out_num,
    # status, ws, wsb, tuning, stream
    base = [A, 100, 12, B, 10, 3, 0x7E000000, C, D, 0x7E100000, E, F, 0x7F000000, 0x7F000100, W, 1 << 30,
            None, None]
    bad = list(base); bad[6] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no keep flags
    bad = list(base); bad[8] = B
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # out_idx is idx
    bad = list(base); bad[9] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no kept count
    bad = list(base); bad[9] = 0x7E100004
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # misaligned count
    bad = list(base); bad[6] = D + 8
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # keep overlaps out_idx
    bad = list(base); bad[15] = 256
    assert f(*bad) == _lib.MRX_ERR_WORKSPACE_TOO_SMALL
    bad = list(base); bad[13] = None
    assert f(*bad) == _lib.MRX_ERR_INVALID_ARGUMENT                              # no status word


def test_gather_rejects_bad_arguments():
    lib = _lib.load()
    g = lib.mrx_gather_attrs
    assert g(A, 10, 0, 0, B, 5, C, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT   # channels
    assert g(A, 10, 16, 2, B, 5, C, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT  # dtype
    assert g(A, 10, 16, 0, B, 5, None, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT
    assert g(A + 4, 10, 16, 0, B, 5, C, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT
    assert g(A, 10, 16, 0, B, 5, A + 64, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT  # overlap
    assert g(A, 2**31, 16, 0, B, 5, C, None, None) == _lib.MRX_ERR_TOO_LARGE
    assert g(A, 10, 16, 0, B, 0, C, None, None) == _lib.MRX_OK                     # nothing to do
    gb = lib.mrx_gather_attrs_backward
    assert gb(A, 5, 16, 0, B, 10, None, 1, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT
    assert gb(A, 5, 16, 0, B, 10, C + 4, 1, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT
    assert gb(A, 5, 16, 1, B, 10, A, 1, None, None) == _lib.MRX_ERR_INVALID_ARGUMENT   # overlap


# ----------------------------------------------------------------- autotune cache (host logic)

def test_autotune_cache_validation(tmp_path, monkeypatch):
    import json
    from paper_2109_09812_amd import autotune as at
    path = str(tmp_path / "tune.json")
    assert at.load_cache(path) == {}                       # missing
    open(path, "w").write("{not json")
    assert at.load_cache(path) == {}                       # corrupt
    json.dump({"schema": 99, "abi": 1, "entries": {"k": {}}}, open(path, "w"))
    assert at.load_cache(path) == {}                       # other schema
    json.dump({"schema": at.SCHEMA, "abi": 999, "entries": {"k": {}}}, open(path, "w"))
    assert at.load_cache(path) == {}                       # other ABI
    t0 = _lib.tunings(12)[0].as_tuple()
    hashed = _lib.MRX_TUNING_HASH_GROUPS
    entries = {"a": {"tuning": list(t0) + [hashed]}, "b": {"tuning": [7, 333, 5, 0]}, "c": {"tuning": "x"},
               "d": {"tuning": list(t0)}, "e": {"tuning": list(t0) + [1]}}
    at.save_cache(entries, path)
    loaded = at.load_cache(path)
    assert loaded == json.loads(json.dumps(entries))
    assert at.cached_tuning(loaded, "a", 12).as_key() == t0 + (hashed,)
    assert at.cached_tuning(loaded, "b", 12) is None       # variant not in the library
    assert at.cached_tuning(loaded, "c", 12) is None       # malformed
    assert at.cached_tuning(loaded, "d", 12) is None       # no strategy (older schema)
    assert at.cached_tuning(loaded, "e", 12) is None       # flags that are not a strategy choice
    # candidates: every shape with both strategies (single meshes and batches),
    # shapes only where a call always sorts all
    single = at.candidates(12, 100_000, False)
    assert len(single) == 2 * len(_lib.tunings(12))
    assert {t.flags for t in single} == {_lib.MRX_TUNING_SORT_ALL, hashed}
    assert {t.flags for t in at.candidates(12, 100_000, True)} == {_lib.MRX_TUNING_SORT_ALL, hashed}
    assert {t.flags for t in at.candidates(12, 1 << 30, True)} == {0}
    assert {t.flags for t in at.candidates(12, 1 << 30, False)} == {0}
    assert at.cached_tuning(loaded, "missing", 12) is None
    k = at.shape_key("gfx950", 12, 26_398_316, False)
    assert k == "gfx950|R=12|n=2^25|single"
    assert at.shape_key("gfx950", 12, 1000, True).endswith("|batched")

"""Seeded random sweep over all four re-index calls (single mesh, batch,
merge, sub-mesh), every record width, every compiled tuning, every flag set,
and records in which random bytes are frozen so that digit passes with a
single live digit (skipped passes) turn up in every pattern. Each case is
compared bit for bit with the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
CASES = 400


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _records(rng, n, k):
    distinct = int(rng.integers(1, max(2, n) + 1))
    pool = rng.integers(0, 2**32, size=(distinct, k), dtype=np.uint64).astype(np.uint32)
    for w in range(k):
        for b in range(4):
            if rng.random() < 0.35:   # this byte is the same in every record
                keep = np.uint32(~(0xFF << (8 * b)) & 0xFFFFFFFF)
                pool[:, w] = (pool[:, w] & keep) | np.uint32(int(rng.integers(0, 256)) << (8 * b))
    return pool[rng.integers(0, distinct, size=n)] if n else np.zeros((0, k), np.uint32)


def _dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).to(DEV)


def _host(*ts):
    return tuple(t.cpu().numpy().view(np.uint32) if i == 0 else t.cpu().numpy() for i, t in enumerate(ts))


def _batch_parts(rng, n, a):
    nm = int(rng.integers(1, 40))
    vo = np.concatenate([[0], np.sort(rng.integers(0, n + 1, size=nm - 1)), [n]]).astype(np.int64)
    parts = [rng.integers(0, s, size=(int(rng.integers(0, 2 * s // a + 1)), a)).astype(np.int32)
             if s else np.zeros((0, a), np.int32) for s in np.diff(vo)]
    idx = np.concatenate(parts)
    eo = np.concatenate([[0], np.cumsum([p.shape[0] for p in parts])]).astype(np.int64)
    return vo, idx, eo


def test_random_sweep():
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(2109_09812)
    for case in range(CASES):
        k, a = int(rng.integers(1, 17)), int(rng.integers(1, 5))
        n = int(rng.choice([0, 1, 2, 63, 64, 65, 4095, 4097, int(rng.integers(1, 200_000))]))
        e = int(rng.integers(0, 2 * n // a + 1)) if n else 0
        vtx = _records(rng, n, k)
        idx = rng.integers(0, max(n, 1), size=(e, a)).astype(np.int32)
        ts = mrx.tunings(4 * k)
        t = ts[int(rng.integers(0, len(ts)))].as_tuple() + (int(rng.integers(0, 4)),)
        kind = ["single", "batched", "merge", "extract"][int(rng.integers(0, 4))]
        _say(case, kind, "N", n, "K", k, "A", a, "E", e, "tuning", t)
        if kind == "single":
            r = mrx.reindex_mesh(_dev(vtx), _dev(idx), tuning=t)
            got = _host(r.out_vtx, r.out_idx, r.old2new, r.new2old)
            exp = oracle.reindex(vtx, idx)
        elif kind == "extract":
            keep = rng.random(e) < rng.random()
            r = mrx.extract_submesh(_dev(vtx), _dev(idx), torch.from_numpy(keep).to(DEV), tuning=t)
            got = _host(r.out_vtx, r.out_idx, r.old2new, r.new2old)
            exp = oracle.extract(vtx, idx, keep)
        else:
            vo, idx, eo = _batch_parts(rng, n, a)
            if kind == "batched":
                r = mrx.reindex_mesh_batched(_dev(vtx), _dev(vo), _dev(idx), _dev(eo), tuning=t)
                got = _host(r.out_vtx, r.out_vtx_offsets, r.out_idx, r.old2new, r.new2old)
                exp = oracle.reindex_batched(vtx, idx, vo, eo)
            else:
                r = mrx.merge_meshes(_dev(vtx), _dev(vo), _dev(idx), _dev(eo), tuning=t)
                got = _host(r.out_vtx, r.out_idx, r.old2new, r.new2old)
                exp = oracle.merge(vtx, idx, vo, eo)
        assert len(got) == len(exp)
        for i, (g, x) in enumerate(zip(got, exp)):
            assert g.shape == x.shape and np.array_equal(g, x), (case, kind, i)

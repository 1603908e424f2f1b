"""The entry point that allocates nothing (mrx_reindex_mesh_noalloc, for
callers that cannot allocate): its fixed per-GPU scratch array gives the
same result as mrx_reindex_mesh with a caller workspace, on two calls in a
row (the second smaller, so the array still holds the first call's
contents), and a call that needs more than the array is refused before
anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import meshgen

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _outs(n, k, m, dev):
    return (torch.empty(n, k, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.zeros(1, dtype=torch.int64, device=dev), torch.full((1,), -99, dtype=torch.int32, device=dev))


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(lib, mesh, stream):
    """Same mesh through mrx_reindex_mesh (caller workspace) and through
    mrx_reindex_mesh_noalloc, both through the C ABI on one stream."""
    from paper_2109_09812_amd import _lib
    from paper_2109_09812_amd.api import workspace_size
    vtx = torch.from_numpy(np.ascontiguousarray(mesh.vtx).view(np.int32)).to(DEV)
    idx = torch.from_numpy(mesh.idx).to(DEV)
    n, k = vtx.shape
    e, a = idx.shape
    ref = _outs(n, k, e * a, DEV)
    wsb = workspace_size(n, 4 * k, e * a)
    assert wsb <= _lib.MRX_NOALLOC_SCRATCH_BYTES, wsb
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    st = lib.mrx_reindex_mesh(_p(vtx), n, 4 * k, _p(idx), e, a, _p(ref[0]), _p(ref[1]), _p(ref[2]), _p(ref[3]),
                              _p(ref[4]), _p(ref[5]), _p(ws), wsb, None, stream)
    assert st == 0, st
    got = _outs(n, k, e * a, DEV)
    st = lib.mrx_reindex_mesh_noalloc(_p(vtx), n, 4 * k, _p(idx), e, a, _p(got[0]), _p(got[1]), _p(got[2]),
                                      _p(got[3]), _p(got[4]), _p(got[5]), None, stream)
    assert st == 0, st
    torch.cuda.synchronize()
    u = int(ref[4].item())
    assert int(got[4].item()) == u == mesh.expected_unique
    assert int(ref[5].item()) == 0 and int(got[5].item()) == 0
    assert torch.equal(got[0][:u], ref[0][:u])
    assert torch.equal(got[1], ref[1])
    assert torch.equal(got[2], ref[2])
    assert torch.equal(got[3][:u], ref[3][:u])
    return u


def test_noalloc_matches_workspace_call_twice_then_smaller():
    from paper_2109_09812_amd import _lib
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    big = meshgen.grid_soup(300, 0.05, 7001, "noalloc-big")
    small = meshgen.grid_soup(97, 0.10, 7002, "noalloc-small")
    _say("noalloc: first call", big.num_vtx, "vertices")
    _both(lib, big, stream)
    _say("noalloc: second call, smaller", small.num_vtx, "vertices")
    _both(lib, small, stream)


def test_noalloc_refuses_what_does_not_fit():
    import paper_2109_09812_amd as mrx
    from paper_2109_09812_amd import _lib
    from paper_2109_09812_amd.api import workspace_size
    n = 2_000_000
    assert workspace_size(n, 12, 3 * n) > _lib.MRX_NOALLOC_SCRATCH_BYTES
    vtx = torch.zeros(n, 3, dtype=torch.int32, device=DEV)
    idx = torch.zeros(n, 3, dtype=torch.int32, device=DEV)
    _say("noalloc: too large")
    with pytest.raises(mrx.MeshrxError) as ei:
        mrx.reindex_mesh_noalloc(vtx, idx)
    assert ei.value.status == _lib.MRX_ERR_NOALLOC_TOO_LARGE
    # the Python wrapper gives the same result as reindex_mesh on a small mesh
    m = meshgen.grid_soup(64, 0.1, 7003, "noalloc-api")
    v = torch.from_numpy(m.vtx.view(np.int32)).to(DEV)
    i = torch.from_numpy(m.idx).to(DEV)
    r1 = mrx.reindex_mesh(v, i)
    r2 = mrx.reindex_mesh_noalloc(v, i)
    assert r1.num_out == r2.num_out == m.expected_unique
    for x, y in ((r1.out_vtx, r2.out_vtx), (r1.out_idx, r2.out_idx), (r1.old2new, r2.old2new),
                 (r1.new2old, r2.new2old)):
        assert torch.equal(x, y)

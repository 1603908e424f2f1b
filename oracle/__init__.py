"""CPU oracle for mesh re-indexing — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import this package. The product path (the HIP
library and its Python binding) never imports, links or calls it.

* ``reindex``            — serial std::map re-indexer (oracle.cpp), the plain
                           definition the GPU path must match bit for bit.
* ``reindex_batched``    — the same, once per mesh of a packed batch.
* ``merge``              — Section 3 "merging meshes": offset each mesh's local
                           indices by its first vertex, then ``reindex`` the
                           concatenation once (equal vertices of different
                           meshes merge).
* ``extract``            — Section 3 "computing a subset of a mesh": keep the
                           flagged elements in order, then ``reindex`` (which
                           drops the vertices only other elements used).
* ``gather_attrs``       — torch CPU ``index_select`` (plus autograd for the
                           backward), the definition of the attribute gather.
* ``paper_steps``        — a re-enactment of Section 2 Steps 1-4 in the
                           paper's order and notation (pins the oracle).
* ``bruteforce``         — O(n^2) grouping by record bytes (pins the oracle).
* ``reindex_parallel``   — the paper's data-parallel steps on host threads
                           (parallel_cpu.cpp): a CPU baseline for timing, not
                           the oracle; tests check it against ``reindex``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_SRC_PAR = os.path.join(_HERE, "parallel_cpu.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK = 0
INVALID_ARGUMENT = 1
INDEX_OUT_OF_RANGE = 3


def build(force: bool = True) -> str:
    """Compile oracle.cpp and parallel_cpu.cpp with g++ into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC, _SRC_PAR])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        if hasattr(lib, "cpu_parallel_reindex"):  # absent from single-file test builds
            lib.cpu_parallel_reindex.restype = ctypes.c_int
            lib.cpu_parallel_reindex.argtypes = [
                ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_reindex.restype = ctypes.c_int
        lib.oracle_reindex.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        _lib = lib
    return _lib


class OracleIndexError(IndexError):
    def __init__(self, pos):
        super().__init__(f"index entry {pos} is out of range")
        self.pos = pos


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def reindex(vtx: np.ndarray, idx: np.ndarray):
    """vtx [N, K] (any 4-byte dtype, read as raw uint32), idx [E, A] int32.

    Returns (out_vtx [U, K] uint32, out_idx [E, A] int32, old2new [N] int32,
    new2old [U] int32). Raises OracleIndexError on an out-of-range index."""
    vtx = np.ascontiguousarray(vtx)
    assert vtx.ndim == 2 and vtx.dtype.itemsize == 4
    words = int(vtx.shape[1])
    v = vtx.view(np.uint32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = int(v.shape[0])
    m = int(idx.size)
    out_vtx = np.empty((max(n, 1), words), dtype=np.uint32)
    out_idx = np.empty(idx.shape, dtype=np.int32)
    old2new = np.empty(n, dtype=np.int32)
    new2old = np.empty(max(n, 1), dtype=np.int32)
    u = ctypes.c_int64(0)
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_reindex(_ptr(v), n, words, _ptr(idx), m, _ptr(out_vtx),
                                _ptr(out_idx), _ptr(old2new), _ptr(new2old),
                                ctypes.byref(u), ctypes.byref(bad))
    if rc == INDEX_OUT_OF_RANGE:
        raise OracleIndexError(bad.value)
    if rc != OK:
        raise ValueError(f"oracle_reindex: invalid argument (status {rc})")
    uu = u.value
    return out_vtx[:uu].copy(), out_idx, old2new, new2old[:uu].copy()


def reindex_parallel(vtx: np.ndarray, idx: np.ndarray, threads: int = 8):
    """Same contract as ``reindex``, computed by the multi-threaded CPU
    baseline (parallel_cpu.cpp) with ``threads`` host threads."""
    vtx = np.ascontiguousarray(vtx)
    assert vtx.ndim == 2 and vtx.dtype.itemsize == 4
    words = int(vtx.shape[1])
    v = vtx.view(np.uint32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = int(v.shape[0])
    out_vtx = np.empty((max(n, 1), words), dtype=np.uint32)
    out_idx = np.empty(idx.shape, dtype=np.int32)
    old2new = np.empty(n, dtype=np.int32)
    new2old = np.empty(max(n, 1), dtype=np.int32)
    u = ctypes.c_int64(0)
    bad = ctypes.c_int64(-1)
    rc = _load().cpu_parallel_reindex(_ptr(v), n, words, _ptr(idx), int(idx.size), int(threads),
                                      _ptr(out_vtx), _ptr(out_idx), _ptr(old2new), _ptr(new2old),
                                      ctypes.byref(u), ctypes.byref(bad))
    if rc == INDEX_OUT_OF_RANGE:
        raise OracleIndexError(bad.value)
    if rc != OK:
        raise ValueError(f"cpu_parallel_reindex: invalid argument (status {rc})")
    uu = u.value
    return out_vtx[:uu].copy(), out_idx, old2new, new2old[:uu].copy()


def reindex_batched(vtx, idx, vtx_offsets, elem_offsets):
    """Per-mesh oracle over a packed batch. Returns packed (out_vtx,
    out_vtx_offsets [B+1], out_idx, old2new, new2old), all ids mesh-local."""
    b = len(vtx_offsets) - 1
    outs_v, outs_i, outs_o2n, outs_n2o = [], [], [], []
    offs = np.zeros(b + 1, dtype=np.int64)
    for i in range(b):
        v0, v1 = int(vtx_offsets[i]), int(vtx_offsets[i + 1])
        e0, e1 = int(elem_offsets[i]), int(elem_offsets[i + 1])
        ov, oi, o2n, n2o = reindex(vtx[v0:v1], idx[e0:e1])
        outs_v.append(ov)
        outs_i.append(oi)
        outs_o2n.append(o2n)
        outs_n2o.append(n2o)
        offs[i + 1] = offs[i] + ov.shape[0]
    k = vtx.shape[1]
    cat = lambda xs, shape: np.concatenate(xs) if xs else np.zeros(shape, np.int32)
    return (np.concatenate(outs_v) if outs_v else np.zeros((0, k), np.uint32), offs,
            cat(outs_i, (0, idx.shape[1])), cat(outs_o2n, (0,)), cat(outs_n2o, (0,)))


def merge(vtx, idx, vtx_offsets, elem_offsets):
    """Merge the meshes of a packed batch into one mesh (Section 3, "Merging
    meshes that share (some) vertices"): the vertex arrays are already
    concatenated; every mesh's local indices are raised by the number of
    vertices of the meshes before it, and the single resulting mesh is
    re-indexed. Returns ``reindex`` of it. A local index outside its own mesh
    raises OracleIndexError with its position in the flat index array."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    arity = idx.shape[1]
    gidx = np.empty(idx.shape, dtype=np.int64)
    for b in range(len(vtx_offsets) - 1):
        v0, v1 = int(vtx_offsets[b]), int(vtx_offsets[b + 1])
        e0, e1 = int(elem_offsets[b]), int(elem_offsets[b + 1])
        local = idx[e0:e1].astype(np.int64)
        bad = np.flatnonzero(((local < 0) | (local >= v1 - v0)).reshape(-1))
        if bad.size:
            raise OracleIndexError(e0 * arity + int(bad[0]))
        gidx[e0:e1] = local + v0
    return reindex(vtx, gidx.astype(np.int32))


def extract(vtx, idx, keep):
    """Compact sub-mesh of the elements whose ``keep`` flag is set (Section 3,
    "Computing a subset of a mesh"): the full vertex array with only those
    elements, in their original order, re-indexed, so every vertex that only
    dropped elements referenced disappears. Returns ``reindex`` of it
    (out_idx has one row per kept element)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    keep = np.asarray(keep).astype(bool).reshape(-1)
    assert keep.shape[0] == idx.shape[0]
    return reindex(vtx, idx[keep])


def gather_attrs(attrs, new2old):
    """new[j, :] = attrs[new2old[j], :] on the CPU (torch index_select)."""
    import torch
    return torch.index_select(attrs, 0, torch.as_tensor(new2old, dtype=torch.int64))


def gather_attrs_backward(grad_out, new2old, num_old):
    """Gradient of gather_attrs w.r.t. attrs via CPU autograd."""
    import torch
    attrs = torch.zeros(num_old, grad_out.shape[1], dtype=grad_out.dtype, requires_grad=True)
    out = gather_attrs(attrs, new2old)
    out.backward(grad_out)
    return attrs.grad.detach()

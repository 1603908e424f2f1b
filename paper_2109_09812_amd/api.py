"""Python API over the C ABI. Torch supplies device memory and the stream;
every step of the re-indexing runs in the HIP library."""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import MRX_ERR_INDEX_OUT_OF_RANGE, MRX_OK, check, load, make_tuning


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def workspace_size(num_vtx: int, vtx_bytes: int, num_idx: int, num_meshes: int = 1,
                   tuning=None) -> int:
    out = ctypes.c_size_t(0)
    check(load().mrx_reindex_workspace_size(int(num_vtx), int(vtx_bytes), int(num_idx),
                                            int(num_meshes), make_tuning(tuning), ctypes.byref(out)),
          "mrx_reindex_workspace_size")
    return int(out.value)


def _check_vtx(vtx: torch.Tensor):
    if not vtx.is_cuda:
        raise ValueError("vtx must be a device tensor")
    if vtx.dim() != 2 or vtx.element_size() != 4 or not vtx.is_contiguous():
        raise ValueError("vtx must be a contiguous [N, K] tensor of a 4-byte dtype")


def _check_idx(idx: torch.Tensor):
    if not idx.is_cuda or idx.dtype != torch.int32 or idx.dim() != 2 or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous [E, A] int32 device tensor")


@dataclasses.dataclass
class Reindexed:
    """Outputs of a re-index. Tensors are sized to capacity until trimmed."""

    out_vtx: torch.Tensor
    out_idx: torch.Tensor
    old2new: torch.Tensor
    new2old: torch.Tensor | None
    meta: torch.Tensor          # int64 [2]: U, status (written by the device)
    num_out: int | None = None

    def trim(self) -> "Reindexed":
        """One device->host read of U and the status; raises on a data error."""
        u, status = (int(x) for x in self.meta[:2].cpu())
        status &= 0xFFFFFFFF
        if status == MRX_ERR_INDEX_OUT_OF_RANGE:
            raise IndexError("an index entry is out of range")
        check(status, "mrx_reindex_mesh (device)")
        self.num_out = u
        self.out_vtx = self.out_vtx[:u]
        if self.new2old is not None:
            self.new2old = self.new2old[:u]
        return self


def reindex_mesh(vtx: torch.Tensor, idx: torch.Tensor, *, tuning=None, workspace=None,
                 in_place: bool = False, want_new2old: bool = True, sync: bool = True) -> Reindexed:
    """Re-index one mesh (Section 2, Steps 1-4) on the GPU.

    vtx: [N, K] 4-byte dtype (records compared as raw 32-bit words);
    idx: [E, A] int32. Returns out_vtx [U, K], out_idx [E, A], old2new [N],
    new2old [U] (trimmed when ``sync``)."""
    _check_vtx(vtx)
    _check_idx(idx)
    n, k = vtx.shape
    dev = vtx.device
    m = idx.numel()
    out_vtx = torch.empty_like(vtx)
    out_idx = idx if in_place else torch.empty_like(idx)
    old2new = torch.empty(n, dtype=torch.int32, device=dev)
    new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
    meta = torch.zeros(2, dtype=torch.int64, device=dev)
    wsb = workspace_size(n, 4 * k, m, 1, tuning)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = load().mrx_reindex_mesh(
        _ptr(vtx), n, 4 * k, _ptr(idx), idx.shape[0], idx.shape[1], _ptr(out_vtx), _ptr(out_idx),
        _ptr(old2new), _ptr(new2old), _ptr(meta), ctypes.c_void_p(meta.data_ptr() + 8),
        _ptr(workspace), workspace.numel(), make_tuning(tuning), ctypes.c_void_p(_stream_handle(dev)))
    check(st, "mrx_reindex_mesh")
    r = Reindexed(out_vtx, out_idx, old2new, new2old, meta)
    return r.trim() if sync else r


def reindex_mesh_noalloc(vtx: torch.Tensor, idx: torch.Tensor, out=None, *, tuning=None,
                         sync: bool = True) -> Reindexed:
    """``reindex_mesh`` through ``mrx_reindex_mesh_noalloc``: the library
    works in its fixed per-GPU scratch array instead of a workspace. With
    ``out`` (a Reindexed of capacity tensors from an earlier call, e.g. made
    before graph capture) nothing is allocated here either."""
    _check_vtx(vtx)
    _check_idx(idx)
    n, k = vtx.shape
    dev = vtx.device
    if out is None:
        out = Reindexed(torch.empty_like(vtx), torch.empty_like(idx), torch.empty(n, dtype=torch.int32, device=dev),
                        torch.empty(n, dtype=torch.int32, device=dev), torch.zeros(2, dtype=torch.int64, device=dev))
    st = load().mrx_reindex_mesh_noalloc(
        _ptr(vtx), n, 4 * k, _ptr(idx), idx.shape[0], idx.shape[1], _ptr(out.out_vtx), _ptr(out.out_idx),
        _ptr(out.old2new), _ptr(out.new2old), _ptr(out.meta), ctypes.c_void_p(out.meta.data_ptr() + 8),
        make_tuning(tuning), ctypes.c_void_p(_stream_handle(dev)))
    check(st, "mrx_reindex_mesh_noalloc")
    return out.trim() if sync else out


def _offsets_ok(o: torch.Tensor) -> bool:
    return o.is_cuda and o.dtype == torch.int64 and o.dim() == 1 and o.is_contiguous()


def merge_meshes(vtx: torch.Tensor, vtx_offsets: torch.Tensor, idx: torch.Tensor,
                 elem_offsets: torch.Tensor, *, tuning=None, workspace=None, in_place: bool = False,
                 want_new2old: bool = True, sync: bool = True) -> Reindexed:
    """Merge the meshes of a packed batch into ONE mesh (Section 3, merging
    meshes): mesh-local indices are offset by each mesh's first vertex and the
    whole is re-indexed once, so bitwise-equal vertices of different meshes
    merge. Returns out_vtx [U, K], out_idx [E, A] (ids into out_vtx),
    old2new [N] over the packed vertices, new2old [U] (packed vertex ids)."""
    _check_vtx(vtx)
    _check_idx(idx)
    if not (_offsets_ok(vtx_offsets) and _offsets_ok(elem_offsets)):
        raise ValueError("offsets must be contiguous int64 device tensors")
    if vtx_offsets.numel() != elem_offsets.numel() or vtx_offsets.numel() < 2:
        raise ValueError("vtx_offsets and elem_offsets must both have num_meshes + 1 entries")
    n, k = vtx.shape
    dev = vtx.device
    out_vtx = torch.empty_like(vtx)
    out_idx = idx if in_place else torch.empty_like(idx)
    old2new = torch.empty(n, dtype=torch.int32, device=dev)
    new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
    meta = torch.zeros(2, dtype=torch.int64, device=dev)
    wsb = workspace_size(n, 4 * k, idx.numel(), 1, tuning)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = load().mrx_merge_meshes(
        _ptr(vtx), _ptr(vtx_offsets), n, 4 * k, _ptr(idx), _ptr(elem_offsets), idx.shape[0], idx.shape[1],
        vtx_offsets.numel() - 1, _ptr(out_vtx), _ptr(out_idx), _ptr(old2new), _ptr(new2old), _ptr(meta),
        ctypes.c_void_p(meta.data_ptr() + 8), _ptr(workspace), workspace.numel(), make_tuning(tuning),
        ctypes.c_void_p(_stream_handle(dev)))
    check(st, "mrx_merge_meshes")
    r = Reindexed(out_vtx, out_idx, old2new, new2old, meta)
    return r.trim() if sync else r


@dataclasses.dataclass
class Extracted(Reindexed):
    """A Reindexed whose out_idx holds only the kept elements once trimmed;
    meta[2] is the kept element count."""

    num_elems_out: int | None = None

    def trim(self) -> "Extracted":
        super().trim()  # raises on a data error first
        kept = int(self.meta[2].cpu())
        self.num_elems_out = kept
        self.out_idx = self.out_idx[:kept]
        return self


def extract_submesh(vtx: torch.Tensor, idx: torch.Tensor, keep: torch.Tensor, *, tuning=None,
                    workspace=None, want_new2old: bool = True, sync: bool = True) -> Extracted:
    """Compact sub-mesh of the elements with keep[e] set (Section 3, computing
    a subset of a mesh): kept elements stay in order, vertices only dropped
    elements used disappear. Returns out_vtx [U, K], out_idx [kept, A],
    old2new [N] (over all input vertices), new2old [U]."""
    _check_vtx(vtx)
    _check_idx(idx)
    if not keep.is_cuda or keep.dim() != 1 or keep.numel() != idx.shape[0] or not keep.is_contiguous():
        raise ValueError("keep must be a contiguous [E] device tensor")
    if keep.dtype == torch.bool:
        keep = keep.view(torch.uint8)
    elif keep.dtype != torch.uint8:
        raise ValueError("keep must be bool or uint8")
    n, k = vtx.shape
    dev = vtx.device
    out_vtx = torch.empty_like(vtx)
    out_idx = torch.empty_like(idx)
    old2new = torch.empty(n, dtype=torch.int32, device=dev)
    new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
    meta = torch.zeros(3, dtype=torch.int64, device=dev)
    wsb = workspace_size(n, 4 * k, idx.numel(), 1, tuning)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = load().mrx_extract_submesh(
        _ptr(vtx), n, 4 * k, _ptr(idx), idx.shape[0], idx.shape[1], _ptr(keep), _ptr(out_vtx), _ptr(out_idx),
        ctypes.c_void_p(meta.data_ptr() + 16), _ptr(old2new), _ptr(new2old), _ptr(meta),
        ctypes.c_void_p(meta.data_ptr() + 8), _ptr(workspace), workspace.numel(), make_tuning(tuning),
        ctypes.c_void_p(_stream_handle(dev)))
    check(st, "mrx_extract_submesh")
    r = Extracted(out_vtx, out_idx, old2new, new2old, meta)
    return r.trim() if sync else r


class MeshMerger:
    """Preallocated merge of a packed batch of fixed shape (see
    merge_meshes); ``launch()`` enqueues it without allocating or
    synchronising."""

    def __init__(self, vtx, vtx_offsets, idx, elem_offsets, *, tuning=None, want_new2old: bool = True):
        _check_vtx(vtx)
        _check_idx(idx)
        if not (_offsets_ok(vtx_offsets) and _offsets_ok(elem_offsets)) or \
                vtx_offsets.numel() != elem_offsets.numel() or vtx_offsets.numel() < 2:
            raise ValueError("offsets must be contiguous int64 device tensors of num_meshes + 1 entries")
        self.vtx, self.vtx_offsets, self.idx, self.elem_offsets = vtx, vtx_offsets, idx, elem_offsets
        n, k = vtx.shape
        dev = vtx.device
        self.out_vtx = torch.empty_like(vtx)
        self.out_idx = torch.empty_like(idx)
        self.old2new = torch.empty(n, dtype=torch.int32, device=dev)
        self.new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
        self.meta = torch.zeros(2, dtype=torch.int64, device=dev)
        wsb = workspace_size(n, 4 * k, idx.numel(), 1, tuning)
        self.workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        self._tuning_ptr = make_tuning(tuning)

    def launch(self):
        n, k = self.vtx.shape
        st = load().mrx_merge_meshes(
            _ptr(self.vtx), _ptr(self.vtx_offsets), n, 4 * k, _ptr(self.idx), _ptr(self.elem_offsets),
            self.idx.shape[0], self.idx.shape[1], self.vtx_offsets.numel() - 1, _ptr(self.out_vtx),
            _ptr(self.out_idx), _ptr(self.old2new), _ptr(self.new2old), _ptr(self.meta),
            ctypes.c_void_p(self.meta.data_ptr() + 8), _ptr(self.workspace), self.workspace.numel(),
            self._tuning_ptr, ctypes.c_void_p(_stream_handle(self.vtx.device)))
        check(st, "mrx_merge_meshes")

    def result(self) -> Reindexed:
        return Reindexed(self.out_vtx, self.out_idx, self.old2new, self.new2old, self.meta).trim()


class SubmeshExtractor:
    """Preallocated sub-mesh extraction for a fixed mesh shape (see
    extract_submesh); refill ``keep`` in place between launches."""

    def __init__(self, vtx, idx, keep, *, tuning=None, want_new2old: bool = True):
        _check_vtx(vtx)
        _check_idx(idx)
        if not keep.is_cuda or keep.dim() != 1 or keep.numel() != idx.shape[0] or not keep.is_contiguous() \
                or keep.dtype not in (torch.bool, torch.uint8):
            raise ValueError("keep must be a contiguous [E] bool/uint8 device tensor")
        self.vtx, self.idx = vtx, idx
        self.keep = keep.view(torch.uint8) if keep.dtype == torch.bool else keep
        n, k = vtx.shape
        dev = vtx.device
        self.out_vtx = torch.empty_like(vtx)
        self.out_idx = torch.empty_like(idx)
        self.old2new = torch.empty(n, dtype=torch.int32, device=dev)
        self.new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
        self.meta = torch.zeros(3, dtype=torch.int64, device=dev)
        wsb = workspace_size(n, 4 * k, idx.numel(), 1, tuning)
        self.workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        self._tuning_ptr = make_tuning(tuning)

    def launch(self):
        n, k = self.vtx.shape
        st = load().mrx_extract_submesh(
            _ptr(self.vtx), n, 4 * k, _ptr(self.idx), self.idx.shape[0], self.idx.shape[1], _ptr(self.keep),
            _ptr(self.out_vtx), _ptr(self.out_idx), ctypes.c_void_p(self.meta.data_ptr() + 16),
            _ptr(self.old2new), _ptr(self.new2old), _ptr(self.meta), ctypes.c_void_p(self.meta.data_ptr() + 8),
            _ptr(self.workspace), self.workspace.numel(), self._tuning_ptr,
            ctypes.c_void_p(_stream_handle(self.vtx.device)))
        check(st, "mrx_extract_submesh")

    def result(self) -> "Extracted":
        return Extracted(self.out_vtx, self.out_idx, self.old2new, self.new2old, self.meta).trim()


class Reindexer:
    """Preallocated outputs and workspace for one mesh shape; ``launch()``
    enqueues the whole re-index on the current stream without allocating or
    synchronising (repeatable, graph-capturable)."""

    def __init__(self, vtx: torch.Tensor, idx: torch.Tensor, *, tuning=None, want_new2old: bool = True):
        _check_vtx(vtx)
        _check_idx(idx)
        self.vtx, self.idx = vtx, idx
        n, k = vtx.shape
        dev = vtx.device
        self.tuning = tuning
        self._tuning_ptr = make_tuning(tuning)
        self.out_vtx = torch.empty_like(vtx)
        self.out_idx = torch.empty_like(idx)
        self.old2new = torch.empty(n, dtype=torch.int32, device=dev)
        self.new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
        self.meta = torch.zeros(2, dtype=torch.int64, device=dev)
        wsb = workspace_size(n, 4 * k, idx.numel(), 1, tuning)
        self.workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)

    def launch(self):
        n, k = self.vtx.shape
        st = load().mrx_reindex_mesh(
            _ptr(self.vtx), n, 4 * k, _ptr(self.idx), self.idx.shape[0], self.idx.shape[1],
            _ptr(self.out_vtx), _ptr(self.out_idx), _ptr(self.old2new), _ptr(self.new2old), _ptr(self.meta),
            ctypes.c_void_p(self.meta.data_ptr() + 8), _ptr(self.workspace), self.workspace.numel(),
            self._tuning_ptr, ctypes.c_void_p(_stream_handle(self.vtx.device)))
        check(st, "mrx_reindex_mesh")

    def result(self) -> Reindexed:
        return Reindexed(self.out_vtx, self.out_idx, self.old2new, self.new2old, self.meta).trim()


@dataclasses.dataclass
class BatchReindexed:
    out_vtx: torch.Tensor
    out_vtx_offsets: torch.Tensor   # int64 [B+1]
    out_idx: torch.Tensor
    old2new: torch.Tensor
    new2old: torch.Tensor | None
    status: torch.Tensor            # int32 [1]

    def trim(self) -> "BatchReindexed":
        st = int(self.status.cpu()[0])
        if st == MRX_ERR_INDEX_OUT_OF_RANGE:
            raise IndexError("an index entry is out of range")
        check(st, "mrx_reindex_mesh_batched (device)")
        u = int(self.out_vtx_offsets[-1].cpu())
        self.out_vtx = self.out_vtx[:u]
        if self.new2old is not None:
            self.new2old = self.new2old[:u]
        return self


class BatchedReindexer:
    """Holds the outputs and workspace of a packed batch of a fixed shape, so
    that the launch sequence can be replayed (e.g. inside a HIP graph)."""

    def __init__(self, vtx: torch.Tensor, vtx_offsets: torch.Tensor, idx: torch.Tensor,
                 elem_offsets: torch.Tensor, *, tuning=None, want_new2old: bool = True):
        _check_vtx(vtx)
        _check_idx(idx)
        for o in (vtx_offsets, elem_offsets):
            if not o.is_cuda or o.dtype != torch.int64 or o.dim() != 1 or not o.is_contiguous():
                raise ValueError("offsets must be contiguous int64 device tensors")
        if vtx_offsets.numel() != elem_offsets.numel() or vtx_offsets.numel() < 2:
            raise ValueError("vtx_offsets and elem_offsets must both have num_meshes + 1 entries")
        self.vtx, self.idx = vtx, idx
        self.vtx_offsets, self.elem_offsets = vtx_offsets, elem_offsets
        n, k = vtx.shape
        dev = vtx.device
        self.num_meshes = vtx_offsets.numel() - 1
        self.tuning = tuning
        self.out_vtx = torch.empty_like(vtx)
        self.out_vtx_offsets = torch.empty(self.num_meshes + 1, dtype=torch.int64, device=dev)
        self.out_idx = torch.empty_like(idx)
        self.old2new = torch.empty(n, dtype=torch.int32, device=dev)
        self.new2old = torch.empty(n, dtype=torch.int32, device=dev) if want_new2old else None
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        wsb = workspace_size(n, 4 * k, idx.numel(), self.num_meshes, tuning)
        self.workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        self._tuning_ptr = make_tuning(tuning)

    def launch(self):
        """Enqueue the whole segmented launch sequence on the current stream."""
        n, k = self.vtx.shape
        st = load().mrx_reindex_mesh_batched(
            _ptr(self.vtx), _ptr(self.vtx_offsets), n, 4 * k, _ptr(self.idx), _ptr(self.elem_offsets),
            self.idx.shape[0], self.idx.shape[1], self.num_meshes, _ptr(self.out_vtx),
            _ptr(self.out_vtx_offsets), _ptr(self.out_idx), _ptr(self.old2new), _ptr(self.new2old),
            _ptr(self.status), _ptr(self.workspace), self.workspace.numel(), self._tuning_ptr,
            ctypes.c_void_p(_stream_handle(self.vtx.device)))
        check(st, "mrx_reindex_mesh_batched")

    def result(self) -> BatchReindexed:
        return BatchReindexed(self.out_vtx, self.out_vtx_offsets, self.out_idx, self.old2new,
                              self.new2old, self.status).trim()


def reindex_mesh_batched(vtx, vtx_offsets, idx, elem_offsets, *, tuning=None,
                         sync: bool = True) -> BatchReindexed:
    """Re-index every mesh of a packed batch independently, in one launch
    sequence. Indices in and out are mesh-local."""
    r = BatchedReindexer(vtx, vtx_offsets, idx, elem_offsets, tuning=tuning)
    r.launch()
    res = BatchReindexed(r.out_vtx, r.out_vtx_offsets, r.out_idx, r.old2new, r.new2old, r.status)
    return res.trim() if sync else res


class GraphedBatchedReindexer(BatchedReindexer):
    """A BatchedReindexer whose launch sequence is captured once into a HIP
    graph (torch.cuda.CUDAGraph) and replayed. Inputs are read from the
    tensors given at construction; refill them in place between replays."""

    def __init__(self, *args, **kwargs):
        super().__init__(*args, **kwargs)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=self.vtx.device)
        side.wait_stream(torch.cuda.current_stream(self.vtx.device))
        with torch.cuda.stream(side):
            self.launch()  # warm-up outside the capture (loads code objects)
        torch.cuda.current_stream(self.vtx.device).wait_stream(side)
        with torch.cuda.graph(self.graph):
            self.launch()

    def replay(self):
        self.graph.replay()


_DT = {torch.float32: 0, torch.float64: 1}


def _raise_on_status(status: torch.Tensor, where: str):
    """One device->host read of a status word written by the library."""
    st = int(status.cpu()[0])
    if st == MRX_ERR_INDEX_OUT_OF_RANGE:
        raise IndexError(f"{where}: a new2old entry is out of range")
    check(st, where)


class GatherAttrs(torch.autograd.Function):
    """new_attrs[j, :] = attrs[new2old[j], :] with a hand-written scatter
    backward. new2old is a frozen int32 map (no gradient).

    ``injective=True`` promises that new2old has no repeated entry (true for
    the new2old of a re-index); the backward then writes each gradient row
    with a plain store. The default (False) accumulates with atomics, which
    is correct for every map. ``validate=True`` (default) has the forward
    report out-of-range map entries through a device status word and raise
    IndexError (one device->host read); with False such entries silently
    give zero rows and dropped gradients."""

    @staticmethod
    def forward(ctx, attrs: torch.Tensor, new2old: torch.Tensor, injective: bool = False,
                validate: bool = True):
        if attrs.dtype not in _DT or attrs.dim() != 2 or not attrs.is_cuda:
            raise ValueError("attrs must be a [N, C] fp32/fp64 device tensor")
        if new2old.dtype != torch.int32 or new2old.dim() != 1 or not new2old.is_cuda:
            raise ValueError("new2old must be a 1-D int32 device tensor")
        a = attrs.contiguous()
        idx = new2old.contiguous()
        out = torch.empty((idx.numel(), a.shape[1]), dtype=a.dtype, device=a.device)
        status = torch.zeros(1, dtype=torch.int32, device=a.device) if validate else None
        check(load().mrx_gather_attrs(_ptr(a), a.shape[0], a.shape[1], _DT[a.dtype], _ptr(idx),
                                      idx.numel(), _ptr(out), _ptr(status),
                                      ctypes.c_void_p(_stream_handle(a.device))),
              "mrx_gather_attrs")
        if validate:
            _raise_on_status(status, "mrx_gather_attrs")
        ctx.save_for_backward(idx)
        ctx.num_old = a.shape[0]
        ctx.injective = bool(injective)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (idx,) = ctx.saved_tensors
        g = grad_out.contiguous()
        grad = torch.empty((ctx.num_old, g.shape[1]), dtype=g.dtype, device=g.device)
        # the map is the one the forward read (and, with validate, checked)
        check(load().mrx_gather_attrs_backward(_ptr(g), g.shape[0], g.shape[1], _DT[g.dtype], _ptr(idx),
                                               ctx.num_old, _ptr(grad), int(ctx.injective), None,
                                               ctypes.c_void_p(_stream_handle(g.device))),
              "mrx_gather_attrs_backward")
        return grad, None, None, None


def gather_attrs(attrs: torch.Tensor, new2old: torch.Tensor, injective: bool = False,
                 validate: bool = True) -> torch.Tensor:
    """Differentiable attribute gather (see GatherAttrs). Pass
    ``injective=True`` for the new2old of a re-index to get the exact
    store-based backward."""
    return GatherAttrs.apply(attrs, new2old, injective, validate)

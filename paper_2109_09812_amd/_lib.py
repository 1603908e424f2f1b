"""ctypes binding of libmeshrx.so (argument marshalling only).

The library must have been built in-tree (``python -m
paper_2109_09812_amd.build``); there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmeshrx.so")

MRX_OK = 0
MRX_ERR_INVALID_ARGUMENT = 1
MRX_ERR_WORKSPACE_TOO_SMALL = 2
MRX_ERR_INDEX_OUT_OF_RANGE = 3
MRX_ERR_TOO_LARGE = 4
MRX_ERR_HIP = 5
MRX_ERR_UNSUPPORTED = 6
MRX_ERR_INTERNAL = 7
MRX_ERR_NOALLOC_TOO_LARGE = 8
MRX_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

# Every symbol include/meshrx.h declares.
EXPORTS = (
    "mrx_abi_version", "mrx_status_string", "mrx_tuning_count", "mrx_tuning_get",
    "mrx_reindex_workspace_size", "mrx_reindex_mesh", "mrx_reindex_mesh_noalloc", "mrx_reindex_mesh_batched",
    "mrx_merge_meshes", "mrx_extract_submesh",
    "mrx_gather_attrs", "mrx_gather_attrs_backward",
    "mrx_profile_enable", "mrx_profile_count", "mrx_profile_get",
)


MRX_TUNING_WIDE_LOOKBACK = 1
MRX_TUNING_CLAIMED_TILES = 2
MRX_TUNING_SORT_ALL = 4
MRX_TUNING_HASH_GROUPS = 8
MRX_TUNING_BANDS = 16


class Tuning(ctypes.Structure):
    _fields_ = [("digit_bits", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("items_per_thread", ctypes.c_int32), ("flags", ctypes.c_int32)]

    def as_tuple(self):
        """The kernel shape (flags excluded)."""
        return (self.digit_bits, self.block_threads, self.items_per_thread)

    def as_key(self):
        """The kernel shape and the flags."""
        return (self.digit_bits, self.block_threads, self.items_per_thread, self.flags)


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t

_SIGS = {
    "mrx_abi_version": (_i32, []),
    "mrx_status_string": (ctypes.c_char_p, [_i32]),
    "mrx_tuning_count": (_i32, [_i32]),
    "mrx_tuning_get": (_i32, [_i32, _i32, ctypes.POINTER(Tuning)]),
    "mrx_reindex_workspace_size": (_i32, [_i64, _i32, _i64, _i32, ctypes.POINTER(Tuning),
                                          ctypes.POINTER(_sz)]),
    "mrx_reindex_mesh": (_i32, [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _sz, ctypes.POINTER(Tuning), _vp]),
    "mrx_reindex_mesh_noalloc": (_i32, [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.POINTER(Tuning), _vp]),
    "mrx_reindex_mesh_batched": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp, _i64, _i32, _i32, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(Tuning), _vp]),
    "mrx_merge_meshes": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp, _sz, ctypes.POINTER(Tuning), _vp]),
    "mrx_extract_submesh": (_i32, [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, _sz, ctypes.POINTER(Tuning), _vp]),
    "mrx_gather_attrs": (_i32, [_vp, _i64, _i32, _i32, _vp, _i64, _vp, _vp, _vp]),
    "mrx_gather_attrs_backward": (_i32, [_vp, _i64, _i32, _i32, _vp, _i64, _vp, _i32, _vp, _vp]),
    "mrx_profile_enable": (_i32, [_i32]),
    "mrx_profile_count": (_i32, []),
    "mrx_profile_get": (_i32, [_i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float)]),
}

_lib = None


class MeshrxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


def load(path: str | None = None):
    """Load the library (once). Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2109_09812_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().mrx_status_string(int(status)).decode()


def check(status: int, where: str):
    if status != MRX_OK:
        raise MeshrxError(status, where)


def tunings(vtx_bytes: int):
    """The compiled sort variants for this record width (variant 0 first)."""
    lib = load()
    out = []
    for i in range(lib.mrx_tuning_count(vtx_bytes)):
        t = Tuning()
        check(lib.mrx_tuning_get(vtx_bytes, i, ctypes.byref(t)), "mrx_tuning_get")
        out.append(t)
    return out


def make_tuning(t) -> ctypes.POINTER(Tuning) | None:
    if t is None:
        return None
    if isinstance(t, Tuning):
        return ctypes.pointer(t)
    d, b, i, *rest = t
    return ctypes.pointer(Tuning(d, b, i, rest[0] if rest else 0))


def profile_enable(on: bool = True):
    check(load().mrx_profile_enable(1 if on else 0), "mrx_profile_enable")


def profile_records():
    """[(kernel name, ms)] recorded since profile_enable(True); waits for them."""
    lib = load()
    out = []
    for i in range(lib.mrx_profile_count()):
        name = ctypes.c_char_p()
        ms = ctypes.c_float()
        check(lib.mrx_profile_get(i, ctypes.byref(name), ctypes.byref(ms)), "mrx_profile_get")
        out.append((name.value.decode(), float(ms.value)))
    return out

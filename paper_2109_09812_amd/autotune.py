"""Autotuner for the radix-sort kernel shape (digit width, workgroup size,
items per thread) and the way duplicates are found (sort all vertices by
their full record, or hash grouping; for a batch the key is (mesh id,
record) either way).

Every compiled variant and either strategy compute the identical result, so
tuning is purely a speed choice. Which strategy wins depends on the data (how
many copies each value has), so the tuner times both on the caller's mesh.
For a given workload shape the tuner runs every candidate once,
checks its outputs bit for bit against variant 0's (a variant that differs is
a bug and raises), times a few launches with HIP events, and keeps the
fastest. Results are cached in a JSON file keyed by GPU architecture, record
width, size bucket and batched/single; a cache with another schema or ABI
version, or one naming a variant the loaded library does not have, is ignored and
re-tuned.

Cache path: $MRX_TUNE_CACHE, else ~/.cache/meshrx/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import statistics

import torch

from . import _lib
from .api import BatchedReindexer, Reindexer

SCHEMA = 3


def cache_path() -> str:
    return os.environ.get("MRX_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "meshrx", "tune.json")


def _arch(device) -> str:
    try:
        return str(torch.cuda.get_device_properties(device).gcnArchName).split(":")[0]
    except Exception:  # pragma: no cover - non-ROCm torch builds
        return "unknown"


def shape_key(arch: str, vtx_bytes: int, num_vtx: int, batched: bool) -> str:
    bucket = int(math.ceil(math.log2(max(num_vtx, 2))))
    return f"{arch}|R={vtx_bytes}|n=2^{bucket}|{'batched' if batched else 'single'}"


def load_cache(path: str | None = None) -> dict:
    """Entries of a valid cache file, or {} (missing, corrupt or stale)."""
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    if not isinstance(data, dict) or data.get("schema") != SCHEMA:
        return {}
    if data.get("abi") != _lib.load().mrx_abi_version():
        return {}
    entries = data.get("entries")
    return entries if isinstance(entries, dict) else {}


def save_cache(entries: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"schema": SCHEMA, "abi": _lib.load().mrx_abi_version(), "entries": entries}, f, indent=1)
    os.replace(tmp, path)


_STRATEGY_FLAGS = (_lib.MRX_TUNING_SORT_ALL, _lib.MRX_TUNING_HASH_GROUPS)


def candidates(vtx_bytes: int, num_vtx: int, batched: bool):
    """Every compiled kernel shape, with each strategy a call of this shape
    can take (meshes and batches of 2^30 or more vertices always sort all)."""
    flags = (0,) if num_vtx >= (1 << 30) else _STRATEGY_FLAGS
    out = []
    for t in _lib.tunings(vtx_bytes):
        for fl in flags:
            out.append(_lib.Tuning(t.digit_bits, t.block_threads, t.items_per_thread, fl))
    return out


def cached_tuning(entries: dict, key: str, vtx_bytes: int):
    """The cached candidate for `key` if the loaded library still has its
    shape and its flags are a strategy choice, else None."""
    e = entries.get(key)
    if not isinstance(e, dict) or not isinstance(e.get("tuning"), list) or len(e["tuning"]) != 4:
        return None
    want = tuple(int(x) for x in e["tuning"])
    if want[3] not in (0,) + _STRATEGY_FLAGS:
        return None
    for t in _lib.tunings(vtx_bytes):
        if t.as_tuple() == want[:3]:
            return _lib.Tuning(*want)
    return None


def _outputs(r):
    """The defined part of a launch's outputs (capacity beyond U is not)."""
    res = r.result()
    out = [res.out_vtx, res.out_idx, res.old2new]
    if res.new2old is not None:
        out.append(res.new2old)
    if hasattr(res, "out_vtx_offsets"):
        out.append(res.out_vtx_offsets)
    return out


def _time(launch, reps: int) -> float:
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        launch()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def autotune(vtx: torch.Tensor, idx: torch.Tensor, vtx_offsets: torch.Tensor | None = None,
             elem_offsets: torch.Tensor | None = None, *, reps: int = 5, use_cache: bool = True,
             path: str | None = None, verbose: bool = False):
    """Pick the fastest candidate (compiled sort variant and strategy) for
    this workload shape.

    Returns (tuning, report) where report maps each candidate (d, block,
    items, flags) to its median milliseconds."""
    batched = vtx_offsets is not None
    vtx_bytes = 4 * vtx.shape[1]
    key = shape_key(_arch(vtx.device), vtx_bytes, vtx.shape[0], batched)
    entries = load_cache(path) if use_cache else {}
    hit = cached_tuning(entries, key, vtx_bytes)
    if hit is not None:
        return hit, {"cached": entries[key]}

    ref = None
    report = {}
    best = None
    for t in candidates(vtx_bytes, vtx.shape[0], batched):
        if batched:
            r = BatchedReindexer(vtx, vtx_offsets, idx, elem_offsets, tuning=t)
        else:
            r = Reindexer(vtx, idx, tuning=t)
        r.launch()
        torch.cuda.synchronize()
        outs = _outputs(r)
        if ref is None:
            ref = [o.clone() for o in outs]
        elif not all(torch.equal(a, b) for a, b in zip(ref, outs)):
            raise RuntimeError(f"candidate {t.as_key()} disagrees with the first one")
        ms = _time(r.launch, reps)
        report[t.as_key()] = ms
        if verbose:
            print(f"[autotune] {key} {t.as_key()}: {ms:.4f} ms", flush=True)
        if best is None or ms < best[1]:
            best = (t, ms)
        del r
    if use_cache:
        entries = load_cache(path)
        entries[key] = {"tuning": list(best[0].as_key()), "ms": best[1],
                        "candidates": {",".join(map(str, k)): v for k, v in report.items()}}
        save_cache(entries, path)
    return best[0], report

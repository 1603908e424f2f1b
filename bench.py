"""Throughput of GPU mesh re-indexing on one MI355X.

    python bench.py [--steps K] [--warmup W] [--no-batched] [--no-gather] [--no-cpu]

One step = one whole re-index (used marking, digit histograms, every LSD
radix pass, run-head flag + scan + scatters, compaction, old->new map, index
remap) of the 2048 x 2048-grid triangle soup: 26,398,316 fp32 xyz vertices
(8,380,418 triangles plus 5% never-referenced vertices, randomly permuted).
Inputs are resident in HBM before the timed region; outputs and workspace are
preallocated. Prints ONE JSON line.

Also measured (extra keys of the same line): the batched segmented re-index
of 4096 soups replayed from a HIP graph vs 4096 per-mesh calls, and the
attribute gather forward/backward on the 10M-vertex soup.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "onesweep_soup2048_traffic.json")
# sources that define the measured LSD pass kernel (its body and the device
# helpers it calls; the files that only instantiate and launch it are left out)
PASS_SOURCES = ("paper_2109_09812_amd/csrc/sort_kernels.hpp", "paper_2109_09812_amd/csrc/device_common.hpp")


def pass_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for rel in PASS_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per LSD pass launch from the committed rocprofv3 counter
    summary, or None if the pass kernel's sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != pass_sources_sha():
        return None
    return int(t["read_bytes_per_launch"] + t["write_bytes_per_launch"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def timed_steps(fn, steps, torch):
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def kernel_table(records):
    """name -> (launches, mean ms)"""
    agg = {}
    for name, ms in records:
        c, t = agg.get(name, (0, 0.0))
        agg[name] = (c + 1, t + ms)
    return {k: (c, t / c) for k, (c, t) in agg.items()}


def step_distribution(fn, steps, torch):
    """Per-step times (one event pair around each step): median, p10, p90."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return {"median_ms": round(float(np.median(t)), 5), "p10_ms": round(float(np.percentile(t, 10)), 5),
            "p90_ms": round(float(np.percentile(t, 90)), 5)}


def transfer_times(mesh, rx, torch):
    """Host<->device copies around one re-index (pinned host buffers), timed
    apart from the GPU-resident step: inputs up, all four outputs down."""
    dev = rx.vtx.device
    hv = torch.from_numpy(mesh.vtx.view("int32")).pin_memory()
    hi = torch.from_numpy(mesh.idx).pin_memory()
    outs = [rx.out_vtx, rx.out_idx, rx.old2new, rx.new2old]
    houts = [torch.empty(o.shape, dtype=o.dtype, pin_memory=True) for o in outs]
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    a.record()
    rx.vtx.copy_(hv, non_blocking=True)
    rx.idx.copy_(hi, non_blocking=True)
    b.record()
    for h, o in zip(houts, outs):
        h.copy_(o, non_blocking=True)
    c.record()
    torch.cuda.synchronize()
    up, down = a.elapsed_time(b), b.elapsed_time(c)
    up_b = hv.numel() * 4 + hi.numel() * 4
    down_b = sum(o.numel() * o.element_size() for o in outs)
    return {"h2d_ms": round(up, 3), "h2d_GBps": round(up_b / (up * 1e-3) / 1e9, 1),
            "d2h_ms": round(down, 3), "d2h_GBps": round(down_b / (down * 1e-3) / 1e9, 1)}


def copy_probe(torch, gib=1):
    """Attainable device-to-device copy bandwidth (read + write bytes / time)."""
    dev = torch.device("cuda:0")
    a = torch.empty(gib << 28, dtype=torch.int32, device=dev).fill_(1)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    ms, _ = timed_steps(lambda: b.copy_(a), 5, torch)
    out = round(2 * a.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def reference_model_bytes(n, m, g, u, r, d=8):
    """Algorithmic bytes of the whole re-index pipeline as the plain method
    (Section 2, Steps 1-4: stable LSD sort of (record, id) over every key bit
    with d-bit digits, run-head flags and scan, compaction, scatter and
    remap) must move them: N vertices of r bytes, M index entries, G
    distinct values, U used ones. This fixed per-workload figure turns a
    step time into the pipeline's fraction of the HBM roofline; a faster
    algorithm that moves fewer bytes still divides this same figure."""
    s = r + 4
    p = -(-8 * r // d)
    parts = {
        "histograms": n * r,
        "sort": n * r + n * s + (p - 1) * 2 * n * s,
        "flag_scan": n * s + 4 * n + g * s,
        "remap_mark": 12 * m + 2 * g,
        "compact": g + g * s + 4 * g + u * s,
        "final_remap": 12 * m + 12 * n,
    }
    return sum(parts.values()), parts


def choose_tuning(args, vtx, idx):
    """--tuning if given, else the autotuner's pick (cached per workload shape)."""
    tuning = args.tuning
    if tuning is None:
        from paper_2109_09812_amd import autotune
        t, report = autotune.autotune(vtx, idx, reps=10)
        tuning = t.as_key()
        log(f"autotuned: {tuning} from {report}")
    args.chosen_tuning = tuning
    return tuning


def bench_single(args, torch, mrx, meshgen):
    m = meshgen.cfg2()
    n, k = m.vtx.shape
    r_bytes = 4 * k
    e, a = m.idx.shape
    dev = torch.device("cuda:0")
    vtx = torch.from_numpy(m.vtx.view("int32")).to(dev)
    idx = torch.from_numpy(m.idx).to(dev)
    tuning = choose_tuning(args, vtx, idx)
    rx = mrx.Reindexer(vtx, idx, tuning=tuning)
    log(f"soup2048: N={n} E={e} K={k}; warmup {args.warmup}")
    for _ in range(args.warmup):
        rx.launch()
    torch.cuda.synchronize()
    ms, wall = timed_steps(rx.launch, args.steps, torch)
    log(f"timed {args.steps} steps: {ms:.4f} ms/step (wall {wall:.3f}s)")
    dist = step_distribution(rx.launch, args.steps, torch)
    xfer = transfer_times(m, rx, torch)

    # per-kernel durations from HIP events recorded on the launch stream
    from paper_2109_09812_amd import _lib
    _lib.profile_enable(True)
    ms_prof, _ = timed_steps(rx.launch, args.steps, torch)
    table = kernel_table(_lib.profile_records())
    _lib.profile_enable(False)

    res = rx.result()
    u = res.num_out
    # verify the last result through properties that fix it
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import check_properties
    t0 = time.perf_counter()
    check_properties(m.vtx, m.idx, res.out_vtx.cpu().numpy().view("uint32"), res.out_idx.cpu().numpy(),
                     res.old2new.cpu().numpy(), res.new2old.cpu().numpy(), expected_unique=2048 * 2048)
    log(f"verified ({time.perf_counter() - t0:.1f}s): U={u}")
    extract = bench_extract(args, torch, mrx, m, vtx, idx, u)

    s_elem = r_bytes + 4
    mi = e * a
    # distinct values of the workload: every grid point plus every unused
    # random vertex (uniform fp32 triples, distinct from each other and from
    # the grid points)
    g = u + (n - mi)
    hashed = "group" in table
    # algorithmic bytes per launch of each kernel (reads + writes the step
    # must make; random 1-4 byte accesses counted at their size)
    if hashed:
        model = {
            "mark_histogram": 5 * mi + n * r_bytes,
            "band_partition": 8 * mi,
            "band_mark": 4 * mi + n,
            "band_mark_histogram": 4 * mi + n + n * r_bytes,
            "hash_histogram": n * r_bytes,
            # the used values' elements packed from their span slots, with
            # their key digits counted (the all-element histogram runs only
            # after a bucket overflowed)
            "compact_histogram": 2 * u * s_elem,
            "onesweep_hash_first": n * r_bytes + n + n * s_elem,
            "onesweep_hash": 2 * n * s_elem,
            "group": n * s_elem + 8 * n + 4 * g + 4 * (g - u) + u * s_elem,
            "onesweep": 2 * u * s_elem,
            "finalize": u * s_elem + u * r_bytes + 12 * u,
            "old2new": 12 * n + 4 * g,
            "remap": 12 * mi,
            # Step 4 by vertex bands: pairs in, (new id, vertex) entries out;
            # per band: its entries and index entries in, old2new and the
            # entries' new ids out; per index tile: slot entries and new ids
            # in, out_idx out
            "pair_partition": 8 * n + 4 * n + 8 * n,
            "band_map": 8 * n + 4 * mi + 4 * n + 4 * mi,
            "band_remap": 12 * mi,
        }
    else:
        model = {
            "mark_histogram": 5 * mi + n * r_bytes,
            "mark_used": 5 * mi,
            "histogram": n * r_bytes,
            "onesweep_first": n * r_bytes + n + n * s_elem,
            "onesweep": 2 * n * s_elem,
            "flag_scan": n * s_elem + 8 * n + g * (r_bytes + 4) + g,
            "compact": g * (1 + r_bytes + 4) + u * (r_bytes + 4) + 4 * g,
            "old2new": 12 * n + 4 * g,
            "remap": 12 * mi,
        }
    kernels = {name: {"launches_per_step": c // args.steps, "mean_ms": round(t, 5)}
               for name, (c, t) in table.items()}
    for name, b in model.items():
        if name in kernels and table[name][1] > 0:
            kernels[name]["model_bytes"] = b
            kernels[name]["model_GBps"] = round(b / (table[name][1] * 1e-3) / 1e9, 1)
    if hashed and (args.chosen_tuning[0] in (0, 8)):
        # key passes of the used values whose digit is the same for every used
        # value are skipped and move nothing (read off the sorted output;
        # counted for 8-bit digits)
        ow = res.out_vtx.cpu().numpy().view("uint32").reshape(u, k)
        passes = 4 * k
        dead = sum(1 for p in range(passes)
                   if u == 0 or np.all(((ow[:, k - 1 - p // 4] >> np.uint32(8 * (p % 4))) & np.uint32(255)) ==
                                       ((ow[0, k - 1 - p // 4] >> np.uint32(8 * (p % 4))) & np.uint32(255))))
        model["onesweep"] = model["onesweep"] * (passes - dead) // passes   # average over the launches
    run_bytes = sum(b * table[name][0] // args.steps for name, b in model.items() if name in table)
    # the dominant kernel: the LSD digit pass, every launch of it in the step
    sweep = [nm for nm in table if nm.startswith("onesweep")]
    sweep_ms = sum(table[nm][0] * table[nm][1] for nm in sweep)
    sweep_bytes = sum(table[nm][0] * model.get(nm, 0) for nm in sweep)
    sweep_launches = sum(table[nm][0] for nm in sweep)
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    ref_bytes, _ = reference_model_bytes(n, mi, g, u, r_bytes)
    pipeline = {"model": "Section 2 pipeline with 8-bit LSD digits over all key bits",
                "model_bytes": ref_bytes, "achieved_GBps": round(ref_bytes / (ms * 1e-3) / 1e9, 1),
                "frac": round(ref_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4), "groups": g,
                "strategy": "hash grouping" if hashed else "sort all",
                # the bytes the kernels that actually ran must move
                "run_model_bytes": run_bytes,
                "run_frac": round(run_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4)}
    return dict(n=n, m=e * a, u=u, ms=ms, ms_prof=ms_prof, kernels=kernels, extract=extract, dist=dist, xfer=xfer,
                pipeline=pipeline,
                roofline_pass=dict(achieved=achieved, bytes=sweep_bytes // max(1, sweep_launches),
                                   mean_ms=sweep_ms / max(1, sweep_launches),
                                   launches_per_step=sweep_launches // args.steps),
                r_bytes=r_bytes)


def bench_batched(args, torch, mrx, meshgen):
    log("generating batch4096 ...")
    b = meshgen.cfg4()
    n = b.vtx.shape[0]
    dev = torch.device("cuda:0")
    vtx = torch.from_numpy(b.vtx.view("int32")).to(dev)
    vo = torch.from_numpy(b.vtx_offsets).to(dev)
    idx = torch.from_numpy(b.idx).to(dev)
    eo = torch.from_numpy(b.elem_offsets).to(dev)
    from paper_2109_09812_amd import autotune
    t, report = autotune.autotune(vtx, idx, vo, eo, reps=4)
    log(f"batch4096: N={n} meshes={b.num_meshes}; autotuned {t.as_key()} from {report}; capturing graph")
    g = mrx.GraphedBatchedReindexer(vtx, vo, idx, eo, tuning=t)
    g.replay()
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 5))
    ms_b, _ = timed_steps(g.replay, reps, torch)
    res = g.result()
    log(f"batched graph replay: {ms_b:.3f} ms")
    # per-kernel view: the same launch sequence outside the graph, with the
    # library's timing events
    from paper_2109_09812_amd import _lib
    br = mrx.BatchedReindexer(vtx, vo, idx, eo, tuning=t)
    br.launch()
    torch.cuda.synchronize()
    _lib.profile_enable(True)
    ms_bp, _ = timed_steps(br.launch, reps, torch)
    btable = kernel_table(_lib.profile_records())
    _lib.profile_enable(False)
    del br
    bkernels = {name: {"launches_per_launch": c // reps, "mean_ms": round(ms_, 4)} for name, (c, ms_) in btable.items()}
    # the plain method's bytes, mesh by mesh (distinct values of a patch soup:
    # its grid points plus its unused random vertices)
    sizes_v = np.diff(b.vtx_offsets)
    sizes_i = np.diff(b.elem_offsets) * 3
    ref_b = 0
    for nb, mb, ub in zip(sizes_v.tolist(), sizes_i.tolist(), b.expected_unique.tolist()):
        ref_b += reference_model_bytes(nb, mb, ub + (nb - mb), ub, 12)[0]
    batched_pipeline = {"model": "Section 2 pipeline per mesh, 8-bit LSD digits over all key bits",
                        "model_bytes": int(ref_b), "frac": round(ref_b / (ms_b * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4)}
    # algorithmic bytes per launch of the kernels of the hash-grouping path
    # (N vertices, M index entries, G distinct and U used values over all
    # meshes; random 1-4 byte accesses counted at their size)
    u_all = int(b.expected_unique.sum())
    g_all = int(u_all + (sizes_v - sizes_i).sum())
    m_all = int(sizes_i.sum())
    s_el = 16
    bmodel = {
        "mark_histogram": 5 * m_all + 12 * n,
        "onesweep_hash_first": 12 * n + n + n * s_el,
        "onesweep_hash": 2 * n * s_el,
        "group": n * s_el + 8 * n + 4 * g_all + 4 * (g_all - u_all) + u_all * s_el,
        "compact_histogram": 2 * u_all * s_el,
        "onesweep": 2 * u_all * s_el,
        "onesweep_mesh": 2 * u_all * s_el,
        "finalize": u_all * s_el + 12 * u_all + 12 * u_all,
        "old2new": 12 * n + 4 * g_all,
        "localize_new2old": 8 * u_all,
        "remap": 12 * m_all,
    } if "group" in btable else {}
    if bmodel and t.as_key()[0] in (0, 8):
        # key passes whose digit is the same for every used value move
        # nothing (read off the output records; 8-bit digits)
        ow = res.out_vtx[:u_all].cpu().numpy().view("uint32").reshape(u_all, 3)
        dead = sum(1 for p in range(12)
                   if u_all == 0 or np.all(((ow[:, 2 - p // 4] >> np.uint32(8 * (p % 4))) & np.uint32(255)) ==
                                           ((ow[0, 2 - p // 4] >> np.uint32(8 * (p % 4))) & np.uint32(255))))
        bmodel["onesweep"] = bmodel["onesweep"] * (12 - dead) // 12   # average over the launches
    for name, nbytes in bmodel.items():
        if name in bkernels and btable[name][1] > 0:
            bkernels[name]["model_bytes"] = nbytes
            bkernels[name]["model_GBps"] = round(nbytes / (btable[name][1] * 1e-3) / 1e9, 1)

    # per-mesh launches: one mrx_reindex_mesh per mesh on one stream, shared
    # workspace, outputs at the mesh's own offsets, no synchronisation; each
    # mesh with the tuning the autotuner picks for its size bucket (tuned on
    # the bucket's largest mesh)
    from paper_2109_09812_amd import _lib
    lib = _lib.load()
    vo_h, eo_h = b.vtx_offsets, b.elem_offsets
    sizes = np.diff(vo_h)
    arch = autotune._arch(dev)
    bucket_of = [autotune.shape_key(arch, 12, int(sz), False) for sz in sizes]
    bucket_tuning = {}
    for key in sorted(set(bucket_of)):
        big = max((i for i in range(b.num_meshes) if bucket_of[i] == key), key=lambda i: sizes[i])
        v0, v1, e0, e1 = int(vo_h[big]), int(vo_h[big + 1]), int(eo_h[big]), int(eo_h[big + 1])
        bt, _ = autotune.autotune(vtx[v0:v1], idx[e0:e1], reps=2)
        bucket_tuning[key] = bt
    log("per-mesh bucket tunings: " + ", ".join(f"{k.split('|')[2]}:{t.as_key()}"
                                                for k, t in sorted(bucket_tuning.items())))
    wsb = max(mrx.workspace_size(int(sizes[i]), 12, int(eo_h[i + 1] - eo_h[i]) * 3, 1, bucket_tuning[bucket_of[i]])
              for i in range(b.num_meshes))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    tptr = {k: _lib.make_tuning(t) for k, t in bucket_tuning.items()}
    out_vtx = torch.empty_like(vtx)
    out_idx = torch.empty_like(idx)
    o2n = torch.empty(n, dtype=torch.int32, device=dev)
    n2o = torch.empty(n, dtype=torch.int32, device=dev)
    counts = torch.zeros(b.num_meshes, dtype=torch.int64, device=dev)
    status = torch.zeros(b.num_meshes, dtype=torch.int32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    calls = []
    for i in range(b.num_meshes):
        v0, v1, e0, e1 = int(vo_h[i]), int(vo_h[i + 1]), int(eo_h[i]), int(eo_h[i + 1])
        calls.append((ctypes.c_void_p(vtx.data_ptr() + 12 * v0), v1 - v0, 12,
                      ctypes.c_void_p(idx.data_ptr() + 12 * e0), e1 - e0, 3,
                      ctypes.c_void_p(out_vtx.data_ptr() + 12 * v0), ctypes.c_void_p(out_idx.data_ptr() + 12 * e0),
                      ctypes.c_void_p(o2n.data_ptr() + 4 * v0), ctypes.c_void_p(n2o.data_ptr() + 4 * v0),
                      ctypes.c_void_p(counts.data_ptr() + 8 * i), ctypes.c_void_p(status.data_ptr() + 4 * i),
                      ctypes.c_void_p(ws.data_ptr()), wsb, tptr[bucket_of[i]], stream))
    f = lib.mrx_reindex_mesh

    def per_mesh():
        for c in calls:
            f(*c)

    per_mesh()
    torch.cuda.synchronize()
    per_reps = [timed_steps(per_mesh, 1, torch)[0] for _ in range(3)]
    ms_p = float(np.median(per_reps))
    log(f"per-mesh launches: {ms_p:.3f} ms (median of {per_reps})")
    same = (torch.equal(out_idx, res.out_idx) and torch.equal(o2n, res.old2new) and
            torch.equal(counts, res.out_vtx_offsets[1:] - res.out_vtx_offsets[:-1]) and
            int(status.abs().sum()) == 0)
    exp_ok = bool((torch.diff(res.out_vtx_offsets).cpu().numpy() == b.expected_unique).all())
    del g, res, out_vtx, out_idx, o2n, n2o, ws
    torch.cuda.empty_cache()
    merge = bench_merge(args, torch, mrx, b, vtx, vo, idx, eo)
    return {"workload": "batch4096: 4096 soups, log-uniform [100, 200000] triangles, 5% unused",
            "total_vertices": n, "batched_ms": round(ms_b, 3), "per_mesh_ms": round(ms_p, 3),
            "per_mesh_reps_ms": [round(x, 3) for x in per_reps],
            "pipeline_frac": batched_pipeline["frac"], "pipeline": batched_pipeline,
            "kernels": bkernels, "ms_profiled": round(ms_bp, 3),
            "per_mesh_tunings": {k.split("|")[2]: list(t.as_key()) for k, t in sorted(bucket_tuning.items())},
            "batched_vertices_per_s": n / (ms_b * 1e-3), "per_mesh_vertices_per_s": n / (ms_p * 1e-3),
            "speedup": round(ms_p / ms_b, 2), "batched_equals_per_mesh": bool(same),
            "tuning": list(t.as_key()), "strategy": strategy_name(t.as_key()[3]),
            "autotune_best_ms_by_strategy": best_by_strategy(report),
            "closed_form_counts_ok": exp_ok, "merge": merge}


def strategy_name(flags):
    return "hash grouping" if flags & 8 else "sort all" if flags & 4 else "library default"


def best_by_strategy(report):
    """Fastest autotuner time of each strategy (None if the tuner's cache answered)."""
    out = {}
    for key, ms in report.items():
        if not isinstance(key, tuple) or len(key) != 4:
            return None
        name = strategy_name(key[3])
        out[name] = round(min(ms, out.get(name, float("inf"))), 3)
    return out


def _sampled_records_ok(vtx_np, src_rows, out_idx, out_vtx, new2old, rng, count=20000):
    """For sampled index entries: the output vertex an entry points to holds
    the bytes of the input vertex it pointed to, and so does its
    representative."""
    import torch
    flat_src = src_rows.reshape(-1)
    k = rng.integers(0, flat_src.size, size=min(count, flat_src.size))
    kk = torch.from_numpy(k).to(out_idx.device)
    u = out_idx.reshape(-1)[kk].long()
    ov = out_vtx[u].cpu().numpy().view(np.uint32)
    rep = new2old[u].cpu().numpy()
    src = vtx_np.view(np.uint32)[flat_src[k]]
    return bool(np.array_equal(ov, src) and np.array_equal(vtx_np.view(np.uint32)[rep], src))


def bench_extract(args, torch, mrx, mesh, vtx, idx, u_full):
    """Section 3 sub-mesh of half of soup2048's triangles (seeded random)."""
    keep_np = np.random.default_rng(2109).random(idx.shape[0]) < 0.5
    keep = torch.from_numpy(keep_np).to(vtx.device)
    x = mrx.SubmeshExtractor(vtx, idx, keep)
    x.launch()
    torch.cuda.synchronize()
    ms, _ = timed_steps(x.launch, max(1, min(args.steps, 10)), torch)
    r = x.result()
    ok = _sampled_records_ok(mesh.vtx, mesh.idx[keep_np], r.out_idx, r.out_vtx, r.new2old,
                             np.random.default_rng(8))
    n = vtx.shape[0]
    out = {"workload": "soup2048, half of the triangles kept (seeded random)", "ms": round(ms, 3),
           "vertices_per_s": n / (ms * 1e-3), "kept_elements": r.num_elems_out,
           "kept_elements_ok": r.num_elems_out == int(keep_np.sum()), "unique_out": r.num_out,
           "fewer_than_full": bool(r.num_out < u_full), "sampled_records_ok": ok}
    log("extract", out)
    del x, r
    torch.cuda.empty_cache()
    return out


def bench_merge(args, torch, mrx, b, vtx, vo, idx, eo):
    """Section 3 merge of the whole batch4096 into one mesh, with each
    strategy (the overlapping patches give grid points thousands of copies,
    which overflow the hash grouping's buckets: it falls back to sorting
    everything); the faster one is the reported time."""
    from paper_2109_09812_amd import _lib
    times = {}
    for name, fl in (("sort_all", _lib.MRX_TUNING_SORT_ALL), ("hash_groups", _lib.MRX_TUNING_HASH_GROUPS)):
        m = mrx.MeshMerger(vtx, vo, idx, eo, tuning=(0, 0, 0, fl))
        m.launch()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        times[name], _ = timed_steps(m.launch, reps, torch)
        del m
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    m = mrx.MeshMerger(vtx, vo, idx, eo, tuning=(0, 0, 0, _lib.MRX_TUNING_SORT_ALL if best == "sort_all"
                                                  else _lib.MRX_TUNING_HASH_GROUPS))
    m.launch()
    torch.cuda.synchronize()
    ms = times[best]
    r = m.result()
    mesh_of_elem = np.repeat(np.arange(b.num_meshes), np.diff(b.elem_offsets))
    glob = b.idx.astype(np.int64) + b.vtx_offsets[mesh_of_elem][:, None]
    ok = _sampled_records_ok(b.vtx, glob, r.out_idx, r.out_vtx, r.new2old, np.random.default_rng(7))
    n = vtx.shape[0]
    out = {"workload": "batch4096 merged into one mesh", "ms": round(ms, 3), "strategy": best,
           "ms_by_strategy": {k: round(v, 3) for k, v in times.items()},
           "vertices_per_s": n / (ms * 1e-3), "unique_out": r.num_out,
           "fewer_than_per_mesh": bool(r.num_out < int(b.expected_unique.sum())), "sampled_records_ok": ok}
    log("merge", out)
    del m, r
    torch.cuda.empty_cache()
    return out


def bench_gather(args, torch, mrx, meshgen):
    m = meshgen.cfg5_mesh()
    dev = torch.device("cuda:0")
    vtx = torch.from_numpy(m.vtx.view("int32")).to(dev)
    idx = torch.from_numpy(m.idx).to(dev)
    r = mrx.reindex_mesh(vtx, idx)
    attrs, w = meshgen.cfg5_features(m.num_vtx, r.num_out)
    a = attrs.to(dev).requires_grad_(True)
    wd = w.to(dev)
    from paper_2109_09812_amd import _lib
    from paper_2109_09812_amd.api import GatherAttrs

    def step():
        a.grad = None
        out = GatherAttrs.apply(a, r.new2old, True, False)
        out.backward(wd)

    step()
    torch.cuda.synchronize()
    ms, _ = timed_steps(step, max(1, min(args.steps, 10)), torch)
    # kernel-level view
    lib = _lib.load()
    u, c = r.num_out, 16
    out = torch.empty(u, c, device=dev)
    grad = torch.empty(m.num_vtx, c, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fw = lambda: lib.mrx_gather_attrs(ctypes.c_void_p(a.data_ptr()), m.num_vtx, c, 0,
                                      ctypes.c_void_p(r.new2old.data_ptr()), u,
                                      ctypes.c_void_p(out.data_ptr()), None, st)
    bw = lambda: lib.mrx_gather_attrs_backward(ctypes.c_void_p(wd.data_ptr()), u, c, 0,
                                               ctypes.c_void_p(r.new2old.data_ptr()), m.num_vtx,
                                               ctypes.c_void_p(grad.data_ptr()), 1, None, st)
    ms_f, _ = timed_steps(fw, 10, torch)
    ms_b, _ = timed_steps(bw, 10, torch)
    fwd_bytes = u * c * 4 * 2 + 4 * u
    bwd_bytes = m.num_vtx * c * 4 + u * c * 4 * 2 + 4 * u
    return {"workload": "soup10M: 10M-vertex soup, features [10M, 16] fp32",
            "fwd_bwd_autograd_ms": round(ms, 4), "gather_fwd_ms": round(ms_f, 4),
            "gather_fwd_GBps": round(fwd_bytes / (ms_f * 1e-3) / 1e9, 1),
            "gather_bwd_ms": round(ms_b, 4), "gather_bwd_GBps": round(bwd_bytes / (ms_b * 1e-3) / 1e9, 1)}


# The paper's Table 1 (RTX 3090, thrust + CUDA, end to end): quads per side ->
# milliseconds. Context only: other hardware, 8-byte keys, transfers unstated.
PAPER_GPU_MS = {1024: 9.2, 4096: 92.0, 8192: 338.0}


def bench_configs(args, torch, mrx, meshgen):
    """Re-index time of the other workloads (inputs resident in HBM, tuned
    variant, mean over `steps` launches), each checked against its closed-form
    output count."""
    from paper_2109_09812_amd import autotune
    dev = torch.device("cuda:0")
    cases = [("soup256", meshgen.cfg1), ("tets64", meshgen.cfg3), ("soup10M", meshgen.cfg5_mesh)]
    cases += [(f"paper_quads{q}", (lambda q=q: meshgen.paper_quads(q))) for q in (1024, 4096, 8192)]
    out = {}
    for name, make in cases:
        m = make()
        vtx = torch.from_numpy(m.vtx.view("int32")).to(dev)
        idx = torch.from_numpy(m.idx).to(dev)
        expected = m.expected_unique
        del m
        t, _ = autotune.autotune(vtx, idx, reps=2)
        rx = mrx.Reindexer(vtx, idx, tuning=t)
        rx.launch()
        torch.cuda.synchronize()
        ms, _ = timed_steps(rx.launch, args.steps, torch)
        u = rx.result().num_out
        n = vtx.shape[0]
        row = {"num_vertices": n, "record_bytes": 4 * vtx.shape[1], "unique_out": u,
               "closed_form_ok": u == expected, "ms": round(ms, 4),
               "vertices_per_s": round(n / (ms * 1e-3)), "tuning": list(t.as_key())}
        if name.startswith("paper_quads"):
            q = int(name[len("paper_quads"):])
            row["paper_rtx3090_ms"] = PAPER_GPU_MS[q]
        out[name] = row
        log(name, row)
        del rx, vtx, idx
        torch.cuda.empty_cache()
    return out


def cpu_baseline(meshgen):
    """The oracle (serial std::map re-indexer) on the host, 1 thread, on a
    smaller soup of the same recipe, sized to ~10-20 s of work."""
    import oracle
    oracle.build(force=False)
    probe = meshgen.grid_soup(256, 0.05, 2109_09812 + 2, "probe")
    t0 = time.perf_counter()
    oracle.reindex(probe.vtx, probe.idx)
    rate = probe.num_vtx / (time.perf_counter() - t0)
    side = 256
    for s in (384, 512, 768, 1024, 1448):
        if 6.3 * s * s * 1.05 / rate <= 15.0:
            side = s
    sample = meshgen.grid_soup(side, 0.05, 2109_09812 + 2, f"soup{side}")
    t0 = time.perf_counter()
    res = oracle.reindex(sample.vtx, sample.idx)
    dt = time.perf_counter() - t0
    assert res[0].shape[0] == side * side
    return {"value": sample.num_vtx / dt, "unit": "vertices/s", "cores": 1, "kind": "oracle",
            "seconds": round(dt, 2), "host_cpu": cpu_model(),
            "sample": f"{side}x{side}-grid soup, same recipe as the timed workload "
                      f"({sample.num_vtx} vertices, 5% unused)"}


def cpu_parallel_baseline(meshgen):
    """The paper's data-parallel steps on host threads (oracle/parallel_cpu.cpp,
    a stronger CPU baseline than the serial oracle), on the full timed
    workload; checked against the closed-form output count."""
    import oracle
    oracle.build(force=False)
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    m = meshgen.cfg2()
    oracle.reindex_parallel(m.vtx[:100_000], np.minimum(m.idx[:30_000], 99_999), threads)  # warm-up
    t0 = time.perf_counter()
    res = oracle.reindex_parallel(m.vtx, m.idx, threads)
    dt = time.perf_counter() - t0
    assert res[0].shape[0] == 2048 * 2048
    return {"value": m.vtx.shape[0] / dt, "unit": "vertices/s", "threads": threads,
            "kind": "parallel CPU (the paper's data-parallel steps on host threads)",
            "seconds": round(dt, 2), "host_cpu": cpu_model(), "sample": "the full timed workload (soup2048)"}


def kernels_only(args, torch, mrx, meshgen):
    """Profiler target: W + K re-index steps of the timed workload, then a
    plain device copy of 1 GiB (torch copy_) three times, whose counter
    readings calibrate the byte counters against a known size."""
    m = meshgen.cfg2()
    dev = torch.device("cuda:0")
    vtx = torch.from_numpy(m.vtx.view("int32")).to(dev)
    idx = torch.from_numpy(m.idx).to(dev)
    rx = mrx.Reindexer(vtx, idx, tuning=choose_tuning(args, vtx, idx))
    torch.cuda.synchronize()
    for _ in range(args.warmup + args.steps):
        rx.launch()
    torch.cuda.synchronize()
    a = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(7)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "kernels", "steps": args.steps, "warmup": args.warmup,
                      "tuning": list(args.chosen_tuning),
                      "copy_probe_bytes_each_way": a.numel() * 4, "unique_out": rx.result().num_out}))


def batched_kernels_only(args, torch, mrx, meshgen):
    """Profiler target: W + K launches of the 4096-mesh batch (no graph, so
    every kernel shows up on its own)."""
    b = meshgen.cfg4()
    dev = torch.device("cuda:0")
    vtx = torch.from_numpy(b.vtx.view("int32")).to(dev)
    vo = torch.from_numpy(b.vtx_offsets).to(dev)
    idx = torch.from_numpy(b.idx).to(dev)
    eo = torch.from_numpy(b.elem_offsets).to(dev)
    tuning = args.tuning or (8, 256, 16, 8)
    r = mrx.BatchedReindexer(vtx, vo, idx, eo, tuning=tuning)
    torch.cuda.synchronize()
    for _ in range(args.warmup + args.steps):
        r.launch()
    torch.cuda.synchronize()
    # the same 1 GiB copy probe as kernels_only, to calibrate the counters
    a = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(7)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "batched-kernels", "steps": args.steps, "warmup": args.warmup,
                      "tuning": list(tuning), "total_vertices": int(b.vtx.shape[0]),
                      "copy_probe_bytes_each_way": a.numel() * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tuning", type=str, default=None,
                    help="digit_bits,block,items[,flags] e.g. 8,256,16,8 (flags 8: hash grouping, 4: sort all)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-gather", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads' re-index times")
    ap.add_argument("--mode", choices=("full", "kernels", "batched-kernels"), default="full",
                    help="kernels: only the timed re-index steps and a 1 GiB copy probe (for profilers); "
                         "batched-kernels: only W + K launches of the 4096-mesh batch")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(multi-GPU sharding is described in the design notes, not implemented).", file=sys.stderr)
        sys.exit(2)
    args.tuning = tuple(int(x) for x in args.tuning.split(",")) if args.tuning else None

    import torch

    import meshgen
    import paper_2109_09812_amd as mrx
    mrx.load()
    assert torch.cuda.is_available(), "no GPU visible"

    if args.mode == "kernels":
        kernels_only(args, torch, mrx, meshgen)
        return
    if args.mode == "batched-kernels":
        batched_kernels_only(args, torch, mrx, meshgen)
        return
    single = bench_single(args, torch, mrx, meshgen)
    extras = {}
    if not args.no_gather:
        extras["gather"] = bench_gather(args, torch, mrx, meshgen)
        log("gather", extras["gather"])
    if not args.no_batched:
        extras["batched"] = bench_batched(args, torch, mrx, meshgen)
        log("batched", extras["batched"])
    if not args.no_configs:
        extras["other_workloads"] = bench_configs(args, torch, mrx, meshgen)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(meshgen)
        log("cpu baseline", cpu)
        extras["cpu_parallel_baseline"] = cpu_parallel_baseline(meshgen)
        log("cpu parallel baseline", extras["cpu_parallel_baseline"])

    n = single["n"]
    ms = single["ms"]
    rp = single["roofline_pass"]
    line = {
        "metric": "input vertices re-indexed/sec + achieved HBM GB/s; batched vs per-mesh launch",
        "value": n / (ms * 1e-3),
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "soup2048: triangle soup of a 2048x2048 grid, 26,398,316 fp32 xyz vertices "
                               "(25,141,254 referenced + 5% unused), 8,380,418 int32 triangles, permuted",
                   "num_vertices": n, "num_indices": single["m"], "unique_out": single["u"],
                   "record_bytes": single["r_bytes"], "tuning": list(args.chosen_tuning)},
        "roofline": {"bound": "hbm", "kernel": "k_onesweep (LSD digit pass; every launch of the step)",
                     "achieved": round(rp["achieved"], 1) if rp["achieved"] else None,
                     "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(rp["achieved"] / PEAK_HBM_GBPS, 4) if rp["achieved"] else None,
                     "traffic": measured_traffic(), "bytes_per_launch": rp["bytes"],
                     "mean_launch_ms": rp["mean_ms"], "launches_per_step": rp["launches_per_step"],
                     # the whole step against the roofline: the plain method's
                     # algorithmic bytes for this workload / step time / peak
                     "pipeline_frac": single["pipeline"]["frac"],
                     "pipeline": single["pipeline"]},
        "cpu_baseline": cpu,
        "kernels": single["kernels"],
        "ms_per_step_profiled": round(single["ms_prof"], 5),
        "step_distribution": single["dist"],
        "transfers_not_in_value": single["xfer"],
        "device_copy_GBps": copy_probe(torch),
        "extract": single["extract"],
    }
    line.update(extras)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

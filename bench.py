"""Benchmark of the compounding hot path on one MI355X.

One step = one whole-spine sweep through the full path: zero the accumulators,
compound 3600 frames (480 x 640 uint8, 0.1 mm pixels, 560 mm path, i.i.d. +-5 deg
jitter) into a 400 x 240 x 1120 grid at 0.5 mm in 57 calls of <= 64 frames, normalise +
hole fill the whole grid, then ALG2 depth map + slab mean/max projections (h = 2, 5, 10).
Inputs are synthetic and already resident in HBM when the timed region starts.

Prints one JSON line.  `value` = frames/s of the whole step.  `roofline` covers the
dominant kernel (the PNN ingest): algorithmic bytes per launch (pixels + maps + 12 bytes
of accumulator read/write per distinct voxel touched by the launch, counted by the CPU
oracle) divided by the launch duration measured with HIP events on the library's stream.
`cpu_baseline` times the CPU oracle on the same step on one host core.
Beside the main line: differentiable splat forward+backward frames/s (512 frames of
320 x 240 into 256 x 192 x 512), single-frame captured-graph ingest from host memory
(frames/s back to back, p50/p99 latency), the real-time pipeline (every frame pushed,
region finalize + depth/projection every 10 frames) and batched 16-sweep ingest frames/s.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s compounded into 0.5 mm voxel grid; % HBM roofline; fwd+bwd frames/s"
HBM_PEAK_GBS = 8000.0
CHUNK = 64
SEG = dict(y_lo=40, k=6, tau_I=128, tau_G=40, r=2, fallback_y=74, half=(2, 5, 10))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


_SWEEP = None


def _distinct_worker(q):
    """Oracle pass over the whole sweep counting, per 64-frame call, the kept pixels, the
    distinct voxels touched and the distinct 64-byte accumulator segments they lie in (16
    uint32 sums or 32 uint16 counts per segment): the accumulator traffic and the atomic
    requests that a perfect merge of the call still has to send."""
    import oracle
    d = _SWEEP
    acc = oracle.Accum(d["grid"])
    prev = np.zeros_like(acc.cnt)
    out = []
    for c in range(0, d["frames"].shape[0], CHUNK):
        kept, U = acc.ingest(d["frames"][c:c + CHUNK], d["poses"][c:c + CHUNK], d["probe"], count_distinct=True)
        idx = np.flatnonzero(acc.cnt != prev)       # voxels this call touched (no count wraps here)
        prev[idx] = acc.cnt[idx]
        out.append((kept, U, int(np.unique(idx >> 4).size), int(np.unique(idx >> 5).size)))
    q.put(out)


def time_oracle_step(d, seg, threads=1, min_seconds=10.0, max_reps=3):
    """CPU baseline: the oracle as it stands, same step (calls of 64 frames, normalise +
    hole fill, ALG2 depth + slabs); threads > 1 runs its multi-thread schedule (threads
    own z planes; same bits).  The step is repeated until about min_seconds of CPU work
    have run.  Returns (seconds per step, repetitions)."""
    import oracle
    reps, total = 0, 0.0
    prm = oracle.seg_params(mode=oracle.ALG2, **seg)
    while reps < max_reps and (reps == 0 or total < min_seconds):
        t0 = time.perf_counter()
        acc = oracle.Accum(d["grid"])
        for c in range(0, d["frames"].shape[0], CHUNK):
            if threads > 1:
                acc.ingest_mt(d["frames"][c:c + CHUNK], d["poses"][c:c + CHUNK], d["probe"], threads)
            else:
                acc.ingest(d["frames"][c:c + CHUNK], d["poses"][c:c + CHUNK], d["probe"])
        if threads > 1:
            V, S, _ = oracle.finalize_mt(d["grid"], acc.sum, acc.cnt, threads)
            oracle.segment_mt(d["grid"], V, S, prm, threads)
        else:
            V, S, _ = oracle.finalize(d["grid"], acc.sum, acc.cnt)
            oracle.segment(d["grid"], V, S, prm)
        total += time.perf_counter() - t0
        reps += 1
    return total / reps, reps


def time_oracle_batched(plan, frames4, threads, per_sweep=100):
    """CPU baseline of the batched workload: the first per_sweep frames of every sweep
    ingested by the oracle (calls of 64, each sweep into its own grid).  Returns frames/s."""
    import oracle
    t0 = time.perf_counter()
    n = 0
    for sw, fr in zip(plan, frames4):
        acc = oracle.Accum(sw["grid"])
        m = min(per_sweep, sw["F"])
        for c in range(0, m, CHUNK):
            k = min(CHUNK, m - c)
            acc.ingest_mt(fr[c:c + k], sw["poses"][c:c + k], sw["probe"], threads)
        n += m
    return n / (time.perf_counter() - t0), n


def time_oracle_splat(d5, n=128):
    """CPU baseline of the differentiable step in FP64 (the oracle, one thread): forward
    splat of the first n frames into the four volumes, overlap loss with its volume
    gradients, backward to intensities and poses.  Returns (frames/s, seconds)."""
    import oracle
    g, p = d5["grid"], d5["probe"]
    t0 = time.perf_counter()
    vols = oracle.splat_forward(g, d5["I"][:n], d5["Tstar"][:n], d5["xi"][:n], p)
    _, G = oracle.overlap_loss(vols)
    oracle.splat_backward(g, d5["I"][:n], d5["Tstar"][:n], d5["xi"][:n], p, G)
    dt = time.perf_counter() - t0
    return n / dt, dt


def counters_record(src_hash, tile):
    """The committed rocprofv3 counter summary of the ingest kernel, if it was taken on the
    current ingest kernel source with the same tile shape; otherwise None."""
    p = os.path.join(ROOT, "profiles", "ingest_cfg2_counters.json")
    try:
        rec = json.load(open(p))
    except (OSError, ValueError):
        return None
    if rec.get("ingest_source_sha256") != src_hash or rec.get("tile") != list(tile):
        return None
    return rec


# device-scope atomic requests (64-byte segments per wave instruction) per second on the
# MI355X, measured by microbench/atomic_rate (profiles/atomics_microbench.txt): 21.6-26.7 G
ATOMIC_REQ_RATE = 23.0e9
# plain VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (the
# published 157.3 TFLOP/s FP32 vector rate counts an FMA as two and packed math as two)
ALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
ALU_OPS_PER_PIXEL = 10


def _per_kernel(csv_path, counter=None):
    """{kernel: {counter: (mean value per dispatch, dispatches)}} from a rocprofv3 --pmc
    run in CSV form (run_counter_collection.csv); kernel names without namespaces and
    arguments."""
    import csv
    agg = {}
    for r in csv.DictReader(open(csv_path)):
        if counter and r["Counter_Name"] != counter:
            continue
        k = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1]
        a = agg.setdefault(k, {}).setdefault(r["Counter_Name"], {})
        a[r["Dispatch_Id"]] = a.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return {k: {c: (sum(v.values()) / len(v), len(v)) for c, v in cs.items()} for k, cs in agg.items()}


def counters_summary(fetch_csv, write_csv, out_json, atomic_csv=None, tile=None):
    """Summarise two rocprofv3 --pmc runs of `bench.py --profile-pass` (FETCH_SIZE, then
    WRITE_SIZE; CSV output) into HBM bytes per ingest launch.  Each counter is scaled by
    what it reads for copy_u32_kernel, which the profile pass runs once on a buffer of
    known size (the accumulator export), so the figure is in true bytes."""
    import synth
    from paper_2412_00058_amd.usv import accumulator_bytes

    g = synth.cfg2(count=0)["grid"]
    copy_bytes = accumulator_bytes(g.dims)
    fetch = {k: v["FETCH_SIZE"] for k, v in _per_kernel(fetch_csv, "FETCH_SIZE").items()}
    write = {k: v["WRITE_SIZE"] for k, v in _per_kernel(write_csv, "WRITE_SIZE").items()}
    f_copy, w_copy = fetch["copy_u32_kernel"][0] * 1024.0, write["copy_u32_kernel"][0] * 1024.0
    kf, kw = copy_bytes / f_copy, copy_bytes / w_copy
    f_ing, n_f = fetch["ingest_kernel"]
    w_ing, n_w = write["ingest_kernel"]
    rec = {"ingest_source_sha256": ingest_source_hash(), "tile": list(tile) if tile else None,
           "fetch_kib_per_dispatch": round(f_ing, 1), "write_kib_per_dispatch": round(w_ing, 1),
           "dispatches": [n_f, n_w], "copy_bytes": copy_bytes,
           "copy_fetch_kib": round(f_copy / 1024.0, 1), "copy_write_kib": round(w_copy / 1024.0, 1),
           "fetch_scale": round(kf, 4), "write_scale": round(kw, 4),
           "hbm_bytes_per_launch": int(f_ing * 1024.0 * kf + w_ing * 1024.0 * kw)}
    if atomic_csv:
        atom = {k: v["TCC_EA0_ATOMIC_sum"] for k, v in _per_kernel(atomic_csv, "TCC_EA0_ATOMIC_sum").items()}
        rec["atomic_requests_per_launch"] = int(atom["ingest_kernel"][0])
    for k in sorted(set(fetch) | set(write)):
        f = fetch.get(k, (0.0, 0))[0]
        w = write.get(k, (0.0, 0))[0]
        print("%-28s FETCH %12.1f KiB  WRITE %12.1f KiB  per dispatch (raw)" % (k, f, w))
    print(json.dumps(rec, indent=1))
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


# wave64 VALU instructions the MI355X can issue per second: 256 CUs x 4 SIMDs, one wave64
# instruction per 4 cycles per SIMD (16 lanes per cycle), 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def pmc_report(csv_paths, stats_csv, fetch_scale=2.0, write_scale=1.0):
    """Per-kernel table of rocprofv3 counters (mean per dispatch) joined with the kernel
    trace's mean duration: HBM bytes from FETCH_SIZE / WRITE_SIZE (KiB, scaled by the copy
    calibration), device atomic requests, VALU instructions and their share of the chip's
    VALU issue rate over the kernel's duration, LDS and SALU instructions, waves."""
    import csv
    dur = {}
    for r in csv.DictReader(open(stats_csv)):
        k = r["Name"].replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1]
        dur[k] = float(r["AverageNs"])
    table = {}
    for pth in csv_paths:
        for k, cs in _per_kernel(pth).items():
            table.setdefault(k, {}).update({c: v[0] for c, v in cs.items()})
    lines = []
    for k in sorted(table):
        c = table[k]
        parts = ["%-32s" % k]
        ns = dur.get(k)
        if ns:
            parts.append("%9.1f us" % (ns / 1e3))
        if "FETCH_SIZE" in c:
            parts.append("fetch %8.2f MB" % (c["FETCH_SIZE"] * 1024 * fetch_scale / 1e6))
        if "WRITE_SIZE" in c:
            parts.append("write %8.2f MB" % (c["WRITE_SIZE"] * 1024 * write_scale / 1e6))
        if "TCC_EA0_ATOMIC_sum" in c:
            parts.append("atomic req %9.0f" % c["TCC_EA0_ATOMIC_sum"])
        if "SQ_INSTS_VALU" in c:
            parts.append("VALU insts %10.0f" % c["SQ_INSTS_VALU"])
            if ns:
                parts.append("VALU issue %5.1f%%" % (100.0 * c["SQ_INSTS_VALU"] / (ns * 1e-9 * VALU_ISSUE_PEAK)))
        for name, lab in (("SQ_INSTS_LDS", "LDS"), ("SQ_INSTS_SALU", "SALU"), ("SQ_WAVES", "waves")):
            if name in c:
                parts.append("%s %9.0f" % (lab, c[name]))
        if "SQ_ACTIVE_INST_VALU" in c and "SQ_BUSY_CU_CYCLES" in c and c["SQ_BUSY_CU_CYCLES"] > 0:
            parts.append("VALU active/CU-busy %5.2f" % (c["SQ_ACTIVE_INST_VALU"] / c["SQ_BUSY_CU_CYCLES"]))
        lines.append("  ".join(parts))
    return "\n".join(lines)


def ingest_source_hash():
    """SHA-256 of what defines the ingest kernel: ingest.hip and the ingest section of
    usv_internal.h (from its start to the finalize section)."""
    csrc = os.path.join(ROOT, "paper_2412_00058_amd", "csrc")
    h = hashlib.sha256()
    h.update(open(os.path.join(csrc, "ingest.hip"), "rb").read())
    hdr = open(os.path.join(csrc, "usv_internal.h"), "rb").read()
    cut = hdr.find(b"// ---- finalize")
    h.update(hdr if cut < 0 else hdr[:cut])
    return h.hexdigest()


def bench_splat(torch, usv, steps, d=None):
    import synth
    d = synth.cfg5() if d is None else d
    g = d["grid"]
    F = d["I"].shape[0]
    ctx = usv.SplatContext(g.dims, g.origin_mm, g.voxel_mm, d["probe"].width, d["probe"].height,
                           d["probe"].pixel_mm, F)
    I = torch.from_numpy(d["I"]).cuda()
    T = torch.from_numpy(d["Tstar"]).cuda()
    xi = torch.from_numpy(d["xi"]).cuda()
    vols = torch.empty((4, g.nvox), dtype=torch.float32, device="cuda")
    grads = torch.empty_like(vols)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    dI = torch.empty_like(I)
    dxi = torch.empty((F, 6), dtype=torch.float64, device="cuda")
    L = usv.lib()
    vp = lambda t: C.c_void_p(t.data_ptr())

    def step():
        L.usv_splat_forward(ctx.h, vp(I), vp(T), vp(xi), F, vp(vols))
        L.usv_overlap_loss(ctx.h, vp(vols), vp(loss), vp(grads))
        L.usv_splat_backward(ctx.h, vp(I), vp(T), vp(xi), F, vp(grads), vp(dI), vp(dxi))

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ctx.close()
    return F / dt, dt * 1e3


def bench_refine(torch, usv, iters=150):
    """Rigid-motion refinement at 256 frames of 320 x 240 (two interleaved passes with a
    1.1 mm / 1.1 deg patient motion between them): ms per device-side Adam step (forward
    splat, loss, pose-only backward, update) and the residual motion after `iters` steps,
    measured with the matrix exponential of the twist (scipy), not the library."""
    import math
    import scipy.linalg
    import synth
    d = synth.two_pass_case()
    g, p = d["grid"], d["probe"]
    F = d["I"].shape[0]
    ctx = usv.SplatContext(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, F)
    I = torch.from_numpy(d["I"]).cuda()
    T = torch.from_numpy(d["Tstar"]).cuda()
    kw = dict(iters=iters, lr_rho=0.1, lr_omega=math.radians(0.1))
    ctx.refine_motion(I, T, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xi, L = ctx.refine_motion(I, T, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    x = xi.cpu().numpy()
    hat = np.zeros((4, 4))
    hat[:3, 3] = x[:3]
    hat[:3, :3] = [[0, -x[5], x[4]], [x[5], 0, -x[3]], [-x[4], x[3], 0]]
    E = scipy.linalg.expm(hat) @ np.linalg.inv(d["delta"])
    ang = math.degrees(math.acos(min(1.0, (np.trace(E[:3, :3]) - 1.0) / 2.0)))
    Lh = L.cpu().numpy()
    return dt * 1e3 / iters, float(np.linalg.norm(E[:3, 3])), ang, float(Lh[-1] / Lh[0])


def bench_cut(torch, usv, d, frames, vol, pid, reps=3):
    """Image-space tissue segmentation on the whole-spine sweep: (ms of the Alg. 2 bands
    over the 3600-frame device stack, its read rate in GB/s, ms of the whole Spine-volume
    pass = Alg. 2 bands + band copy to the host + cut ingest in calls of 64 + finalize,
    mean kept rows per frame)."""
    F, H, W = frames.shape
    prm = usv.cut_params(y_lo=100, k=6, tau_I=128, tau_G=40, r=5, fallback_row=370, half_rows=50)
    scratch = torch.empty(F * (W + 1), dtype=torch.int16, device="cuda")
    rows = torch.empty((F, 2), dtype=torch.int32, device="cuda")
    usv.cut_rows_alg2(frames, prm, scratch, rows)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        usv.cut_rows_alg2(frames, prm, scratch, rows)
    torch.cuda.synchronize()
    ms_alg2 = (time.perf_counter() - t0) * 1e3 / reps
    gbps = F * H * W / (ms_alg2 * 1e-3) / 1e9
    V = torch.empty(tuple(reversed(d["grid"].dims)), dtype=torch.uint8, device="cuda")
    S = torch.empty_like(V)

    def spine():
        vol.reset()
        usv.cut_rows_alg2(frames, prm, scratch, rows)
        R = rows.cpu().numpy()
        for k in range(0, F, 64):
            vol.ingest_cut(pid, frames[k:k + 64], d["poses"][k:k + 64], R[k:k + 64])
        vol.finalize(out=(V, S))
        return R

    spine()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        R = spine()
    torch.cuda.synchronize()
    ms_spine = (time.perf_counter() - t0) * 1e3 / reps
    return ms_alg2, gbps, ms_spine, float(np.mean(R[:, 1] - R[:, 0] + 1))


def bench_variants(torch, usv, d, frames, reps=2):
    """The comparison compounding rules on the whole-spine sweep, calls of 64 frames:
    (ms of voxel-nearest-neighbour ingest + finalize with dmax 0.5 mm, ms of
    distance-weighted (tent kernel) ingest + finalize)."""
    g, p = d["grid"], d["probe"]
    F = frames.shape[0]
    vn = usv.VNN(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, 0.5)
    P = [np.ascontiguousarray(d["poses"][k:k + 64]) for k in range(0, F, 64)]

    def vnn_pass():
        vn.reset()
        for i, k in enumerate(range(0, F, 64)):
            vn.ingest(frames[k:k + 64], P[i])
        return vn.finalize()

    vnn_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        vnn_pass()
    torch.cuda.synchronize()
    ms_vnn = (time.perf_counter() - t0) * 1e3 / reps
    vn.close()
    del vn
    ctx = usv.SplatContext(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, 64)
    Pd = torch.from_numpy(np.ascontiguousarray(d["poses"])).cuda()
    acc = ctx.dw_clear()

    def dw_pass():
        ctx.dw_clear(acc)
        for k in range(0, F, 64):
            ctx.dw_ingest(acc, frames[k:k + 64], Pd[k:k + 64])
        return ctx.dw_finalize(acc, 0.05)

    dw_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dw_pass()
    torch.cuda.synchronize()
    ms_dw = (time.perf_counter() - t0) * 1e3 / reps
    ctx.close()
    return ms_vnn, ms_dw


def bench_graph(torch, usv, d, n=512, n_lat=200):
    """Real-time path: one frame per captured-graph launch from host memory (pinned
    staging copy, H2D, ingest).  Returns (frames/s back to back, p50 and p99 latency in
    ms of launch + completion for single frames)."""
    g, p = d["grid"], d["probe"]
    vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    gr = usv.Graph(vol, pid)
    L = usv.lib()
    n = min(n, d["frames"].shape[0])
    fr = np.ascontiguousarray(d["frames"][:n])
    P = np.ascontiguousarray(d["poses"][:n].reshape(n, 16))
    fp = [C.c_void_p(fr[i].ctypes.data) for i in range(n)]
    pp = [C.c_void_p(P[i].ctypes.data) for i in range(n)]
    stream = torch.cuda.current_stream()
    for i in range(16):
        L.usv_graph_launch(gr.h, fp[i], pp[i], None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n):
        if L.usv_graph_launch(gr.h, fp[i], pp[i], None) != 0:
            raise RuntimeError("graph launch failed")
    torch.cuda.synchronize()
    rate = n / (time.perf_counter() - t0)
    lat = []
    for i in range(n_lat):
        t = time.perf_counter()
        L.usv_graph_launch(gr.h, fp[i % n], pp[i % n], None)
        stream.synchronize()
        lat.append(time.perf_counter() - t)
    gr.close()
    if vol.status() != 0:
        raise RuntimeError("graph ingest reported an error")
    lat = np.sort(np.array(lat)) * 1e3
    return rate, float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def bench_realtime(torch, usv, d, render_every=10, n_upd=30):
    """Real-time incremental imaging: every whole-spine frame pushed from host memory
    through the pipeline (captured-graph ingest), the touched region finalized and the
    depth map + projections recomputed every `render_every` frames.  Returns (sustained
    frames/s over the sweep including renders, median ms of one display update = push of
    `render_every` frames + render + completion)."""
    g, p = d["grid"], d["probe"]
    vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    pl = usv.Pipeline(vol, pid, usv.seg_params(mode=usv.SEG_ALG2, **SEG), render_every)
    L = usv.lib()
    F = d["frames"].shape[0]
    fr = d["frames"]
    P = np.ascontiguousarray(d["poses"].reshape(F, 16))
    fp = [C.c_void_p(fr[i].ctypes.data) for i in range(F)]
    pp = [C.c_void_p(P[i].ctypes.data) for i in range(F)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(F):
        if L.usv_pipeline_push(pl.h, fp[i], pp[i]) != 0:
            raise RuntimeError("pipeline push failed")
    if L.usv_pipeline_flush(pl.h) != 0:
        raise RuntimeError("pipeline flush failed")
    rate = F / (time.perf_counter() - t0)
    upd = []
    for k in range(n_upd):
        t = time.perf_counter()
        for j in range(render_every):
            i = (k * render_every + j) % F
            L.usv_pipeline_push(pl.h, fp[i], pp[i])
        L.usv_pipeline_flush(pl.h)
        upd.append(time.perf_counter() - t)
    pl.close()
    if vol.status() != 0:
        raise RuntimeError("pipeline reported an error")
    return rate, float(np.median(upd)) * 1e3


def bench_batched(torch, usv, plan, frames4, steps):
    """Batched workload: the 16 sweeps of uneven length (linear and convex probes, each
    with its own grid) with their own distinct frames, compounded by one batched launch
    per pass.  Each probe type is autotuned first on 256 of its frames.  Returns (frames/s,
    ms per pass, frames, in-mask pixel bytes per pass, frames/s of the same sweeps through
    plain calls of 64 frames with overlapped launches, pixels kept by one pass: the sum of
    the uint16 counts the accumulators hold after it)."""
    jobs = []
    total = 0
    px_bytes = 0
    tuned = {}
    for sw, fr_h in zip(plan, frames4):
        p, g = sw["probe"], sw["grid"]
        vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
        pid = vol.add_probe(p.width, p.height, p.pixel_mm, None, p.mask)
        fr = torch.from_numpy(fr_h).cuda()
        key = sw["linear"]
        if key not in tuned:
            tuned[key] = vol.autotune(pid, fr[:256], sw["poses"][:256], None)
        else:
            vol.set_tiling(pid, *tuned[key])
        jobs.append((vol, pid, fr, sw["poses"]))
        total += sw["F"]
        inside = p.width * p.height if p.mask is None else int((p.mask != 0).sum())
        px_bytes += sw["F"] * inside
    usv.ingest_batched(jobs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for j in jobs:
            j[0].reset()
        usv.ingest_batched(jobs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kept = 0
    for vol, _, _, _ in jobs:   # the accumulators hold exactly the last pass
        kept += int((vol.cnt.to(torch.int32) & 0xFFFF).sum(dtype=torch.int64).item())
    # the same sweeps through plain calls of 64 frames (overlapped launches), for comparison
    for j in jobs:
        j[0].set_ingest_overlap(True)
    tp = []
    for _ in range(steps):
        for j in jobs:
            j[0].reset()
            j[0].join()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for vol, pid, fr, P in jobs:
            for c in range(0, fr.shape[0], CHUNK):
                vol.ingest(pid, fr[c:c + CHUNK], P[c:c + CHUNK])
        for j in jobs:
            j[0].join()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t1)
    dtp = float(np.median(tp))
    for j in jobs:
        if j[0].status() != 0:
            raise RuntimeError("batched ingest reported an error")
    for j in jobs:
        j[0].close()
    return total / dt, dt * 1e3, total, px_bytes, total / dtp, kept


def bench_pinned(torch, usv, d, reps=2):
    """The whole-spine step fed from pinned host memory: each call's 64 frames are copied
    host -> device (PCIe) into a ring of three device slots on the volume's stream, then
    ingested (launches on that stream, after their copy); then finalize + segment.
    Returns (frames/s, ms per step)."""
    g, p = d["grid"], d["probe"]
    F = d["frames"].shape[0]
    host = torch.from_numpy(d["frames"]).pin_memory()
    ring = torch.empty((3, CHUNK, p.height, p.width), dtype=torch.uint8, device="cuda")
    vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    prm = usv.seg_params(mode=usv.SEG_ALG2, **SEG)
    P = [np.ascontiguousarray(d["poses"][c:c + CHUNK]) for c in range(0, F, CHUNK)]

    def step():
        vol.reset()
        for i, c in enumerate(range(0, F, CHUNK)):
            n = min(CHUNK, F - c)
            slot = ring[i % 3, :n]
            slot.copy_(host[c:c + n], non_blocking=True)
            vol.ingest(pid, slot, P[i])
        V, S = vol.finalize()
        vol.segment_project(prm, V, S)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    if vol.status() != 0:
        raise RuntimeError("pinned-host step reported an error")
    vol.close()
    return F / dt, dt * 1e3


def bench_cfg1(torch, usv, steps=50):
    """Tiny plain sweep (64 frames of 128 x 96 into 64 x 64 x 96): reset, one ingest call,
    finalize, ALG2 depth + slabs, per step; launch-bound.  Also the depth + slab pass on
    that volume alone.  Returns (frames/s, ms per step, ms of segment_project alone)."""
    import synth
    d = synth.cfg1()
    g, p = d["grid"], d["probe"]
    vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    fr = torch.from_numpy(d["frames"]).cuda()
    prm = usv.seg_params(mode=usv.SEG_ALG2, r=2, fallback_y=20, half=(2, 5, 10))
    nx, ny, nz = g.dims
    V = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    S = torch.empty_like(V)
    out = (torch.empty((nz, nx), dtype=torch.int16, device="cuda"),
           torch.empty((3, nz, nx), dtype=torch.float32, device="cuda"),
           torch.empty((3, nz, nx), dtype=torch.float32, device="cuda"))

    def step():
        vol.reset()
        vol.ingest(pid, fr, d["poses"])
        vol.finalize(out=(V, S))
        vol.segment_project(prm, V, S, out)

    for _ in range(5):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        vol.segment_project(prm, V, S, out)
    torch.cuda.synchronize()
    seg_ms = (time.perf_counter() - t0) / steps * 1e3
    vol.close()
    return 64 / dt, dt * 1e3, seg_ms

def splat_pass(args):
    """Three differentiable steps of the 512-frame workload for a profiler (no extras)."""
    import synth
    if args.cache5 and os.path.exists(args.cache5):
        z = np.load(args.cache5, allow_pickle=False)
        d5 = synth.cfg5(n_frames=0)
        d5["I"], d5["Tstar"], d5["xi"] = z["I"], z["Tstar"], z["xi"]
    else:
        d5 = synth.cfg5()
        if args.cache5:
            np.savez(args.cache5, I=d5["I"], Tstar=d5["Tstar"], xi=d5["xi"])
    import torch
    import paper_2412_00058_amd as usv
    fps, ms = bench_splat(torch, usv, 3, d5)
    print(json.dumps({"splat_pass": True, "fwd_bwd_frames_per_s": round(fps, 1), "ms_per_step": round(ms, 3)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the splat and batched lines")
    ap.add_argument("--profile-pass", action="store_true", help="one short pass for rocprofv3 (no oracle, no extras)")
    ap.add_argument("--serial", action="store_true",
                    help="time the step with the ingest launches on one stream (no overlap)")
    ap.add_argument("--extras-only", action="store_true",
                    help="for rocprofv3: only the splat, graph and batched measurements (one pass each)")
    ap.add_argument("--cache", default=None,
                    help="load the generated sweep from this .npz (written there if missing); lets a profiled "
                         "run skip the generator's worker processes")
    ap.add_argument("--counters-summary", nargs="+", metavar="CSV", default=None,
                    help="no GPU: summarise the rocprofv3 --pmc CSV results of the profile pass "
                         "(FETCH_SIZE, WRITE_SIZE[, TCC_EA0_ATOMIC_sum]) into profiles/ingest_cfg2_counters.json")
    ap.add_argument("--pmc-report", nargs="+", metavar="CSV", default=None,
                    help="no GPU: per-kernel counter table of rocprofv3 --pmc CSV results, joined with the "
                         "kernel-trace statistics given by --stats")
    ap.add_argument("--stats", default=None, help="rocprofv3 kernel_stats.csv for --pmc-report")
    ap.add_argument("--splat-pass", action="store_true",
                    help="for rocprofv3: three differentiable steps (forward, loss, backward) on the "
                         "512-frame workload read from --cache5")
    ap.add_argument("--cache5", default=None, help=".npz of the differentiable workload (written if missing)")
    ap.add_argument("--counters-tile", nargs=2, type=int, metavar=("W", "H"), default=None,
                    help="the ingest tile shape of the profiled pass (printed by it), stored with the summary")
    args = ap.parse_args()
    if args.counters_summary:
        dbs = args.counters_summary
        counters_summary(dbs[0], dbs[1], os.path.join(ROOT, "profiles", "ingest_cfg2_counters.json"),
                         dbs[2] if len(dbs) > 2 else None, args.counters_tile)
        return
    if args.pmc_report:
        print(pmc_report(args.pmc_report, args.stats))
        return
    if args.splat_pass:
        splat_pass(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single GPU, and sharding the "
              "path over several GPUs is a documented design, not code", file=sys.stderr)
        sys.exit(2)

    global _SWEEP
    import synth
    print("[bench] generating whole-spine sweep", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    if args.cache and os.path.exists(args.cache):
        z = np.load(args.cache, allow_pickle=False)
        d = synth.cfg2(count=0)
        d["frames"], d["poses"] = z["frames"], z["poses"]
    else:
        d = synth.cfg2()
        if args.cache:
            np.savez(args.cache, frames=d["frames"], poses=d["poses"])
    print("[bench] generated in %.1f s" % (time.perf_counter() - t_gen), file=sys.stderr, flush=True)

    # the batched and differentiable workloads are generated here too, before any GPU call
    # (the generator forks worker processes)
    plan4 = frames4 = d5 = None
    if not args.no_extras and not args.profile_pass:
        t_gen = time.perf_counter()
        plan4 = synth.cfg4_plan()
        frames4 = synth.cfg4_frames(plan4)
        d5 = synth.cfg5()
        print("[bench] batched + differentiable workloads generated in %.1f s" % (time.perf_counter() - t_gen),
              file=sys.stderr, flush=True)

    # the oracle's distinct-voxel pass runs in a child forked before any GPU call
    q = None
    proc = None
    if not args.profile_pass and not args.extras_only:
        _SWEEP = d
        ctx = mp.get_context("fork")
        q = ctx.Queue()
        proc = ctx.Process(target=_distinct_worker, args=(q,), daemon=True)
        proc.start()

    import torch
    import paper_2412_00058_amd as usv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.extras_only:
        out = {"extras_only": True, "fwd_bwd": bench_splat(torch, usv, 3, d5),
               "graph": bench_graph(torch, usv, d, n=128, n_lat=32),
               "refine": bench_refine(torch, usv, 20),
               "batched": bench_batched(torch, usv, plan4, frames4, 1)}
        g, p = d["grid"], d["probe"]
        frames = torch.from_numpy(d["frames"]).cuda()
        vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
        pid = vol.add_probe(p.width, p.height, p.pixel_mm)
        out["cut"] = bench_cut(torch, usv, d, frames, vol, pid, reps=2)
        out["variants"] = bench_variants(torch, usv, d, frames, reps=1)
        print(json.dumps(out))
        return

    g, p = d["grid"], d["probe"]
    F = d["frames"].shape[0]
    frames = torch.from_numpy(d["frames"]).cuda()
    vol = usv.Volume(g.dims, g.origin_mm, g.voxel_mm)
    pid = vol.add_probe(p.width, p.height, p.pixel_mm)
    # tile shape picked by the library's autotuner on the first 1024 frames (untimed); the
    # choice is cached in a temp file so that profiled passes reuse it without re-tuning
    import tempfile
    # consecutive ingest launches overlap on the library's side streams (joined before finalize);
    # the tile is tuned in that mode; the profile pass and the roofline's launch timing
    # then run the launches one after another with the same tile
    vol.set_ingest_overlap(not args.serial)
    vol.autotune(pid, frames[:1024], d["poses"][:1024], os.path.join(tempfile.gettempdir(), "usv_bench_tune.txt"))
    tile = vol.tiling(pid)
    frames_per_launch = vol.chunk(pid)
    overlap = not args.profile_pass and not args.serial
    vol.set_ingest_overlap(overlap)
    nx, ny, nz = g.dims
    V = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    S = torch.empty_like(V)
    prm = usv.seg_params(mode=usv.SEG_ALG2, **SEG)
    dep = torch.empty((nz, nx), dtype=torch.int16, device="cuda")
    mean = torch.empty((3, nz, nx), dtype=torch.float32, device="cuda")
    mx = torch.empty_like(mean)
    L = usv.lib()
    chunks = []
    for c in range(0, F, CHUNK):
        n = min(CHUNK, F - c)
        P = np.ascontiguousarray(d["poses"][c:c + n].reshape(n, 16))
        chunks.append((C.c_void_p(frames[c].data_ptr()), P, P.ctypes.data_as(C.c_void_p), n))
    rp, fp = frames.stride(1), frames.stride(0)
    Vp, Sp = C.c_void_p(V.data_ptr()), C.c_void_p(S.data_ptr())
    outs = [C.c_void_p(t.data_ptr()) for t in (dep, mean, mx)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    host_submit = []

    def step(phases=False):
        """One step.  With phases, events bracket ingest / finalize / segment and the
        ingest streams are joined before the finalize event (so the ingest phase ends
        with its last launch); without, the calls run as a user would make them."""
        vol.reset()
        if phases:
            ev[0].record()
        th = time.perf_counter()
        for fptr, _, pptr, n in chunks:
            st = L.usv_ingest_frames(vol.h, pid, fptr, rp, fp, pptr, n, None)
            if st != 0:
                raise RuntimeError("ingest failed: %d" % st)
        if overlap and phases:
            L.usv_join(vol.h)
        host_submit.append(time.perf_counter() - th)
        if phases:
            ev[1].record()
        L.usv_finalize(vol.h, None, Vp, Sp)
        if phases:
            ev[2].record()
        L.usv_segment_project(vol.h, C.byref(prm), Vp, Sp, *outs)
        if phases:
            ev[3].record()

    def phase_steps(n):
        ph = np.zeros(3)
        for _ in range(n):
            step(phases=True)
            ev[3].synchronize()   # this step's events are read before the next step re-records them
            ph += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
        torch.cuda.synchronize()
        return ph / n

    for _ in range(max(args.warmup, 0 if args.profile_pass else 1)):
        step()
    torch.cuda.synchronize()
    steps = 1 if args.profile_pass else args.steps
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = vol.status()
    if st != 0:
        raise RuntimeError("volume status %d after the timed steps" % st)
    ms_step = (t1 - t0) * 1e3 / steps
    # per-phase times from extra steps with events (not part of the timed region)
    phase = np.zeros(3) if args.profile_pass else phase_steps(3)
    # the same step timed by HIP events on the volume's stream: 2 warm-up + 10 timed runs
    ev_ms = []
    if not args.profile_pass:
        for i in range(12):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step()
            e1.record()
            e1.synchronize()
            if i >= 2:
                ev_ms.append(e0.elapsed_time(e1))
    value = F / (ms_step / 1e3)
    print("[bench] %.3f ms/step  ingest %.3f  finalize %.3f  segment %.3f ms  tile %s  host submit %.3f ms/step" %
          (ms_step, phase[0], phase[1], phase[2], tile, 1e3 * float(np.median(host_submit))), file=sys.stderr,
          flush=True)
    if args.profile_pass:
        # one plain copy of known size (the accumulator export) to calibrate byte counters
        snap = vol.export_accumulators()
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "ms_per_step": ms_step, "tile": list(tile),
                          "copy_bytes": snap.numel() * snap.element_size()}))
        return

    # roofline of the ingest kernel: algorithmic bytes per launch / measured launch time,
    # the launch time from steps with the launches one after another (as in the profiled
    # pass); each call of n frames is split into launches of frames_per_launch
    n_kernel = sum(-(-n // frames_per_launch) for _, _, _, n in chunks)
    overlapped_launch_ms = phase[0] / n_kernel
    if overlap:
        overlap = False
        vol.set_ingest_overlap(False)
        per_launch_ms = phase_steps(3)[0] / n_kernel
    else:
        per_launch_ms = overlapped_launch_ms
    per_chunk = q.get(timeout=600)
    proc.join(timeout=60)
    n_pix = 0
    U = 0
    segs = 0
    for (kept, u, ss, cs), (_, _, _, n) in zip(per_chunk, chunks):
        n_pix += n * p.width * p.height
        U += u
        segs += ss + cs
    alg_bytes = n_pix * 1 + F * 36 + 12 * U
    # distinct voxels are counted per 64-frame call; with smaller launches this undercounts
    # the accumulator bytes (a conservative roofline)
    bytes_launch = alg_bytes / n_kernel
    segs_launch = segs / n_kernel
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    hbm_floor_ms = bytes_launch / (HBM_PEAK_GBS * 1e9) * 1e3
    atomic_floor_ms = segs_launch / ATOMIC_REQ_RATE * 1e3
    rec = counters_record(ingest_source_hash(), tile)
    traffic = rec.get("hbm_bytes_per_launch") if rec else None
    meas_req = rec.get("atomic_requests_per_launch") if rec else None
    # ALU floor: per kept pixel the method needs 3 FP32 adds (the per-column products and
    # per-row constants are shared by a whole column / row), 3 float -> integer
    # conversions, 2 multiply-adds for the linear voxel index and 2 integer adds (sum and
    # count): 10 lane operations, against the chip's 39.3 T lane-operations/s
    alu_ops_launch = ALU_OPS_PER_PIXEL * n_pix / n_kernel
    alu_floor_ms = alu_ops_launch / ALU_PEAK_OPS * 1e3
    floors = {"hbm": hbm_floor_ms, "atomic": atomic_floor_ms, "alu": alu_floor_ms}
    bound = max(floors, key=floors.get)
    if bound == "alu":
        head = {"achieved": round(alu_ops_launch / (per_launch_ms * 1e-3) / 1e12, 2), "peak": ALU_PEAK_OPS / 1e12,
                "unit": "TOP/s"}
    elif bound == "hbm":
        head = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        head = {"achieved": round(segs_launch / (per_launch_ms * 1e-3) / 1e9, 2), "peak": ATOMIC_REQ_RATE / 1e9,
                "unit": "G requests/s"}
    roof = {"bound": bound, **head, "frac": round(floors[bound] / per_launch_ms, 4), "traffic": traffic,
            "kernel": "ingest_kernel (PNN scatter, %d frames per launch)" % frames_per_launch,
            "launch_ms": round(per_launch_ms, 5),
            "floors_ms": {k: round(v, 5) for k, v in floors.items()},
            "hbm": {"alg_bytes_per_launch": int(bytes_launch), "achieved_GBps": round(achieved, 1),
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "distinct_voxels_per_launch": int(U / n_kernel)},
            "alu": {"alg_ops_per_pixel": ALU_OPS_PER_PIXEL, "alg_ops_per_launch": int(alu_ops_launch),
                    "peak_ops_per_s": ALU_PEAK_OPS},
            "atomic": {"alg_segments_per_launch": int(segs_launch),
                       "measured_requests_per_launch": meas_req,
                       "request_excess": round(meas_req / segs_launch, 2) if meas_req else None,
                       "rate_per_s": ATOMIC_REQ_RATE,
                       "rate_source": "measured by microbench/atomic_rate (not a published figure)"},
            "overlapped": {"ingest_phase_ms": round(phase[0], 4), "ms_per_launch": round(overlapped_launch_ms, 5),
                           "frac": round(floors[bound] / overlapped_launch_ms, 4)}}

    extras = {}
    if not args.no_extras:
        try:
            fps, ms = bench_splat(torch, usv, max(3, min(args.steps, 10)), d5)
            extras["fwd_bwd_frames_per_s"] = round(fps, 1)
            extras["fwd_bwd_ms_per_step"] = round(ms, 3)
            # forward + loss + backward against the HBM floor: per pixel I read twice and dI
            # written (4 B each), per voxel the four FP32 volumes written, read by the loss,
            # its four gradients written and read by the backward (16 B each)
            npx, nv5 = int(np.prod(d5["I"].shape)), int(d5["grid"].nvox)
            b5 = 12 * npx + 64 * nv5
            f5 = b5 / (HBM_PEAK_GBS * 1e9) * 1e3
            extras["fwd_bwd_roofline"] = {"bound": "hbm", "alg_bytes": b5, "floor_ms": round(f5, 4),
                                          "step_ms": round(ms, 3), "achieved": round(b5 / (ms * 1e-3) / 1e9, 1),
                                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(f5 / ms, 4)}
        except Exception as e:  # report, do not hide
            extras["fwd_bwd_error"] = repr(e)
        try:
            ms_a2, gbps, ms_sp, kept_rows = bench_cut(torch, usv, d, frames, vol, pid)
            extras["cut_alg2_ms"] = round(ms_a2, 3)
            extras["cut_alg2_read_GBps"] = round(gbps, 1)
            extras["spine_volume_ms"] = round(ms_sp, 3)
            extras["spine_volume_frames_per_s"] = round(F / (ms_sp * 1e-3), 1)
            extras["spine_kept_rows_per_frame"] = round(kept_rows, 1)
        except Exception as e:
            extras["cut_error"] = repr(e)
        try:
            ms_vnn, ms_dw = bench_variants(torch, usv, d, frames)
            extras["vnn_ms_per_sweep"] = round(ms_vnn, 3)
            extras["vnn_frames_per_s"] = round(F / (ms_vnn * 1e-3), 1)
            extras["dw_ms_per_sweep"] = round(ms_dw, 3)
            extras["dw_frames_per_s"] = round(F / (ms_dw * 1e-3), 1)
        except Exception as e:
            extras["variants_error"] = repr(e)
        try:
            ms, rt, ra, drop = bench_refine(torch, usv)
            extras["refine_ms_per_iter"] = round(ms, 4)
            extras["refine_residual_mm"] = round(rt, 5)
            extras["refine_residual_deg"] = round(ra, 5)
            extras["refine_loss_ratio"] = float("%.3g" % drop)
        except Exception as e:
            extras["refine_error"] = repr(e)
        try:
            rate, p50, p99 = bench_graph(torch, usv, d)
            extras["graph_frames_per_s"] = round(rate, 1)
            extras["graph_latency_ms_p50"] = round(p50, 4)
            extras["graph_latency_ms_p99"] = round(p99, 4)
        except Exception as e:
            extras["graph_error"] = repr(e)
        try:
            rate, upd = bench_realtime(torch, usv, d)
            extras["realtime_frames_per_s"] = round(rate, 1)
            extras["realtime_update_ms_p50"] = round(upd, 3)
        except Exception as e:
            extras["realtime_error"] = repr(e)
        try:
            fps, ms, tot, pxb, fps_plain, kept = bench_batched(torch, usv, plan4, frames4, max(2, min(args.steps, 5)))
            extras["batched_frames_per_s"] = round(fps, 1)
            extras["batched_same_frames_plain_calls_frames_per_s"] = round(fps_plain, 1)
            extras["batched_ms_per_pass"] = round(ms, 3)
            extras["batched_frames"] = tot
            extras["batched_pixel_GBps"] = round(pxb / (ms * 1e-3) / 1e9, 1)
            extras["batched_hbm_frac_pixels_only"] = round(pxb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            # the batched kernel's ALU floor, as for the plain launch: ALU_OPS_PER_PIXEL lane
            # operations per kept pixel; the pass time also holds the 16 volumes' resets
            floor_ms = ALU_OPS_PER_PIXEL * kept / ALU_PEAK_OPS * 1e3
            extras["batched_roofline"] = {
                "bound": "alu", "kept_pixels": kept, "alg_ops_per_pass": ALU_OPS_PER_PIXEL * kept,
                "achieved": round(ALU_OPS_PER_PIXEL * kept / (ms * 1e-3) / 1e12, 2), "peak": ALU_PEAK_OPS / 1e12,
                "unit": "TOP/s", "floor_ms": round(floor_ms, 3), "frac": round(floor_ms / ms, 4),
                "pass_ms": round(ms, 3)}
        except Exception as e:
            extras["batched_error"] = repr(e)
        try:
            fps, ms = bench_pinned(torch, usv, d)
            extras["pinned_host_frames_per_s"] = round(fps, 1)
            extras["pinned_host_ms_per_step"] = round(ms, 3)
        except Exception as e:
            extras["pinned_host_error"] = repr(e)
        try:
            fps, ms, seg_ms = bench_cfg1(torch, usv)
            extras["cfg1_frames_per_s"] = round(fps, 1)
            extras["cfg1_ms_per_step"] = round(ms, 4)
            extras["cfg3_segment_ms"] = {"whole_spine_grid": round(phase[2], 4), "cfg1_grid": round(seg_ms, 4)}
        except Exception as e:
            extras["cfg1_error"] = repr(e)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on the same step", file=sys.stderr, flush=True)
        nproc = os.cpu_count() or 1
        threads = max(1, min(nproc, int(os.environ.get("OMP_NUM_THREADS", nproc))))
        t_mt, reps_mt = time_oracle_step(d, SEG, threads=threads, min_seconds=5.0, max_reps=2)
        t_1, reps_1 = time_oracle_step(d, SEG, threads=1, min_seconds=1.0, max_reps=1)
        cpu = {"value": round(F / t_mt, 2), "unit": "frames/s", "cores": threads, "kind": "oracle",
               "sample": "the full step (3600 frames in 57 calls + normalise/fill + ALG2 depth and slabs), "
                         "%d repetition(s), %d threads of the oracle's multi-thread schedule (threads own z "
                         "planes; same bits as one thread), %s, %d logical CPUs" % (reps_mt, threads, cpu_model(), nproc),
               "seconds": round(t_mt, 2), "host_nproc": nproc,
               "single_thread": {"value": round(F / t_1, 2), "seconds": round(t_1, 2)}}
        if plan4 is not None:
            try:
                fps4, n4 = time_oracle_batched(plan4, frames4, threads)
                cpu["batched_frames_per_s"] = round(fps4, 2)
                cpu["batched_sample"] = "first 100 frames of each of the 16 sweeps (%d frames), %d threads" % (n4, threads)
            except Exception as e:
                cpu["batched_error"] = repr(e)
        if d5 is not None:
            try:
                fps5, t5 = time_oracle_splat(d5)
                cpu["fwd_bwd_fp64_frames_per_s"] = round(fps5, 2)
                cpu["fwd_bwd_fp64_sample"] = ("128 of the 512 frames: FP64 forward splat, overlap loss and "
                                              "backward, one thread, %.1f s" % t5)
            except Exception as e:
                cpu["fwd_bwd_error"] = repr(e)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "frames/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "whole-spine sweep: 3600 frames 480x640 uint8 (0.1 mm px), 560 mm path with "
                                  "+-20 mm meander and +-5 deg jitter, grid 400x240x1120 @ 0.5 mm, calls of 64 "
                                  "frames, full finalize, ALG2 depth + slab projection h=2/5/10",
                      "tile": list(tile), "frames_per_launch": frames_per_launch,
                      "ingest_streams": 1 if args.serial else usv.INGEST_STREAMS, "parallelism": "single GPU"},
           "breakdown_ms": {"ingest": round(phase[0], 4), "finalize": round(phase[1], 4),
                            "segment_project": round(phase[2], 4)},
           "event_ms_per_step": {"median": round(float(np.median(ev_ms)), 4), "min": round(float(np.min(ev_ms)), 4),
                                 "runs": len(ev_ms), "warmup": 2},
           "roofline": roof, "cpu_baseline": cpu}
    if not args.profile_pass:
        try:
            # finalize phase (zero fill of the outputs + stencil) against its HBM floor: the
            # accumulators of the live box (touched box dilated by one) read once, 6 B per voxel,
            # and V + state written for the whole grid, 2 B per voxel
            tb = usv.dirty_box(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, p.calib, d["poses"])
            live = 1
            for k in range(3):
                live *= max(0, min(g.dims[k], tb.hi[k] + 1) - max(0, tb.lo[k] - 1))
            nvox = g.dims[0] * g.dims[1] * g.dims[2]
            fbytes = 6 * live + 2 * nvox
            ffloor = fbytes / (HBM_PEAK_GBS * 1e9) * 1e3
            out["finalize_roofline"] = {"bound": "hbm", "alg_bytes": int(fbytes), "live_voxels": int(live),
                                        "floor_ms": round(ffloor, 4), "phase_ms": round(phase[1], 4),
                                        "achieved": round(fbytes / (phase[1] * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": round(ffloor / phase[1], 4) if phase[1] > 0 else None}
            # depth map + slab projection against its HBM floor: V read once over the scanned
            # rows [y_lo, ny), state over each column's widest slab, the depth map and the mean /
            # max projections written
            nx, ny, nz = g.dims
            hmax = max(SEG["half"])
            sbytes = (nx * nz * (ny - SEG["y_lo"]) + nx * nz * min(ny, 2 * hmax + 1)
                      + 2 * nx * nz + 2 * 4 * len(SEG["half"]) * nx * nz)
            sfloor = sbytes / (HBM_PEAK_GBS * 1e9) * 1e3
            out["segment_roofline"] = {"bound": "hbm", "alg_bytes": int(sbytes), "floor_ms": round(sfloor, 4),
                                       "phase_ms": round(phase[2], 4),
                                       "achieved": round(sbytes / (phase[2] * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                       "unit": "GB/s", "frac": round(sfloor / phase[2], 4) if phase[2] > 0 else None}
        except Exception as e:   # the main line is printed whatever happens here
            out["phase_roofline_error"] = repr(e)
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: batched polar-stroking tessellation on one MI355X.

Workload (one "step" = count -> scan -> emit with arc length, the whole hot
path, over one batch): 4,096 open paths with log-uniform [1,512] segments
(60/25/15 % cubic/quadratic/conic, 5 % cusp and 5 % coincident-point cubics),
coordinates in [0,4096)^2, width log-uniform [0.5,64], q = pi/64, round joins,
butt caps; synthetic, seeded.  The batched form replays one hipGraph per step.

Prints one JSON line: stroke vertices/s of the batched form, the emit kernel's
HBM roofline fraction, the per-path form on the same GPU, the FP64 CPU oracle
timed on the host, and the maximum vertex / arc-length error against it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """sha256 over the kernel sources; a stored counter summary applies only to
    the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("ps_kernels.hip", "ps_device.h"):
        with open(os.path.join(ROOT, "paper_2007_00308_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(per_launch_config: str):
    """HBM bytes per emit launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    stored in profiles/ (scaled by the copy-kernel calibration), or None when
    they were taken on other kernel sources or another emit mapping."""
    path = os.path.join(ROOT, "profiles", "emit_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    return rec.get("emit_configs", {}).get(per_launch_config)


def algorithmic_bytes(V: int, S: int, P: int) -> int:
    # each vertex written once as x, y, s (FP32); control data read once per
    # segment (4 x,y FP32 points, kind, weight); path data (CSR, width, styles)
    return 12 * V + 37 * S + 10 * P


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp32_fixup", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-per-path", action="store_true", help="skip the per-path form")
    ap.add_argument("--no-c5", action="store_true", help="skip the 2^20-segment leg at q = pi/256")
    ap.add_argument("--no-c1c3", action="store_true", help="skip the single-path legs (C1, C3)")
    ap.add_argument("--profile", action="store_true", help="few steps, no oracle (for rocprofv3)")
    ap.add_argument("--emit-config", default=None, metavar="M,K,W",
                    help="fixed emit mapping (PS_MAP_* mapping, ribs per lane, waves per group) "
                         "instead of the plan's autotuning, e.g. for profiles of one mapping")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--study", choices=["precision", "c3", "c5", "emit", "c1", "facets", "coverage", "mappings"],
                    default=None,
                    help="secondary measurements: the near-degenerate precision study, the long "
                         "dashed path, or the stress configuration at q in {pi/16, pi/64, pi/256}")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the stroking path runs on one GPU: --gpus must be 1"}), flush=True)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print(json.dumps({"error": "--steps must be >= 1 and --warmup >= 0"}), flush=True)
        return 2
    if args.profile:
        args.no_cpu = True
        args.no_per_path = True
        args.no_c5 = True
        args.no_c1c3 = True

    import torch
    import paper_2007_00308_amd as ps
    from paper_2007_00308_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.study:
        return STUDIES[args.study](args, torch, ps, W, dev)
    prec = {"fp32": ps.PS_PREC_FP32, "fp32_fixup": ps.PS_PREC_FP32_FIXUP, "fp64": ps.PS_PREC_FP64}[args.precision]

    t0 = time.time()
    b = W.config2_fast()
    log(f"workload {b.name}: {b.n_paths} paths, {b.n_segs} segments ({time.time() - t0:.1f}s)")
    db = ps.DeviceBatch(b, device=dev)

    # size the outputs from one counting pass (outside the timed region)
    first = ps.stroke(db, b.q, precision=prec)
    R = first["total_ribs"]
    V = 2 * R
    cap = V
    log(f"ribs {R}, vertices {V}")
    del first
    torch.cuda.synchronize()

    emit = tuple(int(x) for x in args.emit_config.split(",")) if args.emit_config else (ps.PS_MAP_DEFAULT, 0, 0)
    plan = ps.Plan(db, b.q, vertex_capacity=cap, precision=prec, emit=emit)
    mapping, K, waves = plan.config()
    log(f"plan: emit mapping {mapping} K={K} waves/group={waves} ({'given' if args.emit_config else 'autotuned'})")
    stream = torch.cuda.current_stream()

    # one event pair per timed step around the emit graph, on the stream the
    # kernels run on (recorded once first so that the events exist)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for a, c in ev:
        a.record(stream); c.record(stream)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, c in ev:
        plan.launch_timed(a, c)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = 1e3 * t_total / args.steps
    st = plan.status()
    assert st.flags == 0, f"status flags {st.flags}"
    assert st.total_ribs == R
    vps = V / (ms_step * 1e-3)
    B_alg = algorithmic_bytes(V, b.n_segs, b.n_paths)
    log(f"batched: {ms_step:.3f} ms/step, {vps / 1e9:.2f} G vertices/s, "
        f"{B_alg / (ms_step * 1e-3) / 1e9:.0f} GB/s; fix-ups {st.fixups}")

    # the emit (tile table + emit kernel) of every timed step, from its events
    emit_ms = sum(a.elapsed_time(c) for a, c in ev) / len(ev)
    emit_bytes = algorithmic_bytes(V, b.n_segs, b.n_paths)
    emit_gbs = emit_bytes / (emit_ms * 1e-3) / 1e9
    log(f"emit call: {emit_ms:.3f} ms, {emit_gbs:.0f} GB/s algorithmic ({emit_gbs / HBM_PEAK_GBS:.1%} of peak)")

    if args.copy_calib:
        n = args.copy_calib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calib} MiB read + written")

    per_path = None
    if not args.no_per_path:
        # plain per-path form: count, scan, emit launched per path into the same output
        log("per-path form ...")
        off = plan.offsets.cpu().numpy()
        sb = b.seg_begin.astype(np.int64)
        subs = []
        max_ws = 0
        for p in range(b.n_paths):
            sub = ps.DeviceBatch(b.subset([p]), device=dev)
            r0 = int(off[2 * sb[p] + p]); r1 = int(off[2 * sb[p + 1] + p + 1])
            subs.append((sub, r0, r1))
            max_ws = max(max_ws, ps.ps_workspace_bytes(sub, plan.params, 2 * (r1 - r0)))
        ws = ps.alloc_workspace(max_ws, dev)
        lr = torch.empty(2 * int(np.diff(sb).max()) + 1, dtype=torch.int32, device=dev)
        of = torch.empty(lr.numel() + 1, dtype=torch.int64, device=dev)
        px, py, pv = torch.empty_like(plan.vx), torch.empty_like(plan.vy), torch.empty_like(plan.vs)

        def run_per_path():
            for sub, r0, r1 in subs:
                ps.ps_count(sub, plan.params, lr, ws)
                ps.ps_scan(lr, sub.n_links, of, ws)
                ps.ps_emit(sub, plan.params, of, px[2 * r0:], py[2 * r0:], pv[2 * r0:], 2 * (r1 - r0), ws)

        run_per_path()
        torch.cuda.synchronize()
        steps_pp = 2
        t1 = time.perf_counter()
        for _ in range(steps_pp):
            run_per_path()
        torch.cuda.synchronize()
        pp_ms = 1e3 * (time.perf_counter() - t1) / steps_pp
        same = bool(torch.equal(px[:V], plan.vx[:V]) and torch.equal(pv[:V], plan.vs[:V]))
        per_path = {"value": V / (pp_ms * 1e-3), "unit": "vertices/s", "ms_per_step": pp_ms,
                    "launches_per_step": 7 * b.n_paths, "identical_output": same}
        log(f"per-path: {pp_ms:.1f} ms/step ({V / (pp_ms * 1e-3) / 1e9:.3f} G vertices/s), "
            f"identical output: {same}")

    cpu = None
    errors = None
    if not args.no_cpu:
        import oracle
        threads = len(os.sched_getaffinity(0))
        log(f"oracle on the host, {threads} threads ...")
        # whole passes over the full workload until ~1.5 s of wall time
        t2 = time.perf_counter()
        passes = 0
        while True:
            ref = oracle.stroke(b, nthreads=threads)
            passes += 1
            if time.perf_counter() - t2 > 1.5:
                break
            del ref
        cpu_s = (time.perf_counter() - t2) / passes
        cpu = {"value": V / cpu_s, "unit": "vertices/s", "cores": threads, "kind": "oracle",
               "sample": f"the full workload ({b.n_paths} paths, {V} vertices), {passes} passes, "
                         f"{cpu_s:.3f} s each (output allocation included)"}
        log(f"oracle: {cpu_s:.2f} s ({V / cpu_s / 1e6:.1f} M vertices/s)")
        # and one pass on a single thread, for the per-core rate
        t3 = time.perf_counter()
        del ref
        ref = oracle.stroke(b, nthreads=1)
        one_s = time.perf_counter() - t3
        cpu["one_thread"] = {"value": V / one_s, "unit": "vertices/s", "s_per_pass": one_s}
        log(f"oracle, 1 thread: {one_s:.2f} s ({V / one_s / 1e6:.1f} M vertices/s)")
        counts_equal = bool(np.array_equal(plan.link_ribs[:db.n_links].cpu().numpy(), ref["link_ribs"]))
        vx = plan.vx[:V].cpu().numpy(); vy = plan.vy[:V].cpu().numpy(); vs = plan.vs[:V].cpu().numpy()
        verr = np.hypot(vx - ref["vx"], vy - ref["vy"])
        serr = np.abs(vs[0::2] - ref["vs"])
        rel = serr / np.maximum(ref["vs"], 1.0)
        errors = {"counts_bit_exact": counts_equal, "max_vertex_err_px": float(verr.max()),
                  "p99999_vertex_err_px": float(np.quantile(verr, 0.99999)),
                  "max_arclen_err_px": float(serr.max()), "max_arclen_rel_err": float(rel.max()),
                  "fixup_ribs": int(st.fixups), "fixup_frac": float(st.fixups) / max(1, R)}
        log(f"errors: {errors}")
        del ref

    c1 = c3 = None
    if not args.no_c1c3:
        # the single-path configurations: latency of one path through the same chain
        log("C1 and C3 ...")
        c1 = c1_leg(torch, ps, W, dev, args.steps, args.warmup)
        c3 = c3_leg(torch, ps, W, dev, args.steps, args.warmup)
        log(f"C1: {c1}")
        log(f"C3: {c3}")

    c5 = None
    if not args.no_c5:
        # the largest configuration: same chain, 2^20 segments, the finest q
        plan.close()
        del db
        torch.cuda.empty_cache()
        log("C5 at q = pi/256 ...")
        c5 = c5_leg(torch, ps, W, dev, 256, args.steps, args.warmup)
        log(f"C5: {c5}")

    result = {
        "metric": "stroke vertices/s & % HBM peak, batched vs per-path, <=2e-3 px vs FP64 oracle",
        "value": vps,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == ps.PS_PREC_FP32 else ("f64" if prec == ps.PS_PREC_FP64 else "f32+f64"),
        "data": "synthetic",
        "fixup_newton_step_tol": float(os.environ.get("PS_FIXUP_TOL", "1e-4")),
        "config": {"workload": "batched: 4096 paths, log-uniform [1,512] segments, 60/25/15% C/Q/K, "
                               "q=pi/64, round joins, butt caps",
                   "paths": b.n_paths, "segments": b.n_segs, "ribs": R, "vertices": V,
                   "precision": args.precision, "emit_mapping": mapping, "emit_K": K,
                   "emit_waves_per_group": waves},
        "gb_per_s": B_alg / (ms_step * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": emit_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": emit_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(f"{mapping},{K},{waves}"),
                     "kernel": "emit (the persistent emit kernel of the plan's graph, between its event nodes; "
                               "its tile table comes from the link scan)",
                     "ms_per_launch": emit_ms, "algorithmic_bytes_per_launch": emit_bytes},
        "per_path": per_path,
        "cpu_baseline": cpu,
        "errors": errors,
        "c1": c1,
        "c3": c3,
        "c5": c5,
    }
    plan.close()
    print(json.dumps(result), flush=True)
    return 0


def _time_plan(torch, plan, steps, warmup):
    for _ in range(warmup):
        plan.launch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        plan.launch()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t) / steps


def matching_ribs(lr_a, off_a, lr_b, off_b):
    """Rib indices (into a and into b) of the links whose rib counts agree, in
    link order; and the mask of links that agree."""
    same = lr_a == lr_b
    n = lr_a[same].astype(np.int64)
    first_a = off_a[:-1][same]
    first_b = off_b[:-1][same]
    rep = np.repeat(np.arange(n.size), n)
    within = np.arange(int(n.sum()), dtype=np.int64) - np.repeat(np.cumsum(n) - n, n)
    return first_a[rep] + within, first_b[rep] + within, same


def study_precision(args, torch, ps, W, dev):
    """The three precision modes against the FP64 oracle on the full
    near-degenerate configuration (C4): link count mismatches; on the links
    whose counts agree, the largest vertex distance; on the paths whose links
    all agree, the largest arc-length difference; ribs re-solved in FP64.  Then
    each mode's step and emit time on the benchmark batch (C2)."""
    import oracle
    b = W.config4()
    db = ps.DeviceBatch(b, device=dev)
    threads = len(os.sched_getaffinity(0))
    ref = oracle.stroke(b, nthreads=threads)
    lr_o, off_o = ref["link_ribs"], ref["offsets"]
    P = b.n_paths
    path_of_link = np.repeat(np.arange(P), 2 * np.diff(b.seg_begin.astype(np.int64)) + 1)
    rows = {}
    modes = (("fp64", ps.PS_PREC_FP64), ("fp32_fixup", ps.PS_PREC_FP32_FIXUP), ("fp32", ps.PS_PREC_FP32))
    for name, prec in modes:
        out = ps.stroke(db, b.q, precision=prec)
        lr = out["link_ribs"].cpu().numpy()
        off = out["offsets"].cpu().numpy()
        ia, ib, same = matching_ribs(lr, off, lr_o, off_o)
        vx, vy, vs = (out[k].cpu().numpy() for k in ("vx", "vy", "vs"))
        # vertex 2r and 2r+1 belong to rib r
        va = np.concatenate([2 * ia, 2 * ia + 1]); vb = np.concatenate([2 * ib, 2 * ib + 1])
        verr = np.hypot(vx[va] - ref["vx"][vb], vy[va] - ref["vy"][vb])
        bad_path = np.zeros(P, bool)
        bad_path[path_of_link[~same]] = True
        rib_path_a = np.repeat(path_of_link, lr.astype(np.int64))
        ok = ~bad_path[rib_path_a[ia]]
        serr = np.abs(vs[2 * ia[ok]] - ref["vs"][ib[ok]])
        rows[name] = {"count_mismatches": int((~same).sum()), "links": int(same.size),
                      "paths_with_a_mismatch": int(bad_path.sum()),
                      "max_vertex_err_px": float(verr.max()) if verr.size else 0.0,
                      "p999_vertex_err_px": float(np.quantile(verr, 0.999)) if verr.size else 0.0,
                      "max_arclen_err_px": float(serr.max()) if serr.size else 0.0,
                      "fixup_ribs": int(out["status"].fixups), "ribs": int(out["total_ribs"])}
        log(f"C4 {name}: {rows[name]}")
        del out
    del db
    # speed of each mode on the benchmark batch
    b2 = W.config2_fast()
    db2 = ps.DeviceBatch(b2, device=dev)
    stream = torch.cuda.current_stream()
    for name, prec in modes:
        first = ps.stroke(db2, b2.q, precision=prec)
        R = first["total_ribs"]
        del first
        plan = ps.Plan(db2, b2.q, vertex_capacity=2 * R, precision=prec, emit=(ps.PS_MAP_TILES, 7, 4))
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        for a, c in ev:
            a.record(stream); c.record(stream)
        for _ in range(args.warmup):
            plan.launch()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a, c in ev:
            plan.launch_timed(a, c)
        torch.cuda.synchronize()
        rows[name]["c2_ms_per_step"] = 1e3 * (time.perf_counter() - t) / args.steps
        rows[name]["c2_emit_ms"] = sum(a.elapsed_time(c) for a, c in ev) / args.steps
        rows[name]["c2_ribs"] = R
        plan.close()
        log(f"C2 {name}: step {rows[name]['c2_ms_per_step']:.3f} ms, emit {rows[name]['c2_emit_ms']:.3f} ms")
    print(json.dumps({"study": "precision", "workload": b.name, "segments": b.n_segs,
                      "reference": "the FP64 oracle", "meta": b.meta,
                      "timing": "C2 batch, tiles mapping K=7, 4 waves per group", "modes": rows}), flush=True)
    return 0


def c3_leg(torch, ps, W, dev, steps: int, warmup: int) -> dict:
    """One 5,000-cubic random-walk path: stroke with arc length, then dashing."""
    b = W.config3()
    db = ps.DeviceBatch(b, device=dev)
    first = ps.stroke(db, b.q)
    R = first["total_ribs"]
    del first
    rcap, dcap = 4 * R, R
    plan = ps.Plan(db, b.q, vertex_capacity=2 * R, dash=b.dash, dash_phase=b.dash_phase,
                   dash_rib_capacity=rcap, dash_capacity=dcap)
    ms = _time_plan(torch, plan, steps, warmup)
    st = plan.status()
    assert st.flags == 0, f"status flags {st.flags}"
    plain = ps.Plan(db, b.q, vertex_capacity=2 * R)
    ms_plain = _time_plan(torch, plain, steps, warmup)
    res = {"workload": "C3: 1 path x 5000 C1 cubics (random walk), width 2, q=pi/128, dash [10, 5]",
           "ribs": R, "vertices": 2 * R,
           "ms_stroke": ms_plain, "ms_stroke_and_dash": ms, "ms_dash": ms - ms_plain,
           "dash_ribs": int(st.dash_ribs), "dashes": int(st.dash_count),
           "path_length_px": float(plan.vs[2 * R - 1].item()),
           "dash_bytes": 12 * 2 * int(st.dash_ribs) + 12 * 2 * R}
    plan.close()
    plain.close()
    return res


def study_c3(args, torch, ps, W, dev):
    res = dict(study="c3", **c3_leg(torch, ps, W, dev, args.steps, args.warmup))
    log(str(res))
    print(json.dumps(res), flush=True)
    return 0


def c5_leg(torch, ps, W, dev, qn: int, steps: int, warmup: int, fixed=(1, 8, 4)) -> dict:
    """C5 at q = pi/qn: 2^20 segments over 65,536 Zipf(1.2) paths.  The whole
    step through an autotuned plan (wall clock over `steps` replays) and its
    emit from the graph's own events, then the emit call alone with the
    autotuned and with a fixed mapping."""
    q = math.pi / qn
    b = W.config5(q=q)
    db = ps.DeviceBatch(b, device=dev)
    first = ps.stroke(db, q)
    R = first["total_ribs"]
    del first
    V = 2 * R
    plan = ps.Plan(db, q, vertex_capacity=V)
    cfg = plan.config()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, c in ev:
        a.record(stream); c.record(stream)
    for _ in range(warmup):
        plan.launch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for a, c in ev:
        plan.launch_timed(a, c)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / steps
    st = plan.status()
    assert st.flags == 0 and st.total_ribs == R, f"C5 status flags {st.flags}"
    emit_ms = sum(a.elapsed_time(c) for a, c in ev) / steps
    B = algorithmic_bytes(V, b.n_segs, b.n_paths)
    # the emit call alone: the autotuned mapping vs a fixed one
    call_ms = {}
    for name, emit in (("autotuned", cfg), ("fixed", fixed)):
        pp = ps.make_params(q, emit=emit)
        for _ in range(2):
            ps.ps_emit(db, pp, plan.offsets, plan.vx, plan.vy, plan.vs, V, plan.ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            ps.ps_emit(db, pp, plan.offsets, plan.vx, plan.vy, plan.vs, V, plan.ws)
        e1.record(stream)
        torch.cuda.synchronize()
        call_ms[name] = e0.elapsed_time(e1) / steps
    plan.close()
    del db
    torch.cuda.empty_cache()
    return {"workload": b.name, "q": f"pi/{qn}", "segments": b.n_segs, "paths": b.n_paths,
            "ribs": R, "vertices": V, "ms_per_step": ms, "vertices_per_s": V / (ms * 1e-3),
            "gb_per_s": B / (ms * 1e-3) / 1e9, "emit_ms": emit_ms,
            "emit_frac": B / (emit_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "autotuned": {"mapping": cfg[0], "K": cfg[1], "waves": cfg[2]},
            "emit_call_ms_autotuned": call_ms["autotuned"],
            "fixed": {"mapping": fixed[0], "K": fixed[1], "waves": fixed[2]},
            "emit_call_ms_fixed": call_ms["fixed"]}


def study_c5(args, torch, ps, W, dev):
    """2^20 segments over 65,536 Zipf(1.2) paths at three q; autotuned vs fixed mapping."""
    rows = []
    for qn in (16, 64, 256):
        row = c5_leg(torch, ps, W, dev, qn, args.steps, args.warmup)
        rows.append(row)
        log(str(row))
    print(json.dumps({"study": "c5", "rows": rows}), flush=True)
    return 0


def study_emit(args, torch, ps, W, dev):
    """The emit stage of the benchmark batch by output mode and mapping: vertices
    and arc length (ps_emit), vertices only (ps_emit without vs), arc length only
    (ps_arclen), for every mapping."""
    b = W.config2_fast()
    db = ps.DeviceBatch(b, device=dev)
    first = ps.stroke(db, b.q)
    R = first["total_ribs"]
    del first
    plan = ps.Plan(db, b.q, vertex_capacity=2 * R)
    stream = torch.cuda.current_stream()

    def timed(fn, reps=10 if not args.emit_config else 40):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    cap, ws = 2 * R, plan.ws
    rows = []
    configs = [(m, K, w_) for m in (ps.PS_MAP_TILES, ps.PS_MAP_LINKS) for K in (4, 6, 7, 8, 16)
               for w_ in (1, 2, 4)]
    if args.emit_config:   # one mapping only
        configs = [tuple(int(x) for x in args.emit_config.split(","))]
    for emit in configs:
        P = ps.make_params(b.q, emit=emit)
        try:
            row = {"mapping": emit[0], "K": emit[1], "waves": emit[2],
                   "ms_xy_s": timed(lambda: ps.ps_emit(db, P, plan.offsets, plan.vx, plan.vy, plan.vs, cap, ws)),
                   "ms_xy": timed(lambda: ps.ps_emit(db, P, plan.offsets, plan.vx, plan.vy, None, cap, ws)),
                   "ms_s": timed(lambda: ps.ps_arclen(db, P, plan.offsets, plan.vs, cap, ws))}
        except ps.PsError:
            continue   # a mapping this build does not offer
        rows.append(row)
        log(str(row))
    plan.close()
    print(json.dumps({"study": "emit", "ribs": R, "rows": rows}), flush=True)
    return 0


def study_mappings(args, torch, ps, W, dev):
    """Every emit mapping (tiles and links) x K x wavefronts per group on each
    configuration: C1, C3, C2 and C5 at q = pi/16, pi/64, pi/256; ms per
    unplanned ps_emit with arc length, the best of each mapping, and what a
    plan picks."""
    configs = [(m, K, w_) for m in (ps.PS_MAP_TILES, ps.PS_MAP_LINKS) for K in (4, 6, 7, 8, 16)
               for w_ in (1, 2, 4)]
    cases = [("C1", W.config1), ("C3", W.config3), ("C2", W.config2_fast)] + \
            [(f"C5 q=pi/{qn}", (lambda qn=qn: W.config5(q=math.pi / qn))) for qn in (16, 64, 256)]
    stream = torch.cuda.current_stream()
    out = []
    for name, make in cases:
        b = make()
        db = ps.DeviceBatch(b, device=dev)
        first = ps.stroke(db, b.q)
        R = first["total_ribs"]
        del first
        plan = ps.Plan(db, b.q, vertex_capacity=2 * R)
        picked = plan.config()
        reps = 20 if R < 10_000_000 else 5
        times = {}
        for emit in configs:
            P = ps.make_params(b.q, emit=emit)
            for _ in range(2):
                ps.ps_emit(db, P, plan.offsets, plan.vx, plan.vy, plan.vs, 2 * R, plan.ws)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                ps.ps_emit(db, P, plan.offsets, plan.vx, plan.vy, plan.vs, 2 * R, plan.ws)
            e1.record(stream)
            torch.cuda.synchronize()
            times[emit] = e0.elapsed_time(e1) / reps
        plan.close()
        best = {}
        for m, label in ((ps.PS_MAP_TILES, "tiles"), (ps.PS_MAP_LINKS, "links")):
            c = min((k for k in times if k[0] == m), key=lambda k: times[k])
            best[label] = {"K": c[1], "waves": c[2], "ms": times[c]}
        row = {"workload": name, "ribs": R, "plan_picks": {"mapping": picked[0], "K": picked[1], "waves": picked[2]},
               "plan_pick_ms": times.get(tuple(picked)), "best": best,
               "all_ms": {f"{k[0]},{k[1]},{k[2]}": round(v, 4) for k, v in times.items()}}
        out.append(row)
        log(f"{name}: ribs {R}, plan picks {picked}, best {best}")
        del db
        torch.cuda.empty_cache()
    print(json.dumps({"study": "mappings", "rows": out}), flush=True)
    return 0


def c1_leg(torch, ps, W, dev, steps: int, warmup: int) -> dict:
    """C1, one path of 64 cubics: latency of the whole chain per path (one plan
    replay, and the three unplanned calls) and its vertices/s."""
    b = W.config1()
    db = ps.DeviceBatch(b, device=dev)
    first = ps.stroke(db, b.q)
    R = first["total_ribs"]
    del first
    plan = ps.Plan(db, b.q, vertex_capacity=2 * R)
    ms = _time_plan(torch, plan, max(steps, 50), warmup)
    lr = torch.empty(db.n_links, dtype=torch.int32, device=dev)
    of = torch.empty(db.n_links + 1, dtype=torch.int64, device=dev)

    def calls():
        ps.ps_count(db, plan.params, lr, plan.ws)
        ps.ps_scan(lr, db.n_links, of, plan.ws)
        ps.ps_emit(db, plan.params, of, plan.vx, plan.vy, plan.vs, 2 * R, plan.ws)

    for _ in range(5):
        calls()
    torch.cuda.synchronize()
    n = max(steps, 50)
    t0 = time.perf_counter()
    for _ in range(n):
        calls()
    torch.cuda.synchronize()
    ms_calls = 1e3 * (time.perf_counter() - t0) / n
    st = plan.status()
    assert st.flags == 0, f"status flags {st.flags}"
    plan.close()
    return {"workload": "C1: 1 path x 64 cubics, q=pi/90, round joins", "ribs": R,
            "us_per_path_plan": 1e3 * ms, "us_per_path_calls": 1e3 * ms_calls,
            "vertices_per_s_plan": 2 * R / (ms * 1e-3)}


def study_c1(args, torch, ps, W, dev):
    row = dict(study="c1", **c1_leg(torch, ps, W, dev, args.steps, args.warmup))
    log(str(row))
    print(json.dumps(row), flush=True)
    return 0


def study_facets(args, torch, ps, W, dev):
    """Polar stroking vs the uniform parametric baseline at the same quad budget
    (Sec. "Versus Uniform Parametric Tessellation"): ordinary facet angles on
    synthetic cubic serpentines and loops (w = 100, q = 4 deg, as the paper's
    serpentine figure) and on exact cusps, and the time of both emits."""
    rng = np.random.default_rng(2026)

    def batch(n, cusp):
        segs = []
        for _ in range(n):
            P0 = rng.uniform(0, 512, 2); P3 = P0 + rng.uniform(-300, 300, 2)
            P1 = P0 + rng.uniform(-200, 200, 2)
            P2 = (P0 + P1 - P3) if cusp else P3 + rng.uniform(-200, 200, 2)
            segs.append([(W.KIND_C, [tuple(np.round(P * 256) / 256) for P in (P0, P1, P2, P3)], 1.0)])
        return W.paths(segs, widths=[100.0] * n, q=math.radians(4.0))

    rows = []
    for name, b in (("serpentines and loops", batch(4096, False)), ("exact cusps", batch(4096, True))):
        db = ps.DeviceBatch(b, device=dev)
        out = ps.stroke(db, b.q)
        R = out["total_ribs"]
        vxu, vyu = torch.empty_like(out["vx"]), torch.empty_like(out["vy"])
        stats = torch.zeros(4, dtype=torch.float64, device=dev)
        row = {"segments": name, "n": b.n_segs, "quads": R - b.n_paths}   # one segment, butt caps per path
        for mode in ("polar", "uniform"):
            if mode == "uniform":
                ps.ps_emit_uniform(db, out["params"], out["offsets"], vxu, vyu, out["capacity"], out["ws"])
                vx, vy = vxu, vyu
            else:
                vx, vy = out["vx"], out["vy"]
            ps.ps_facet_stats(db, out["offsets"], vx, vy, stats)
            torch.cuda.synchronize()
            n, mx, s1, s2 = (float(x) for x in stats.cpu().numpy())
            mean = s1 / n
            row[mode] = {"count": int(n), "max_deg": math.degrees(mx), "mean_deg": math.degrees(mean),
                         "sd_deg": math.degrees(math.sqrt(max(0.0, s2 / n - mean * mean)))}
        rows.append(row)
        log(str(row))
    print(json.dumps({"study": "facets", "rows": rows}), flush=True)
    return 0


def study_coverage(args, torch, ps, W, dev):
    """Coverage of the 4096-path batch's quad strip on a 4096 x 4096 canvas
    (one sample per pixel centre), quads as quads (winding number, bow-ties as
    two lobes) and as the triangle pairs a triangle rasterizer draws: time per
    pass, covered samples, and the algorithmic work -- the summed area of the
    quads in px^2, about one winding test per covered (quad, sample) pair."""
    b = W.config2()
    db = ps.DeviceBatch(b, device=dev)
    out = ps.stroke(db, b.q)
    R = out["total_ribs"]
    vx, vy, off = out["vx"][:2 * R], out["vy"][:2 * R], out["offsets"]
    # area of the quads between ribs of one link (bridges between links are
    # zero-area), by the shoelace formula on the N_r P_r P_{r+1} N_{r+1} loop
    link = torch.searchsorted(off, torch.arange(R, device=dev), right=True) - 1
    same = link[:-1] == link[1:]
    ax, ay, bx, by = vx[0::2].double(), vy[0::2].double(), vx[1::2].double(), vy[1::2].double()
    sh = (ax[:-1] * by[:-1] - bx[:-1] * ay[:-1]) + (bx[:-1] * by[1:] - bx[1:] * by[:-1]) \
        + (bx[1:] * ay[1:] - ax[1:] * by[1:]) + (ax[1:] * ay[:-1] - ax[:-1] * ay[1:])
    area = float((0.5 * sh.abs() * same).sum())
    del link, same, ax, ay, bx, by, sh
    top = torch.empty((4096, 4096), dtype=torch.int32, device=dev)
    rows = []
    covered = {}
    for mode, name in ((ps.PS_COVER_QUAD, "quads"), (ps.PS_COVER_TRIANGLES, "triangles")):
        for _ in range(2):
            ps.ps_coverage(db, off, vx, vy, R, top, 0.0, 0.0, mode)
        torch.cuda.synchronize()
        reps = max(3, args.steps // 4)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ps.ps_coverage(db, off, vx, vy, R, top, 0.0, 0.0, mode)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        covered[name] = top >= 0
        # 4 edges x 7 FP64 operations per winding test (3 edges twice for triangles)
        ops = area * (28 if mode == ps.PS_COVER_QUAD else 42)
        row = {"mode": name, "ms": ms, "covered_samples": int(covered[name].sum()),
               "quad_area_px2": area, "samples_per_s": area / (ms * 1e-3),
               "roofline": {"bound": "alu", "achieved": ops / (ms * 1e-3) / 1e12, "peak": 78.6,
                            "unit": "TFLOP/s (fp64)", "frac": ops / (ms * 1e-3) / 1e12 / 78.6}}
        rows.append(row)
        log(str(row))
    excess = int((covered["triangles"] & ~covered["quads"]).sum())
    print(json.dumps({"study": "coverage", "workload": "4096-path batch, 4096 x 4096 canvas, 1 sample/px",
                      "ribs": R, "rows": rows, "triangle_excess_samples": excess}), flush=True)
    return 0


STUDIES = {"precision": study_precision, "c3": study_c3, "c5": study_c5, "emit": study_emit, "c1": study_c1,
           "mappings": study_mappings,
           "facets": study_facets, "coverage": study_coverage}


if __name__ == "__main__":
    sys.exit(main())

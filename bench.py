#!/usr/bin/env python3
"""Throughput of the binary-fluid LBM hot path on one MI355X.

Workload: the 2048 x 16384 droplet field (seeded discs, radii 8-64, ink area
>= 25 %, flat wetting wall at 120 deg, tau 0.8 ink / 1.0 ambient).  One step
is one collide-stream pass over the whole lattice (a row launch over the
plain rows, a tile launch over the rows next to walls); the droplet
diagnostics (mass, momentum, per-row ink profile and segments) run every 50
steps inside the timed region.  Prints one JSON line:

  value      whole-job MLUPS = nx * ny * steps / timed seconds / 1e6
  roofline   the collide-stream kernels' algorithmic HBM bytes (14 float
             distributions read and written per fluid node, 112 B) over their
             mean time per step (both launches), against the 8 TB/s HBM peak;
             traffic is the counter-measured HBM bytes of one step
  sweep      cases per hour of the 256-case table, batched vs one at a time,
             and the surrogate's gain (measured end to end on 96 queries)
  cpu_baseline  the FP64 oracle on a bounded slab of the same workload

Usage: python bench.py [--gpus 1] [--steps 5000] [--warmup 100]
                       [--no-3d] [--no-sweep] [--no-surrogate] [--no-cpu-baseline]
                       [--extra single_case,sweep_as_written]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = 112  # 9 f + 5 g float32, read once and written once
DIAG_EVERY = 50
KERNEL_SOURCE = os.path.join(ROOT, "paper_1702_04487_amd", "csrc", "lbm_core.hip")

# HBM traffic of one step (both collide-stream launches) on this workload:
# rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, averaged over 34 steps
# and scaled by true bytes / counter reading for the copy_calib program
# (2.000 for FETCH_SIZE, 1.000 for WRITE_SIZE).  The figure holds for the
# kernel source with this SHA-256 only; for any other it is reported as null.
MEASURED_TRAFFIC = {
    "kernel_source_sha256": "eb3fe2a585fb4f9c6cc0bd34b76f59feebbb7c3999fd4b18985d009511efc51a",
    "read_bytes": 1965641077,
    "write_bytes": 1950426020,
}


def measured_traffic():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    if digest != MEASURED_TRAFFIC["kernel_source_sha256"]:
        return None
    return MEASURED_TRAFFIC["read_bytes"] + MEASURED_TRAFFIC["write_bytes"]


def cpu_baseline(cfg, rows: int = 8192, steps: int = 100) -> dict:
    """FP64 oracle on a full-width band of the same disc field (rows
    [0, rows), periodic), timed over `steps` steps after one warm-up step."""
    from oracle import oracle as O
    import workloads as W
    import numpy as np
    p = dict(cfg["params"], ny=rows)
    wall = np.ascontiguousarray(cfg["wall"][:rows])
    d = np.ascontiguousarray(cfg["distance"][:rows])
    sim = O.OracleSim(p, wall)
    sim.init_distance(d)
    sim.step(1)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    nodes = p["nx"] * rows
    sim.close()
    cores = O.max_threads()
    # the same oracle on one thread, over a smaller band
    rows1, steps1 = 512, 10
    O.set_threads(1)
    try:
        p1 = dict(cfg["params"], ny=rows1)
        s1 = O.OracleSim(p1, np.ascontiguousarray(cfg["wall"][:rows1]))
        s1.init_distance(np.ascontiguousarray(cfg["distance"][:rows1]))
        s1.step(1)
        t0 = time.perf_counter()
        s1.step(steps1)
        dt1 = time.perf_counter() - t0
        s1.close()
    finally:
        O.set_threads(cores)
    return {"value": round(nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{p['nx']}x{rows} band (rows 0-{rows - 1}) of the same disc field, periodic, "
                      f"{steps} steps after 1 warm-up, FP64",
            "one_thread": {"value": round(p["nx"] * rows1 * steps1 / dt1 / 1e6, 3), "unit": "MLUPS",
                           "sample": f"{p['nx']}x{rows1} band, {steps1} steps after 1 warm-up"}}


def copy_ceiling_gbs(mib: int = 1792, reps: int = 5):
    """(read+write GB/s, source) of the best plain device copy of one
    distribution buffer of the droplet field (1792 MiB), measured on this
    GPU: boxes of the same part differ by several per cent, so the kernel is
    compared with copies timed beside it.  The library's copy calibration
    program (six copy shapes, run as a child process) when it is built, else
    a torch device copy."""
    import re
    import subprocess
    exe = os.path.join(ROOT, "paper_1702_04487_amd", "bin", "copy_calib")
    if os.path.exists(exe):
        r = subprocess.run([exe, str(mib), str(reps)], capture_output=True, text=True, timeout=300)
        m = re.search(r"best ([0-9.]+) GB/s", r.stdout)
        if r.returncode == 0 and m:
            return float(m.group(1)), "copy_calib: best of six plain copy shapes"
    import torch
    n = (mib << 20) // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9, "torch device copy"


def log(msg: str) -> None:
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def sweep_bench(batched_steps: int = 600, plain_steps: int = 300, plain_every: int = 16, graph: int = 50) -> dict:
    """Cases per hour of the 256-case sweep table (seed 1234, the stable
    variant), 40000 steps per case, diagnostics every 50 steps: every case in
    one batch (autotuned tile shape, graphs of 50 steps) timed over
    `batched_steps` steps, against the same cases run one at a time through
    ij_step, each with its own autotuned tile shape (every `plain_every`-th
    case timed over `plain_steps` steps).  `graph` 0 launches the batch's
    kernels one by one instead of replaying captured graphs (same kernels, for
    per-dispatch counter collection)."""
    import torch
    import workloads as W
    from paper_1702_04487_amd import lbm
    cases = W.sweep_cases(256, seed=1234, stable=True)
    steps_case = cases[0]["steps"]
    nodes = sum(c["params"]["nx"] * c["params"]["ny"] for c in cases)
    stream = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    log(f"sweep: batch of {len(cases)} cases, {nodes / 1e6:.1f} M nodes")
    b = lbm.Batch([c["params"] for c in cases])
    for sim in b.cases:
        sim.init_default()
    w, r, mixed, persistent, tune_ms = b.autotune(10)
    log(f"sweep: autotuned tile {w} waves x {r} rows, mixed strips {mixed}, persistent {persistent} "
        f"({tune_ms:.3f} ms per step)")
    if graph:
        b.set_graph(graph)
    b.step(100)
    ms_b = timed(lambda: b.step(batched_steps)) / batched_steps
    unstable = sum(1 for c in b.cases if c.check() != lbm.IJ_OK)
    b.close()
    del b
    log(f"sweep: batched {ms_b:.3f} ms per step, {unstable} cases flagged unstable")

    per_case = []
    for c in cases[::plain_every]:
        sim = lbm.Sim(c["params"])
        sim.init_default()
        sim.autotune(10)   # each case with its own best tile shape
        sim.step(50)
        per_case.append(timed(lambda: sim.step(plain_steps)) / plain_steps)
        sim.close()
    ms_p = float(np.mean(per_case))
    log(f"sweep: plain {ms_p:.4f} ms per case-step over {len(per_case)} sampled cases")
    batched_cph = len(cases) * 3600.0 / (ms_b * 1e-3 * steps_case)
    plain_cph = 3600.0 / (ms_p * 1e-3 * steps_case)
    return {"table": "256 nozzle cases, seed 1234, stable variant (Gamma*sigma <= 0.01, pulse scaled to a "
                     "0.2 viscous speed bound), 40000 steps each, diagnostics every 50",
            "nodes": nodes, "steps_per_case": steps_case,
            "plain_cases_per_hour": round(plain_cph, 1),
            "batched_cases_per_hour": round(batched_cph, 1),
            "batched_over_plain": round(batched_cph / plain_cph, 2),
            "batched_ms_per_step": round(ms_b, 4), "batched_mlups": round(nodes / (ms_b * 1e-3) / 1e6, 1),
            "plain_ms_per_case_step": round(ms_p, 5),
            "tile": [w, r], "mixed_strips": mixed, "persistent": persistent, "graph_steps": 50, "unstable_cases": unstable,
            "timed": {"batched_steps": batched_steps, "plain_cases": len(per_case), "plain_steps": plain_steps}}


def surrogate_bench(queries: int = 100000, held: int = 256, e2e_queries: int = 96) -> dict:
    """The sweep surrogate on the stored solver cases: train the 4-member
    ensemble (the library's kernels), calibrate its trust threshold on a 10 %
    split, score it on `held` held-out cases (the breakup / no-breakup call
    over the answered cases, breakup-time and drop-velocity errors over the
    answered cases that break up), then answer `queries` new query points
    with the network where it is trusted.  Measured end to end on
    `e2e_queries` further query points: the prediction plus a batched solver
    run of the full horizon for every point the network leaves to it.  The
    solver alone is costed per case from a timed batched run."""
    import torch
    from paper_1702_04487_amd import surrogate as S
    x, y, horizon, _ = S.load_dataset()
    xt, yt, xh, yh = x[:-held], y[:-held], x[-held:], y[-held:]
    ncal = len(xt) // 10
    sur = S.Surrogate(4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.fit(xt[:-ncal], yt[:-ncal], steps=3000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pc, sc = sur.predict(xt[-ncal:])
    thr = S.calibrate(sc, S.scores(pc, yt[-ncal:], horizon))
    ph, sh = sur.predict(xh)
    rep = S.summary(S.scores(ph, yh, horizon), sh <= thr)
    xq = S.sample_inputs(queries, 4242)
    sur.predict(xq)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sq = sur.predict(xq)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t0
    aq = float(np.mean(sq <= thr))
    log(f"surrogate: trained in {t_train:.2f} s; answers {aq:.3f} of {queries} queries in {t_pred * 1e3:.2f} ms")
    t_case = S.solver_seconds_per_case(xh, horizon)
    solver_cph = 3600.0 / t_case
    # end to end: predict, then the solver on what the network leaves
    xe = S.sample_inputs(e2e_queries, 4343)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, se = sur.predict(xe)
    fall = se > thr
    if fall.any():
        S.run_lbm(xe[fall], horizon, progress=False)
    torch.cuda.synchronize()
    t_e2e = time.perf_counter() - t0
    e2e_cph = e2e_queries * 3600.0 / t_e2e
    log(f"surrogate: end to end {e2e_queries} queries, {int(fall.sum())} to the solver, {t_e2e:.1f} s")
    modelled_cph = queries * 3600.0 / (t_pred + (1.0 - aq) * queries * t_case)
    return {"cases": "256 x 2048 nozzle (w 32, L 256), 7 sweep inputs, periodic pulse, stable variant, "
                     f"{horizon} steps; {len(x)} stored solver cases ({len(xt) - ncal} train, {ncal} calibrate, "
                     f"{held} held out)",
            "members": 4, "train_seconds": round(t_train, 3), "threshold": thr,
            "held_out": rep,
            "queries": queries, "answered_fraction": round(aq, 4), "predict_ms": round(t_pred * 1e3, 3),
            "solver_seconds_per_case": round(t_case, 4),
            "batched_cases_per_hour": round(solver_cph, 1),
            "end_to_end": {"queries": e2e_queries, "to_solver": int(fall.sum()), "seconds": round(t_e2e, 3),
                           "cases_per_hour": round(e2e_cph, 1), "gain": round(e2e_cph / solver_cph, 3)},
            "modelled_cases_per_hour_1e5": round(modelled_cph, 1),
            "modelled_gain_1e5": round(modelled_cph / solver_cph, 3)}


BYTES_PER_NODE_3D = 208   # 19 + 7 float populations read and written per fluid node
KERNEL_SOURCE_3D = os.path.join(ROOT, "paper_1702_04487_amd", "csrc", "lbm3d.hip")
# HBM bytes of one step of the 256 x 512 x 256 round nozzle (k3_ghost_g,
# k3_collide, k3_open), from rocprofv3 FETCH_SIZE (x 2.000) and WRITE_SIZE
# (x 1.000) runs of this script, scaled as for the two-dimensional kernel;
# valid for the kernel source with this SHA-256 only.
MEASURED_TRAFFIC_3D = {
    "kernel_source_sha256": "218f8aad7ddc990c5a7f72aaefeab266449f982156cef655cff716fcc5dd9654",
    "read_bytes": 3768243413,
    "write_bytes": 3082571333,
}


def measured_traffic_3d():
    import hashlib
    with open(KERNEL_SOURCE_3D, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    if digest != MEASURED_TRAFFIC_3D["kernel_source_sha256"]:
        return None
    return MEASURED_TRAFFIC_3D["read_bytes"] + MEASURED_TRAFFIC_3D["write_bytes"]


def round_nozzle_3d_bench(steps: int = 300, warmup: int = 20, oracle: bool = True) -> dict:
    """The three-dimensional lattice (D3Q19 f, D3Q7 g): a 256 x 512 x 256
    round nozzle, one step = phi, ghosts, the collide-and-push launch and the
    open rows."""
    import torch
    import workloads as W
    from paper_1702_04487_amd import lbm3d
    c = W.config_round_nozzle()
    p, wall = c["params"], c["wall"]
    fluid = int((wall == 0).sum())
    g = lbm3d.Sim3D(p, wall)
    g.init_distance(c["distance"])
    log(f"3-D round nozzle {p['nx']}x{p['ny']}x{p['nz']}: {warmup} warm-up steps, then {steps} timed")
    g.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s = g.sample(c["row0"])
    g.close()
    achieved = BYTES_PER_NODE_3D * fluid / (ms * 1e-3) / 1e9
    traffic = measured_traffic_3d()
    out = {"workload": f"round nozzle {p['nx']}x{p['ny']}x{p['nz']} (bore radius {c['nozzle'][0]:g}, "
                       f"length {c['nozzle'][1]}, contact angles 60/120, pulse)",
           "fluid_nodes": fluid, "steps": steps, "ms_per_step": round(ms, 5),
           "mlups": round(fluid / (ms * 1e-3) / 1e6, 1),
           "algorithmic_gbs": round(achieved, 1), "frac_of_8tbs": round(achieved / HBM_PEAK_GBS, 4),
           "bytes_per_node": BYTES_PER_NODE_3D, "nan_count": s["nan_count"], "max_u": s["max_u"],
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "traffic_gbs": None if traffic is None else round(traffic / (ms * 1e-3) / 1e9, 1),
                        "scope": "one whole step (k3_ghost_g, k3_collide, k3_open)"}}
    if oracle:
        from oracle import oracle3d as O3
        n3 = 64
        band = dict(p, nx=n3, nz=n3, ny=64)
        wb = W.round_nozzle_wall3d(n3, 64, n3, 16.0, 32)
        o = O3.Oracle3D(band, wb)
        o.init_distance(W.meniscus_distance3d(n3, 64, n3, 32))
        o.step(1)
        t0 = time.perf_counter()
        o.step(5)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"mlups": round(int((wb == 0).sum()) * 5 / dt / 1e6, 3),
                             "sample": "64x64x64 round nozzle (bore radius 16), 5 FP64 steps after 1 warm-up",
                             "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}
    return out


def single_case_bench() -> dict:
    """The 256 x 2048 single nozzle case (contact angle 60 deg, tau 0.8 / 1.0,
    pulse +2e-4 x 2000, -1e-4 x 1000, idle to 60000 steps): as written, and
    with both amplitudes scaled so that the viscous centreline speed of the
    channel, F w^2 / (8 n0 nu_ink), is 0.35 down to 0.1.  Breakup step, drop
    velocity and volume (diagnostics every 50 steps), or the step at which
    the stability guard stopped the run."""
    import workloads as W
    from paper_1702_04487_amd import lbm
    c = W.config_nozzle_single()
    p0 = dict(c["params"], diag_row0=c["row0"], diag_every=50)
    w = c["nozzle"][1]
    bound = max(p0["f_pos"], p0["f_neg"]) * w * w / (8.0 * 0.55 * (0.8 - 0.5) / 3.0)
    out = {"workload": "256x2048 nozzle, w 32, L 256, theta 60, 60000 steps", "speed_bound_as_written": round(bound, 4)}
    for name, cap in (("as_written", None), ("scaled_0.35", 0.35), ("scaled_0.3", 0.3), ("scaled_0.25", 0.25),
                      ("scaled_0.2", 0.2), ("scaled_0.1", 0.1)):
        k = 1.0 if cap is None else cap / bound
        p = dict(p0, f_pos=p0["f_pos"] * k, f_neg=p0["f_neg"] * k)
        sim = lbm.Sim(p, c["wall"])
        sim.init_distance(W.meniscus_distance(p["nx"], p["ny"], c["row0"]))
        t0 = time.perf_counter()
        done = 0
        while done < c["steps"] and sim.check() == lbm.IJ_OK:
            n = min(250, c["steps"] - done)
            sim.step(n)
            done += n
        d = sim.diagnostics()
        secs = time.perf_counter() - t0
        # a breakup read after the guard tripped is not a result
        valid = d["breakup_step"] >= 0 and (d["unstable_step"] < 0 or d["breakup_step"] < d["unstable_step"])
        out[name] = {"f_pos": p["f_pos"], "f_neg": p["f_neg"], "steps": done, "seconds": round(secs, 2),
                     "unstable_step": d["unstable_step"], "breakup_step": d["breakup_step"] if valid else -1,
                     "v_drop": d["v_drop"] if valid and d["v_drop"] == d["v_drop"] else None,
                     "vol_drop": d["vol_drop"] if valid else 0, "satellite": d["satellite"] if valid else 0,
                     "drop_len": d["drop_len"] if valid else 0}
        log(f"single case {name}: {out[name]}")
        sim.close()
    return out


def sweep_as_written_bench(steps: int = 40000) -> dict:
    """The 256-case sweep table as written (no scaling): the whole batch run
    for its 40000 steps; the cases the stability guard stops are then run
    again in their scaled (stable) form as the fallback, and the cases per
    hour count both runs."""
    import torch
    import workloads as W
    from paper_1702_04487_amd import lbm
    raw = W.sweep_cases(256, seed=1234, stable=False)
    stable = W.sweep_cases(256, seed=1234, stable=True)

    def run(cases):
        b = lbm.Batch([c["params"] for c in cases])
        for sim in b.cases:
            sim.init_default()
        b.autotune(10)
        b.set_graph(50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            n = min(10000, steps - done)
            b.step(n)
            done += n
            torch.cuda.synchronize()
            log(f"sweep as written: {len(cases)} cases, step {done} of {steps}")
        secs = time.perf_counter() - t0
        bad = [i for i, s in enumerate(b.cases) if s.check() != lbm.IJ_OK]
        b.close()
        return secs, bad

    t_raw, bad = run(raw)
    t_fb, bad2 = run([stable[i] for i in bad]) if bad else (0.0, [])
    return {"table": "256 nozzle cases, seed 1234, as written, 40000 steps each, diagnostics every 50",
            "seconds": round(t_raw, 2), "unstable": len(bad), "fallback_seconds": round(t_fb, 2),
            "fallback_unstable": len(bad2),
            "cases_per_hour": round(len(raw) * 3600.0 / (t_raw + t_fb), 1),
            "valid_cases_per_hour_without_fallback": round((len(raw) - len(bad)) * 3600.0 / t_raw, 1)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the sweep cases/hour measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the three-dimensional round-nozzle leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg of the sweep")
    ap.add_argument("--sweep-graph", type=int, default=50,
                    help="steps per captured graph of the batched sweep (0: plain launches)")
    ap.add_argument("--extra", default="",
                    help="comma list of legs not run by default: single_case (the 256x2048 case as written and "
                         "scaled), sweep_as_written (the 256-case table unscaled, with fallbacks)")
    ap.add_argument("--kernel-steps", type=int, default=500,
                    help="launches timed back-to-back for the fused kernel's mean duration")
    ap.add_argument("--tiling", default="",
                    help="waves_x,rows_per_block of the fused kernel (default: the library's choice)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the lattice update is measured on a "
              "single MI355X", file=sys.stderr)
        return 2

    import torch
    import workloads as W
    from paper_1702_04487_amd import lbm

    cfg = W.config_droplet_field()
    p = dict(cfg["params"], diag_row0=cfg["row0"], diag_every=DIAG_EVERY)
    nx, ny = p["nx"], p["ny"]
    fluid_nodes = int((cfg["wall"] == 0).sum())
    sim = lbm.Sim(p, cfg["wall"])
    if args.tiling:
        wx, rows = (int(v) for v in args.tiling.split(","))
        sim.set_tiling(wx, rows)
    sim.init_distance(cfg["distance"])
    stream = torch.cuda.current_stream()

    def run(n):
        # a step at t % DIAG_EVERY == 0 also takes the diagnostics sample of
        # its input state (inside the collide kernels)
        sim.step(n)

    log(f"droplet field {nx}x{ny}: {args.warmup} warm-up steps, then {args.steps} timed")
    run(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)

    # mean duration of the fused collide-stream kernel alone: back-to-back
    # launches on the same stream over the steps between two samples (the
    # sampling steps run untimed)
    timed_k, kern_total = 0, 0.0
    torch.cuda.synchronize()
    while timed_k < args.kernel_steps:
        sim.step(1 if sim.t % DIAG_EVERY == 0 else 0)
        n = min(args.kernel_steps - timed_k, DIAG_EVERY - sim.t % DIAG_EVERY)
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        sim.step(n)
        k1.record(stream)
        torch.cuda.synchronize()
        kern_total += k0.elapsed_time(k1)
        timed_k += n
    kern_ms = kern_total / args.kernel_steps

    if sim.check() != lbm.IJ_OK:
        print("bench.py: the run failed the stability guard", file=sys.stderr)
        return 1
    samples = sim.samples()
    mass_drift = abs(samples[-1]["mass_n"] - samples[0]["mass_n"]) / abs(samples[0]["mass_n"])

    copy_gbs, copy_src = copy_ceiling_gbs()
    achieved = BYTES_PER_NODE * fluid_nodes / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    mlups = nx * ny * args.steps / (ms * 1e-3) / 1e6
    out = {
        "metric": "binary-LBM MLUPS + % HBM peak; sweep cases/hour plain vs batched+surrogate",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"droplet field {nx}x{ny} (seeded discs r 8-64, 25% ink, "
                               f"wall 120 deg, periodic)",
                   "nx": nx, "ny": ny, "diag_every": DIAG_EVERY, "tiling": args.tiling or "default"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_collide_rows (plain rows) + k_collide_fused (rows next to walls), one step",
                     "kernel_ms": round(kern_ms, 5), "bytes_per_launch": BYTES_PER_NODE * fluid_nodes,
                     "traffic_gbs": None if traffic is None else round(traffic / (kern_ms * 1e-3) / 1e9, 1),
                     "copy_ceiling_gbs": round(copy_gbs, 1), "copy_ceiling_source": copy_src},
        "mass_drift": mass_drift,
    }
    sim.close()
    del sim
    if not args.no_3d:
        out["round_nozzle_3d"] = round_nozzle_3d_bench(oracle=not args.no_cpu_baseline)
    if not args.no_sweep:
        out["sweep"] = sweep_bench(graph=args.sweep_graph)
        if not args.no_surrogate:
            out["sweep"]["surrogate"] = surrogate_bench()
    extra = [e for e in args.extra.split(",") if e]
    if "single_case" in extra:
        out["single_case"] = single_case_bench()
    if "sweep_as_written" in extra:
        out["sweep_as_written"] = sweep_as_written_bench()
    if not args.no_cpu_baseline:
        log("cpu baseline: the FP64 oracle on a band of the droplet field")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())

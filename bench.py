#!/usr/bin/env python3
"""Benchmark of the SiPO PDHG hot path on one MI355X.

Workload: 3D 256^3 volume (cylindrical vial, rotation axis z), 360 views over
360 degrees, 256 x 256 detector rows per view, Beer-Lambert attenuation with
1/e depth equal to the vial radius, union of 6 random ellipsoids (seed 3000),
band width 10 voxels, isotropic Gaussian blur sigma = 1.5 voxels, Case 1
(in-part normalised dose in [0.9, 1.0]), FP32, restarted PDHG.

A step is one PDHG iteration: blur + project + primal update, backproject +
blur, fused dual update, scalar update, with the KKT / restart check every 64
iterations included.  ``value`` is iterations per second measured over the
timed solve (setup and final KKT evaluation included, so it is a lower bound
on the steady-state rate).  The operator pair P + P^T is also timed on its own
with HIP events on the launch stream, which gives the A + A^T figure and the
roofline entry for the dominant kernel.

Only one GPU is used; --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--angles", type=int, default=360)
    ap.add_argument("--op-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=8, help="z slices in the bounded oracle sample")
    return ap.parse_args()


def cpu_baseline(n, angles, slices):
    """The oracle's PDHG iteration timed on a bounded sample: the same slice
    geometry with ``slices`` z slices instead of n, scaled to the full volume."""
    import numpy as np
    from oracle import lp as olp, pdhg as opdhg, blur as oblur
    from oracle.geometry import make_geometry
    from oracle.projector import Projector
    from sipo_inputs import ellipsoids_target, angles_uniform
    g = make_geometry(n, angles_uniform(angles), nz=slices, atten=1.0)
    P = Projector(g)
    f = ellipsoids_target(n, 3000, nz=n)[n // 2 - slices // 2: n // 2 - slices // 2 + slices]
    prob = olp.build(P, f, olp.CASE1, taps=oblur.psf_taps((1.5, 1.5, 1.5)), band_width=10.0)
    sc = opdhg.diagonal_scaling(prob)
    st = opdhg.initial_state(prob)
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        st = opdhg.step(prob, st, 0.95 * sc.T, 0.95 * sc.Tu, 0.95 * sc.Tv, 0.95 * sc.S_up, 0.95 * sc.S_lo)
    dt = (time.perf_counter() - t0) / reps
    per_full_iter = dt * (n / slices)
    return {"value": 1.0 / per_full_iter, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} oracle PDHG iterations on {slices} of {n} z slices ({n}^2 x {angles} views, "
                      f"blur 1.5, Case 1), scaled by {n}/{slices}; scipy.sparse runs single-threaded"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    import paper_2604_08997_amd as sipo
    from sipo_inputs import ellipsoids_target, angles_uniform

    n, na = args.n, args.angles
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    plan = sipo.Plan(n, list(angles_uniform(na)), nz=n, atten=1.0, sigma=(1.5, 1.5, 1.5), dtype=torch.float32,
                     device=dev)
    f = torch.as_tensor(ellipsoids_target(n, 3000), dtype=torch.float32, device=dev)
    lp = sipo.LP.build(plan, f, sipo.CASE1, band_width=10.0, f_min=1.0)
    print(f"[bench] workload built: {n}^3, {na} views, gel voxels {int((lp.labels == 2).sum())}, "
          f"band voxels {int((lp.labels == 1).sum())}, active rays {int(lp.act.sum())}", file=sys.stderr, flush=True)

    # --- operator pair, timed with events on the launch stream
    vol = torch.rand(plan.vol_shape, device=dev)
    sino = torch.rand(plan.sino_shape, device=dev)
    out_v, out_s = plan.empty_vol(), plan.empty_sino()
    plan.project(vol, out=out_s); plan.backproject(sino, out=out_v); torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(args.op_reps):
        plan.project(vol, out=out_s)
    ev[1].record()
    for _ in range(args.op_reps):
        plan.backproject(sino, out=out_v)
    ev[2].record()
    torch.cuda.synchronize()
    t_p = ev[0].elapsed_time(ev[1]) / args.op_reps
    t_bp = ev[1].elapsed_time(ev[2]) / args.op_reps
    samples = float(n) * n * n * na
    flops = 4.0 * samples                                   # 2 FMA per (voxel, view) sample
    bytes_pair = 2.0 * 4.0 * (plan.n_angles * n * n + n * n * n)   # each operator reads one array and writes the other
    dom_name, dom_t = ("project", t_p) if t_p >= t_bp else ("backproject", t_bp)
    achieved = flops / (dom_t * 1e-3) / 1e12
    print(f"[bench] project {t_p:.3f} ms, backproject {t_bp:.3f} ms", file=sys.stderr, flush=True)

    # --- PDHG iterations
    opts_w = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max(args.warmup, 1), tol=1e-12, check_every=64)
    ws = None
    sipo.solve(lp, opts_w, want_dose=False)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} iterations done", file=sys.stderr, flush=True)
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=args.steps, tol=1e-12, check_every=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sipo.solve(lp, opts, want_dose=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = res["iters"]
    ips = iters / dt
    print(f"[bench] {iters} iterations in {dt:.3f} s; rel KKT p/d/gap {res['rel_primal']:.2e}/"
          f"{res['rel_dual']:.2e}/{res['rel_gap']:.2e}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, na, args.cpu_slices)
        cpu["cores"] = 1
    line = {
        "metric": "PDHG iters/s",
        "value": round(ips, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / max(iters, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D {n}^3 vial, {na} views over 360 deg, {n}x{n} detector, 6 random ellipsoids "
                               f"(seed 3000), band 10, blur sigma 1.5, Case 1 [0.9,1.0], restarted PDHG",
                   "n": n, "views": na, "case": 1, "blur_sigma": 1.5},
        "a_plus_at_gbs": round(bytes_pair / ((t_p + t_bp) * 1e-3) / 1e9, 2),
        "project_ms": round(t_p, 4),
        "backproject_ms": round(t_bp, 4),
        "roofline": {"bound": "alu", "kernel": dom_name, "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

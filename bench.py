#!/usr/bin/env python3
"""Benchmark of the SiPO PDHG hot path on one MI355X.

Workload: 3D 256^3 volume (cylindrical vial, rotation axis z), 360 views over
360 degrees, 256 x 256 detector rows per view, Beer-Lambert attenuation with
1/e depth equal to the vial radius, union of 6 random ellipsoids (seed 3000),
band width 10 voxels, isotropic Gaussian blur sigma = 1.5 voxels, Case 1
(in-part normalised dose in [0.9, 1.0]), FP32, restarted PDHG.

A step is one PDHG iteration: blur + project + primal update, backproject +
blur, fused dual update, scalar update, with the KKT / restart check every 64
iterations included.  ``value`` is the steady iteration rate of one solve of
``--steps`` iterations run as a caller would (iteration blocks captured in a HIP
graph), after a warm-up solve of ``--warmup`` iterations: ``--steps`` divided by
the solver's own loop time, which HIP events on the solve's stream take from the
first iteration launch to the end of the last block and its check.  The one-time
setup of the solve (scalings, layout changes, graph capture, final evaluation)
is reported separately (``setup_ms``), as is the wall time of the whole call.
A second solve of the same length runs in profile mode: the library records HIP
events around every iteration launch, which gives the per-phase times and the
roofline entry of the dominant kernel (the forward projector as the solve runs
it).  The full operators are timed standalone, as the ABI calls run them
(median of 20 launches each): ``a_plus_at_gbs`` is their algorithmic bytes over
their time.  ``time_to_1e-4`` is a cold graph-captured solve of the same LP to
relative KKT 1e-4 (256^3 workload; the solver prints its residuals every 64
checks).

Only one GPU is used; --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(HERE, "profiles", "traffic_project3d_256cube_360.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", choices=["vol256", "vol512"], default="vol256",
                    help="vol256: 256^3 x 360, ellipsoids, blur 1.5, Case 1; "
                         "vol512: 512^3 x 720, lattice, blur (1, 1, 2), Case 2 cap 0.65")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=32, help="z slices in the bounded oracle sample")
    ap.add_argument("--no-ttk", dest="ttk", action="store_false",
                    help="skip the cold solve to relative KKT 1e-4 (time_to_1e-4, about 95 s at 256^3)")
    ap.add_argument("--ttk-iters", type=int, default=200000, help="iteration budget of the time-to-1e-4 solve")
    ap.add_argument("--batch", type=int, default=8,
                    help="instances of the uneven 2D batch (seeds 2000..) for the batched-vs-plain time to 1e-4, "
                         "cold and h_min-screened (0 = skip)")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched-vs-plain comparison")
    ap.add_argument("--screened", action="store_true",
                    help="batched-vs-plain comparison also by the h_min-screened route (Case 2 instances first solve "
                         "their h_min LP)")
    ap.add_argument("--two-stage", type=int, default=0,
                    help="run only the two-stage Case 1 -> Case 2 workflow on this many instances of the uneven "
                         "2D batch, against Case 2 at the fixed cap 0.7 on the same targets")
    ap.add_argument("--margin", type=float, default=0.02,
                    help="relative widening of the stage-1 bound handed to stage 2 (--two-stage)")
    ap.add_argument("--sweep", action="store_true",
                    help="run only the (w1, w2) x band-width sweep of the general LP on the 256^2 x 360 slice, "
                         "batched against one by one")
    ap.add_argument("--probe", choices=["project", "copy"], default=None,
                    help="run only a few launches of one kernel (for hardware counter runs) and exit")
    return ap.parse_args()


def vial_voxels(n):
    """Voxels of an n x n slice whose centre lies in the unit disk (exact integer test)."""
    import numpy as np
    c = 2 * np.arange(n, dtype=np.int64) + 1 - n
    return int(((c[:, None] ** 2 + c[None, :] ** 2) <= n * n).sum())


def source_digest():
    """Digest of the sources that decide the in-solve projector's work (the kernel and the solver's
    skip flags): recorded traffic is valid only for these sources."""
    h = hashlib.sha256()
    for name in ("projector.hip", "pdhg.hip"):
        with open(os.path.join(HERE, "paper_2604_08997_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def lp_work(n, angles, n_bins, labels, act, psf_radius):
    """Algorithmic work of the LP's operators, counted on the host from the geometry.

    P on the LP's active rays: one FMA per nonzero of P in an active row (a voxel
    contributes to bins floor(u) and floor(u) + 1 with weights 1 - f and f, u the
    detector coordinate of its centre).  P^T where the blurred dose is read: one
    FMA per nonzero of P^T in the columns of labelled voxels and their PSF
    neighbourhood (in the vial).  Returns nonzero counts.
    """
    import numpy as np
    from scipy import ndimage
    h = 2.0 / n
    q = 2 * np.arange(n, dtype=np.int64) + 1 - n
    rr, cc = np.nonzero((q[:, None] ** 2 + q[None, :] ** 2) <= n * n)
    x, y = -1.0 + (cc + 0.5) * h, -1.0 + (rr + 0.5) * h
    nz = labels.shape[0]
    act_ab = act.sum(axis=1, dtype=np.int64)                 # [view][bin]: active slices
    per_vox = np.zeros(len(rr), dtype=np.int64)
    nnz_act = nnz_full = 0
    for a, th in enumerate(angles):
        u = (-x * np.sin(th) + y * np.cos(th) + 1.0) * (0.5 * n_bins) - 0.5
        b0 = np.floor(u).astype(np.int64)
        f = u - b0
        m0 = (f < 1.0) & (b0 >= 0) & (b0 < n_bins)
        m1 = (f > 0.0) & (b0 + 1 < n_bins) & (b0 + 1 >= 0)
        cnt = np.bincount(b0[m0], minlength=n_bins) + np.bincount(b0[m1] + 1, minlength=n_bins)
        nnz_full += int(cnt.sum()) * nz
        nnz_act += int((cnt * act_ab[a]).sum())
        per_vox += m0.astype(np.int64) + m1.astype(np.int64)
    rz, ry, rx = psf_radius
    need = ndimage.maximum_filter((labels > 0).astype(np.uint8), size=(2 * rz + 1, 2 * ry + 1, 2 * rx + 1)) > 0
    nnz_bp = int((need[:, rr, cc] * per_vox[None, :]).sum())
    return {"p_nnz_active": nnz_act, "p_nnz_full": nnz_full, "bp_nnz_needed": nnz_bp,
            "active_ray_fraction": round(float(act.mean()), 5), "needed_voxel_fraction": round(float(need.mean()), 5)}


def recorded_traffic(kernel):
    """HBM bytes per launch of the in-solve forward projector from the committed counter runs, or
    None when they are absent, were taken on another version of the sources, or on another kernel
    variant than ``kernel``."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_digest() or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


# Work splits of the masked operators in the benchmark's solves (a result's op_config): the
# solver's tuner, run in the warm-up solve, picks among candidates that differ by a few percent at
# this workload, so the timed, profiled and counter-collection solves fix one choice -- the fastest
# in repeated tuner runs on MI355X: 16 slices per projector thread, 3 queue workgroups per CU, the
# primal step fused, candidate skipping on, two listed march steps per staged chunk; 8 slices and 8
# view splits for the backprojector, 4 slices per blur chunk -- and the line reports the tuner's own
# pick beside it.
BENCH_OPS = {"p_zc": 16, "bp_zc": 8, "bp_splits": 8, "blur_zc": 4, "p_queue": 3, "p_fuse": 1, "p_skip": 1,
             "p_chunk": 2}


def in_solve_projector(tuning, ops):
    """Name of the projector kernel an LP solve of the 256^3 x 360 workload runs (view pairs, 3
    candidates per step, slices per thread, work queue and listed march steps per staged chunk as
    the solve reports them in ``ops``)."""
    zc = ops["p_zc"]
    if tuning["p3d_dma"]:
        queue = "true" if ops.get("p_queue", -1) > 0 else "false"
        skip = "true" if ops.get("p_skip", 1 if tuning["p3d_skip"] else -1) > 0 else "false"
        cm = ops.get("p_chunk", 1) or 1
        return f"project3d_dma_kernel<{zc}, 3, true, {skip}, {cm}, true, {queue}>"
    return f"project3d_kernel<float, {zc}, 3, true>"


def host_cpu():
    """Model name of this host's CPU and its logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(n, angles, slices):
    """The oracle's PDHG iteration timed on a bounded sample: the same slice geometry with
    ``slices`` z slices instead of n.  The projector pair is block-diagonal in z (one detector
    row per slice), so the oracle's work per iteration is linear in the slice count; the
    per-slice rate is reported as measured and the full-volume rate is that rate over n slices."""
    from threadpoolctl import threadpool_limits
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
    reps = 24
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(reps):
            st = opdhg.step(prob, st, 0.95 * sc.T, 0.95 * sc.Tu, 0.95 * sc.Tv, 0.95 * sc.S_up, 0.95 * sc.S_lo)
        total = time.perf_counter() - t0
    dt = total / reps
    model, ncpu = host_cpu()
    slice_iters_per_s = slices / dt          # slice-iterations per second
    return {"value": round(slice_iters_per_s / n, 5), "unit": "iters/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_cores": ncpu, "per_slice_iters_per_s": round(slice_iters_per_s, 4),
            "sample_seconds": round(total, 2),
            "sample": f"{reps} oracle PDHG iterations (FP64 SciPy CSR) on the central {slices} of {n} z slices "
                      f"({n}^2 x {angles} views, blur 1.5, Case 1), one thread (1 of {ncpu} cores of {model}); "
                      f"value = measured slice-iterations per second / {n} slices"}


def batch_vs_plain(count, dev, max_iters=40000, infeas_tol=1e-4, h_min_tol=1e-5, screened=False):
    """Time to relative KKT 1e-4 (or a checked infeasibility certificate) of the first ``count``
    instances of the uneven 2D batch, one batched graph-captured solve against the same solver run
    instance by instance (also graph-captured), on the same GPU, by two routes:

    * cold: every instance as posed (Case 1 [0.9, 1.0] or Case 2 cap 0.7) from zero;
    * screened (``screened``, --screened): the Case-2 instances first solve their h_min LP (the smallest feasible band cap,
      general LP with w = (1, 0)); a Case 2 whose cap lies below it starts from the h_min
      multipliers, which the solver's iteration-0 Farkas test accepts as its certificate.  In the
      batched route the h_min LPs form one batch and all instances the second; one by one, each
      Case 2 runs its h_min LP and then itself.

    The Farkas tolerance equals the KKT tolerance (1e-4, relative to the ray's dual objective)."""
    import torch
    import paper_2604_08997_amd as sipo
    from paper_2604_08997_amd import workflow
    from sipo_inputs import batch_instances, angles_uniform
    from collections import Counter
    insts = batch_instances(count, 2000)
    items, cold = [], []
    for b in insts:
        plan = sipo.Plan(b.n, list(angles_uniform(b.n_angles)), dtype=torch.float32, device=dev)
        f = torch.as_tensor(b.target, dtype=torch.float32, device=dev)
        items.append((plan, f, b.case))
        cold.append(sipo.LP.build(plan, f, b.case, band_width=10.0, f_min=1.0))
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-4, infeas_tol=infeas_tol, use_graph=1)
    h_opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=h_min_tol, use_graph=1)
    stream = torch.cuda.Stream()
    keys = ("status", "iters", "restarts", "primal_obj", "dual_obj", "rel_primal", "rel_dual", "rel_gap", "u", "v")

    def reset(lps):
        for lp in lps:
            lp.y.zero_(); lp.lam_up.zero_(); lp.lam_lo.zero_()
        torch.cuda.synchronize()

    def timed(fn):
        with torch.cuda.stream(stream):
            t0 = time.perf_counter()
            out = fn()
            stream.synchronize()
        return out, time.perf_counter() - t0

    # ---- cold route: the batched solve tunes the 2D pair's work shapes on the batch (its time counts);
    # the instances one by one run those shapes, so both legs do the same arithmetic
    reset(cold)
    t_opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-4, infeas_tol=infeas_tol, use_graph=1,
                               tune_operators=1, progress_every=1 << 30)
    rb, t_batch = timed(lambda: sipo.solve(cold, t_opts, want_dose=False))
    tiles = rb[0]["tiles_2d"]
    print(f"[bench] batch of {count}, cold: batched {t_batch:.2f} s, {dict(Counter(r['status_name'] for r in rb))}, "
          f"2D work shapes {tiles}", file=sys.stderr, flush=True)
    reset(cold)
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-4, infeas_tol=infeas_tol, use_graph=1,
                             tiles_2d=tiles)
    h_opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=h_min_tol, use_graph=1, tiles_2d=tiles)

    def one_by_one():
        out = []
        for k, lp in enumerate(cold):
            out.append(sipo.solve(lp, opts, want_dose=False))
            print(f"[bench] cold one by one: instance {k} {out[-1]['status_name']} after {out[-1]['iters']} iterations",
                  file=sys.stderr, flush=True)
        return out
    rp, t_plain = timed(one_by_one)
    print(f"[bench] batch of {count}, cold: one by one {t_plain:.2f} s", file=sys.stderr, flush=True)
    same = all(all(a[k] == b[k] for k in keys) for a, b in zip(rb, rp))
    capped = [k for k, r in enumerate(rb) if r["status_name"] not in ("optimal", "infeasible")]

    samples = sum(float(b.n) * b.n * b.n_angles for b in insts)
    out = {"instances": count, "seeds": f"2000-{2000 + count - 1}", "samples_per_application": samples,
           "max_iters": max_iters, "infeas_tol": infeas_tol, "compared_fields": list(keys), "tiles_2d": tiles,
           "cold": {"batched_s": round(t_batch, 3), "plain_s": round(t_plain, 3),
                    # a time to 1e-4 only when every instance ended optimal or with a certificate
                    "speedup": round(t_plain / t_batch, 3) if not capped else None,
                    "speedup_with_capped_instances": round(t_plain / t_batch, 3),
                    "status": dict(Counter(r["status_name"] for r in rb)), "capped_instances": capped,
                    "iters": [r["iters"] for r in rb], "per_instance_results_identical": same}}
    if not screened:
        return out

    # ---- screened route (Case 2 in general units: band cap 0.7, f~_T = 1)
    def screened_lps():
        hms, finals = {}, []
        for k, (plan, f, case) in enumerate(items):
            lab, act = cold[k].labels, cold[k].act
            if case == sipo.CASE2:
                hms[k] = workflow.h_min_lp(plan, lab, act, 1.0)
                finals.append(workflow.case2_lp(plan, lab, act, 1.0, 0.7))
            else:
                finals.append(sipo.LP.build(plan, f, case, band_width=10.0, f_min=1.0))
        return hms, finals

    def warm(lp, hm, r):
        if r["status_name"] in ("optimal", "iter_limit") and 0.7 < r["u"]:
            lp.lam_up.copy_(hm.lam_up)
            lp.lam_lo.copy_(hm.lam_lo)

    hms, finals = screened_lps()

    def screened_batched():
        ks = sorted(hms)
        rh = sipo.solve([hms[k] for k in ks], h_opts, want_dose=False) if ks else []
        for k, r in zip(ks, rh):
            warm(finals[k], hms[k], r)
        return sipo.solve(finals, opts, want_dose=False), dict(zip(ks, rh))
    (sb, sbh), ts_batch = timed(screened_batched)
    print(f"[bench] batch of {count}, screened: batched {ts_batch:.2f} s, "
          f"{dict(Counter(r['status_name'] for r in sb))}", file=sys.stderr, flush=True)
    hms, finals = screened_lps()

    def screened_one_by_one():
        out, outh = [], {}
        for k, lp in enumerate(finals):
            if k in hms:
                outh[k] = sipo.solve(hms[k], h_opts, want_dose=False)
                warm(lp, hms[k], outh[k])
            out.append(sipo.solve(lp, opts, want_dose=False))
            print(f"[bench] screened one by one: instance {k} {out[-1]['status_name']} after {out[-1]['iters']} "
                  f"iterations", file=sys.stderr, flush=True)
        return out, outh
    (sp, sph), ts_plain = timed(screened_one_by_one)
    print(f"[bench] batch of {count}, screened: one by one {ts_plain:.2f} s", file=sys.stderr, flush=True)
    s_same = all(all(a[k] == b[k] for k in keys) for a, b in zip(sb, sp)) and \
        all(all(sbh[k][q] == sph[k][q] for q in keys) for k in sbh)
    s_capped = [k for k, r in enumerate(sb) if r["status_name"] not in ("optimal", "infeasible")]
    out["screened"] = {"batched_s": round(ts_batch, 3), "plain_s": round(ts_plain, 3),
                       "speedup": round(ts_plain / ts_batch, 3) if not s_capped else None,
                       "speedup_with_capped_instances": round(ts_plain / ts_batch, 3),
                       "status": dict(Counter(r["status_name"] for r in sb)), "capped_instances": s_capped,
                       "h_min_tol": h_min_tol, "h_min": {str(k): round(r["u"], 6) for k, r in sbh.items()},
                       "certified_at_iteration_0": sum(1 for r in sb if r["status_name"] == "infeasible"
                                                       and r["iters"] == 0),
                       "iters": [r["iters"] for r in sb], "per_instance_results_identical": s_same}
    return out


def two_stage_batch(count, dev, margin, max_iters=20000):
    """Two-stage workflow (Case 1 with h_min, then Case 2 at the transferred bound; each stage one batched,
    graph-captured solve) on the first ``count`` instances of the uneven 2D batch, against the one-stage
    route on the same targets: Case 2 at the fixed cap 0.7, cold and screened by h_min."""
    import torch
    import paper_2604_08997_amd as sipo
    from paper_2604_08997_amd import workflow
    from sipo_inputs import batch_instances, angles_uniform
    from statistics import median
    from collections import Counter
    insts = batch_instances(count, 2000)
    items = []
    for b in insts:
        plan = sipo.Plan(b.n, list(angles_uniform(b.n_angles)), dtype=torch.float32, device=dev)
        items.append((plan, torch.as_tensor(b.target, dtype=torch.float32, device=dev)))
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-4, infeas_tol=1e-5, use_graph=1)
    print(f"[bench] two-stage: {count} instances built", file=sys.stderr, flush=True)
    times = {}
    stream = torch.cuda.Stream()                      # graph capture needs a non-default stream
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        res = workflow.two_stage(items, band_width=10.0, margin=margin, opts=opts, times=times)
        print(f"[bench] two-stage: stage 1 {times['stage1']:.2f} s, stage 2 {times.get('stage2', 0.0):.2f} s",
              file=sys.stderr, flush=True)
        lps = [sipo.LP.build(p, f, sipo.CASE2, band_width=10.0, cap=0.7) for p, f in items]
        t0 = time.perf_counter()
        direct = sipo.solve(lps, opts, want_dose=False)
        t_direct = time.perf_counter() - t0
        print(f"[bench] one-stage Case 2 cap 0.7: {t_direct:.2f} s", file=sys.stderr, flush=True)
        st = {}
        # FP32 multipliers carry reduced-cost errors near 1e-4 of the ray objective: the screened
        # route solves h_min to 1e-5 and accepts rays at a Farkas tolerance of 1e-3
        scr = workflow.case2_screened(
            items, [0.7] * count, band_width=10.0, times=st,
            opts=sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-4, infeas_tol=1e-3, use_graph=1),
            h_min_opts=sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-5, use_graph=1))
        print(f"[bench] screened Case 2 cap 0.7: h_min {st['h_min']:.2f} s, Case 2 {st['case2']:.2f} s",
              file=sys.stderr, flush=True)
    ok = [d for d in res if d["stage2"] is not None and d["stage2"]["status_name"] == "optimal"]
    hm = [d["h_min"] for d in res if d["h_min"] == d["h_min"]]
    return {
        "instances": count, "seeds": f"2000-{2000 + count - 1}", "max_iters": max_iters, "margin": margin,
        "stage1_s": round(times["stage1"], 3), "stage2_s": round(times.get("stage2", 0.0), 3),
        "stage1_status": dict(Counter(d["stage1"]["status_name"] for d in res)),
        "h_min_status": dict(Counter(d["h_min_result"]["status_name"] for d in res)),
        "stage2_status": dict(Counter(d["stage2"]["status_name"] for d in res if d["stage2"] is not None)),
        "stage1_iters_max": max(d["stage1"]["iters"] for d in res),
        "stage2_iters_max": max((d["stage2"]["iters"] for d in res if d["stage2"] is not None), default=0),
        "median_h_min": round(median(hm), 5) if hm else None,
        "median_u1": round(median(d["u1"] for d in ok), 5) if ok else None,
        "median_psr_f_stage1_stage2": [round(median(d["metrics1"]["psr_f"] for d in ok), 5),
                                       round(median(d["metrics2"]["psr_f"] for d in ok), 5)] if ok else None,
        "median_dtvr_stage1_stage2": [round(median(d["metrics1"]["dtvr"] for d in ok), 5),
                                      round(median(d["metrics2"]["dtvr"] for d in ok), 5)] if ok else None,
        "cap_0.7_below_h_min": sum(1 for h in hm if h > 0.7),
        "one_stage_cap_0.7_s": round(t_direct, 3),
        "one_stage_cap_0.7_status": dict(Counter(r["status_name"] for r in direct)),
        "screened_cap_0.7_s": [round(st["h_min"], 3), round(st["case2"], 3)],
        "screened_h_min_status": dict(Counter(d["h_min_result"]["status_name"] for d in scr)),
        "screened_cap_0.7_status": dict(Counter(d["result"]["status_name"] for d in scr)),
        "screened_cap_0.7_started_from_h_min": sum(1 for d in scr if d["screened"]),
        "screened_cap_0.7_certified_at_iteration_0": sum(1 for d in scr if d["result"]["status_name"] == "infeasible"
                                                          and d["result"]["iters"] == 0),
    }


def sweep_slice(dev, max_iters=20000):
    """General LP over 4 weight pairs x 3 band widths (5, 10, band-free) on the 256^2 x 360 slice
    (annulus + disks target, seed 1000): one batched, graph-captured solve against the same 12 solves one by one."""
    import math
    import torch
    import paper_2604_08997_amd as sipo
    from paper_2604_08997_amd import workflow
    from sipo_inputs import annulus_disks_target, angles_uniform
    from collections import Counter
    n, na = 256, 360
    plan = sipo.Plan(n, list(angles_uniform(na)), dtype=torch.float32, device=dev)
    f = torch.as_tensor(annulus_disks_target(n, 1000), dtype=torch.float32, device=dev)
    weights = [(0.25, 1.0), (1.0, 1.0), (4.0, 1.0), (16.0, 1.0)]
    bands = [5.0, 10.0, math.inf]
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max_iters, tol=1e-4, infeas_tol=1e-5, use_graph=1)
    stream = torch.cuda.Stream()                      # graph capture needs a non-default stream
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        out = workflow.sweep(plan, f, weights, bands, opts=opts)
        t_batch = time.perf_counter() - t0
        print(f"[bench] sweep of {len(out)}: batched {t_batch:.2f} s", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        single = []
        for bw in bands:
            for w in weights:
                single.append(workflow.sweep(plan, f, [w], [bw], opts=opts)[0])
                print(f"[bench] sweep one by one: band {bw} w {w} {single[-1]['result']['status_name']}",
                      file=sys.stderr, flush=True)
        t_plain = time.perf_counter() - t0
    same = all(a["result"]["status"] == b["result"]["status"] and a["result"]["iters"] == b["result"]["iters"]
               for a, b in zip(out, single))
    return {"instances": len(out), "grid": "256^2 x 360 views, annulus + disks", "weights": weights,
            "band_widths": ["inf" if math.isinf(b) else b for b in bands], "batched_s": round(t_batch, 3),
            "plain_s": round(t_plain, 3), "speedup": round(t_plain / t_batch, 3),
            "status": dict(Counter(d["result"]["status_name"] for d in out)),
            "per_instance_results_identical": same,
            "points": [{"band": "inf" if math.isinf(d["band_width"]) else d["band_width"], "w1": d["w1"],
                        "u": round(d["result"]["u"], 5), "v": round(d["result"]["v"], 5),
                        "psr_f": round(d["metrics"]["psr_f"], 5), "dtvr": round(d["metrics"]["dtvr"], 5),
                        "iters": d["result"]["iters"]} for d in out]}


def full_operators(plan, dev, work, reps=20):
    """Standalone full operators as the ABI calls run them (every ray and voxel, layout changes
    included): P on x ~ U[0,1) (seed 3002), P^T on y ~ U[0,1) (seed 3001) and K, each the median of
    ``reps`` launches timed with events on the current stream after a warm-up launch.  Algorithmic
    bytes: P reads the volume and writes the sinogram, P^T the reverse, K reads and writes a volume."""
    import statistics
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(3002)
    vol = torch.rand(plan.vol_shape, device=dev, generator=g)
    g.manual_seed(3001)
    sino = torch.rand(plan.sino_shape, device=dev, generator=g)
    vout, sout = plan.empty_vol(), plan.empty_sino()

    def med(fn):
        fn()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return statistics.median(times)
    t_p = med(lambda: plan.project(vol, out=sout))
    t_bp = med(lambda: plan.backproject(sino, out=vout))
    t_k = med(lambda: plan.blur(vol, out=vout)) if plan.sigma is not None else 0.0
    vb, sb = 4.0 * plan.nz * plan.n * plan.n, 4.0 * plan.n_angles * plan.nz * plan.n_bins
    pair = 2.0 * (vb + sb)
    gbs = pair / ((t_p + t_bp) * 1e-3) / 1e9
    gbs_k = (pair + 4.0 * vb) / ((t_p + t_bp + 2.0 * t_k) * 1e-3) / 1e9
    del vol, sino, vout, sout
    return {"p_ms": round(t_p, 4), "pt_ms": round(t_bp, 4), "k_ms": round(t_k, 4),
            "pair_bytes": pair, "a_plus_at_gbs": round(gbs, 2), "a_plus_at_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "pair_with_blur_bytes": pair + 4.0 * vb, "a_plus_at_with_blur_gbs": round(gbs_k, 2),
            "a_plus_at_with_blur_hbm_frac": round(gbs_k / HBM_PEAK_GBS, 4),
            "blur_gbs": round(2.0 * vb / (t_k * 1e-3) / 1e9, 2) if t_k > 0 else None,
            "p_valu_frac": round(2.0 * work["p_nnz_full"] / (t_p * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
            "pt_valu_frac": round(2.0 * work["p_nnz_full"] / (t_bp * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)}


def probe(args, plan, dev):
    """A few launches of one kernel, for hardware-counter runs (rocprofv3 --pmc)."""
    import torch
    if args.probe == "copy":
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)     # 256 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[probe] copy of {a.numel() * 4} bytes x 3", file=sys.stderr, flush=True)
        return 0
    # the projector as the timed solve runs it: a short restarted solve of the benchmark LP (its most
    # frequent projector kernel is the in-solve variant)
    import paper_2604_08997_amd as sipo
    from sipo_inputs import ellipsoids_target
    plan.autotune()
    f = torch.as_tensor(ellipsoids_target(plan.n, 3000), dtype=torch.float32, device=dev)
    lp = sipo.LP.build(plan, f, sipo.CASE1, band_width=10.0, f_min=1.0)
    r = sipo.solve(lp, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=32, tol=1e-12, op_config=BENCH_OPS),
                   want_dose=False)
    torch.cuda.synchronize()
    print(f"[probe] 32-iteration solve after autotune; masked operators {r['op_config']}", file=sys.stderr, flush=True)
    return 0


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only; --gpus must be 1", file=sys.stderr)
        return 2
    import torch
    import paper_2604_08997_amd as sipo
    from sipo_inputs import ellipsoids_target, angles_uniform, lattice_target

    big = args.workload == "vol512"
    n, na = (512, 720) if big else (256, 360)
    sigma = (1.0, 1.0, 2.0) if big else (1.5, 1.5, 1.5)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.batch_only:
        print(json.dumps({"batched_vs_plain_time_to_1e-4": batch_vs_plain(args.batch, dev, screened=args.screened)}),
              flush=True)
        return 0
    if args.two_stage > 0:
        print(json.dumps({"two_stage": two_stage_batch(args.two_stage, dev, args.margin)}), flush=True)
        return 0
    if args.sweep:
        print(json.dumps({"sweep": sweep_slice(dev)}), flush=True)
        return 0
    plan = sipo.Plan(n, list(angles_uniform(na)), nz=n, atten=1.0, sigma=sigma, dtype=torch.float32, device=dev)
    if args.probe:
        return probe(args, plan, dev)
    plan.autotune()
    tuning = plan.tuning()
    print(f"[bench] autotuned work splits: {tuning}", file=sys.stderr, flush=True)
    if big:
        f = torch.as_tensor(lattice_target(n, 4000), dtype=torch.float32, device=dev)
        lp = sipo.LP.build(plan, f, sipo.CASE2, band_width=10.0, f_min=1.0, cap=0.65)
    else:
        f = torch.as_tensor(ellipsoids_target(n, 3000), dtype=torch.float32, device=dev)
        lp = sipo.LP.build(plan, f, sipo.CASE1, band_width=10.0, f_min=1.0)
    print(f"[bench] workload built: {n}^3, {na} views, gel voxels {int((lp.labels == 2).sum())}, "
          f"band voxels {int((lp.labels == 1).sum())}, active rays {int(lp.act.sum())}", file=sys.stderr, flush=True)

    # --- warm-up solve; the timed solve (graph-captured iteration blocks, as a caller runs it); then a
    # profiled solve of the same length (HIP events on the solve's stream) for the per-phase times
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        wres = sipo.solve(lp, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=max(args.warmup, 1), tol=1e-12,
                                                tune_operators=1, progress_every=1 << 30, use_graph=1), want_dose=False)
        # the 256^3 line keeps the fixed splits its counter record describes; the 512^3 workload (no
        # counter record) runs the tuner's pick
        ops_run = wres["op_config"] if big else BENCH_OPS
        torch.cuda.synchronize()
        print(f"[bench] warmup {args.warmup} iterations done", file=sys.stderr, flush=True)
        lp.y.zero_(); lp.lam_up.zero_(); lp.lam_lo.zero_()
        opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=args.steps, tol=1e-12, check_every=64, use_graph=1,
                                 op_config=ops_run)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sipo.solve(lp, opts, want_dose=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        iters = res["iters"]
        loop_s = res["loop_ms"] * 1e-3
        ips = iters / loop_s
        print(f"[bench] {iters} iterations in {loop_s:.4f} s of solver loop ({dt:.4f} s for the whole call, "
              f"graph-captured blocks)", file=sys.stderr, flush=True)
        lp.y.zero_(); lp.lam_up.zero_(); lp.lam_lo.zero_()
        popts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=args.steps, tol=1e-12, check_every=64, profile=1,
                                  op_config=ops_run)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        pres = sipo.solve(lp, popts, want_dose=False)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp0
    ph_ms, ph_n = pres["phase_ms"], pres["phase_launches"]
    ph_avg = {k: (ph_ms[k] / ph_n[k] if ph_n[k] else 0.0) for k in ph_ms}
    print(f"[bench] profiled solve: {pres['iters']} iterations in {dtp:.3f} s; per-phase ms per launch: "
          + ", ".join(f"{k} {v:.4f}" for k, v in ph_avg.items()), file=sys.stderr, flush=True)

    # --- operator pair and roofline of the dominant kernel.  Inside the solve the 3D operators skip
    # the work the LP never reads, so their algorithmic work is that of the LP's operators: P on the
    # active rays, P^T on the voxels the blurred dose is read at (2 flop per nonzero).
    import numpy as np
    from sipo_inputs import angles_uniform as _ang
    rad = len(sipo.gaussian_taps(sigma[0])) // 2, len(sipo.gaussian_taps(sigma[1])) // 2, len(sipo.gaussian_taps(sigma[2])) // 2
    work = lp_work(n, _ang(na), plan.n_bins, lp.labels.cpu().numpy(), lp.act.cpu().numpy(), (rad[2], rad[1], rad[0]))
    print(f"[bench] LP operator work: {work}", file=sys.stderr, flush=True)
    t_p, t_bp = ph_avg["project"], ph_avg["backproject"]
    dom = max(("project", "backproject"), key=lambda k: ph_avg[k])
    flops = 2.0 * (work["p_nnz_active"] if dom == "project" else work["bp_nnz_needed"])
    achieved = flops / (ph_avg[dom] * 1e-3) / 1e12
    p_kernel = in_solve_projector(tuning, pres["op_config"])
    traffic = recorded_traffic(p_kernel) if (dom == "project" and not big) else None
    ops = full_operators(plan, dev, work)
    print(f"[bench] standalone operators (median of 20): {ops}", file=sys.stderr, flush=True)

    ttk = None
    if args.ttk and not big:   # the 512^3 workload runs at about 9 ms per iteration: no time-to-1e-4 leg
        lp.y.zero_(); lp.lam_up.zero_(); lp.lam_lo.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # graph-captured like the timed solve; the solver reports its residuals every 64 checks
        with torch.cuda.stream(stream):
            r = sipo.solve(lp, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=args.ttk_iters, tol=1e-4, use_graph=1,
                                                 progress_every=64, op_config=ops_run), want_dose=False)
            torch.cuda.synchronize()
        ttk = {"seconds": round(time.perf_counter() - t1, 3), "iters": r["iters"], "status": r["status_name"],
               "restarts": r["restarts"], "objective": r["primal_obj"], "rel_primal": r["rel_primal"],
               "rel_dual": r["rel_dual"], "rel_gap": r["rel_gap"]}
        print(f"[bench] time to 1e-4: {ttk}", file=sys.stderr, flush=True)

    bvp = batch_vs_plain(args.batch, dev, screened=args.screened) if args.batch > 0 else None
    cpu = None if (args.no_cpu_baseline or big) else cpu_baseline(n, na, args.cpu_slices)
    line = {
        "metric": "PDHG iters/s",
        "value": round(ips, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * loop_s / max(iters, 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": ({"workload": f"3D {n}^3 vial, {na} views over 360 deg, {n}x{n} detector, jittered lattice "
                                f"(seed 4000), band 10, blur sigma (1,1,2), Case 2 cap 0.65, restarted PDHG",
                    "n": n, "views": na, "case": 2, "blur_sigma": [1.0, 1.0, 2.0]} if big else
                   {"workload": f"3D {n}^3 vial, {na} views over 360 deg, {n}x{n} detector, 6 random ellipsoids "
                                f"(seed 3000), band 10, blur sigma 1.5, Case 1 [0.9,1.0], restarted PDHG",
                    "n": n, "views": na, "case": 1, "blur_sigma": 1.5}),
        "setup_ms": round(res["time_ms"] - res["loop_ms"], 3),
        "solve_call_s": round(dt, 4),
        "solve_call_iters_per_s": round(iters / dt, 3),
        # standalone full operators (every ray and voxel, ABI layouts): algorithmic bytes over time
        "a_plus_at_gbs": ops["a_plus_at_gbs"],
        "full_operators": ops,
        # the same pair inside the solve: the masked operators of the LP (active rays, needed voxels)
        "in_solve_pair_ms": round(t_p + t_bp, 4),
        "phase_ms": {k: round(v, 4) for k, v in ph_avg.items()},
        "profiled_solve_iters_per_s": round(pres["iters"] / (pres["loop_ms"] * 1e-3), 3),
        "tuning": tuning,
        # the masked operators' work splits of the timed and profiled solves, and the solver's own
        # tuner's pick in the warm-up solve
        "in_solve_ops": res["op_config"],
        "in_solve_ops_tuned": wres["op_config"],
        "roofline": {"bound": "alu", "kernel": (p_kernel + " (LP rays)" if dom == "project" else "backproject3d (LP voxels)"),
                     "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": traffic},
        "roofline_full_operator": {"bound": "alu", "kernel": "project3d (all rays, standalone ABI call)",
                                   "ms": ops["p_ms"], "achieved": round(2.0 * work["p_nnz_full"] / (ops["p_ms"] * 1e-3) / 1e12, 3),
                                   "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ops["p_valu_frac"]},
        "lp_operator_work": work,
        "cpu_baseline": cpu,
    }
    if ttk is not None:
        line["time_to_1e-4"] = ttk
    if bvp is not None:
        line["batched_vs_plain_time_to_1e-4"] = bvp
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

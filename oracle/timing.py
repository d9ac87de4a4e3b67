"""Wall-clock cost of the FP64 oracle per workload (test infrastructure, not part of the GPU path).

Times, on the host that runs it and with one thread (SciPy's sparse products do not multithread),
what the oracle spends per operator application and per PDHG iteration, and how long its solves to a
relative KKT error of 1e-4 take where they finish in reasonable time:

* P and P^T applications on U[0, 1) fields (seeds 3002 and 3001), the blur K where the workload has
  a PSF, and the explicit slice matrix's construction, each the median of several runs when one run
  is short;
* one restarted-PDHG iteration (Sec. 2.8; one Chambolle-Pock step with diagonal steps, i.e. the
  operator pair, two blurs and the updates) on the workload's LP;
* solves: the 64^2 slice runs 2000 plain PDHG iterations (its stated budget); the 256^2 slice (both
  cases) and the reduced 3D instance (64^3, 90 views, blur 1.5, Case 1; at most 120000 iterations)
  run restarted PDHG to 1e-4;
* the uneven 2D batch: P and P^T per distinct (grid, views) shape, and their sum over the batch.

Every figure is measured; nothing is scaled from a smaller run.

    python -m oracle.timing slice64|slice256|batch64|vol64|vol256|vol512 [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time
from collections import Counter

import numpy as np

from . import blur as _blur, lp as _lp, pdhg as _pdhg
from .geometry import make_geometry
from .projector import Projector


def _host() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "cores": len(os.sched_getaffinity(0)), "threads_used": 1}


def _timed(fn, min_total: float = 1.0, max_reps: int = 7) -> float:
    """Median seconds of fn() over repeated runs (one run if it alone takes longer than min_total)."""
    ts = []
    start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
        if len(ts) >= max_reps or time.perf_counter() - start >= min_total:
            break
    return statistics.median(ts)


def _log(msg: str) -> None:
    print(f"[oracle timing] {msg}", file=sys.stderr, flush=True)


def operators(n: int, angles, nz: int = 1, sigma=None) -> dict:
    from sipo_inputs import uniform_field
    t0 = time.perf_counter()
    P = Projector(make_geometry(n, angles, nz=nz, atten=1.0))
    out = {"build_s": time.perf_counter() - t0, "nnz_slice_matrix": int(P.PT.nnz)}
    g = P.geom
    x = uniform_field(g.vol_shape, 3002)
    y = uniform_field(g.sino_shape, 3001)
    out["p_s"] = _timed(lambda: P.project(x))
    out["pt_s"] = _timed(lambda: P.backproject(y))
    if sigma is not None:
        taps = _blur.psf_taps(sigma)
        out["k_s"] = _timed(lambda: _blur.apply(x, taps))
    _log(f"operators {n}^2 x {nz} x {len(angles)} views: {out}")
    return out, P


def iteration(prob) -> dict:
    sc = _pdhg.diagonal_scaling(prob)
    st = _pdhg.initial_state(prob)
    e = 0.95

    def one():
        nonlocal st
        st = _pdhg.step(prob, st, e * sc.T, e * sc.Tu, e * sc.Tv, e * sc.S_up, e * sc.S_lo)
    return {"iter_s": _timed(one, min_total=2.0, max_reps=5)}


def restarted_solve(prob, tol=1e-4, max_iters=200000) -> dict:
    t0 = time.perf_counter()
    r = _pdhg.pdhg_restarted(prob, tol=tol, max_iters=max_iters, infeas_tol=tol)
    dt = time.perf_counter() - t0
    names = {_pdhg.OPTIMAL: "optimal", _pdhg.PRIMAL_INFEASIBLE: "infeasible", _pdhg.ITER_LIMIT: "iter_limit",
             _pdhg.NUMERICAL: "numerical"}
    return {"seconds": dt, "status": names.get(r.status, str(r.status)), "iters": r.iters, "restarts": r.restarts,
            "rel_kkt": float(max(r.kkt.eps_p, r.kkt.eps_d, r.kkt.eps_gap)) if r.kkt is not None else None}


def run(workload: str) -> dict:
    from sipo_inputs import (angles_uniform, ellipses_target, annulus_disks_target, ellipsoids_target,
                             lattice_target, batch_instances)
    res = {"workload": workload, "host": _host()}
    if workload == "slice64":
        ops, P = operators(64, angles_uniform(180))
        prob = _lp.build(P, ellipses_target(64, 0), _lp.CASE1, band_width=10.0)
        res.update(ops, **iteration(prob))
        t0 = time.perf_counter()
        _pdhg.pdhg_plain(prob, 2000)
        res["plain_2000_iters_s"] = time.perf_counter() - t0
    elif workload == "slice256":
        ops, P = operators(256, angles_uniform(360))
        f = annulus_disks_target(256, 1000)
        p1 = _lp.build(P, f, _lp.CASE1, band_width=10.0)
        res.update(ops, **iteration(p1))
        res["solve_case1"] = restarted_solve(p1)
        _log(f"slice256 case 1: {res['solve_case1']}")
        res["solve_case2"] = restarted_solve(_lp.build(P, f, _lp.CASE2, band_width=10.0, cap=0.7))
        _log(f"slice256 case 2: {res['solve_case2']}")
    elif workload == "batch64":
        insts = batch_instances(64, 2000)
        shapes = Counter((b.n, b.n_angles) for b in insts)
        per = {}
        for (n, na), _ in sorted(shapes.items()):
            ops, _ = operators(n, angles_uniform(na))
            per[f"{n}x{na}"] = {k: ops[k] for k in ("p_s", "pt_s", "build_s")}
        res["shapes"] = {f"{n}x{na}": c for (n, na), c in sorted(shapes.items())}
        res["per_shape"] = per
        res["batch_p_plus_pt_s"] = sum(c * (per[f"{n}x{na}"]["p_s"] + per[f"{n}x{na}"]["pt_s"])
                                       for (n, na), c in shapes.items())
    elif workload == "vol64":
        sigma = (1.5, 1.5, 1.5)
        ops, P = operators(64, angles_uniform(90), nz=64, sigma=sigma)
        prob = _lp.build(P, ellipsoids_target(64, 3100), _lp.CASE1, taps=_blur.psf_taps(sigma), band_width=10.0)
        res.update(ops, **iteration(prob))
        _log(f"vol64 iteration: {res['iter_s']:.4f} s")
        # about 70 ms per iteration on one core: the budget bounds the solve to a few hours
        res["solve_case1"] = restarted_solve(prob, max_iters=120000)
        _log(f"vol64 case 1: {res['solve_case1']}")
    elif workload == "vol256":
        sigma = (1.5, 1.5, 1.5)
        ops, P = operators(256, angles_uniform(360), nz=256, sigma=sigma)
        prob = _lp.build(P, ellipsoids_target(256, 3000), _lp.CASE1, taps=_blur.psf_taps(sigma), band_width=10.0)
        res.update(ops, **iteration(prob))
    elif workload == "vol512":
        sigma = (1.0, 1.0, 2.0)
        ops, P = operators(512, angles_uniform(720), nz=512, sigma=sigma)
        res.update(ops)
        prob = _lp.build(P, lattice_target(512, 4000), _lp.CASE2, taps=_blur.psf_taps(sigma), band_width=10.0,
                         cap=0.65)
        res.update(iteration(prob))
    else:
        raise SystemExit(f"unknown workload {workload}")
    return res


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload", choices=["slice64", "slice256", "batch64", "vol64", "vol256", "vol512"])
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        res = run(a.workload)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()

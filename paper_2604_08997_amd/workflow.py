"""Two-stage Case 1 -> Case 2 design and trade-off sweeps (Sec. 3.2) as batched GPU solves.

Host-side orchestration only: every LP is solved by ``sipo_pdhg_solve`` (all
instances of a stage in one batched call), and regions, active rays, doses and
metrics come from the library's kernels.

Units.  All stages use the normalisation of the general LP, f_crit = min_gel
f_T, so a binary target has gel lower bound L = 1 (Case 1 with window
[tol_lo, tol_hi] f_T has the same L and upper bound tol_hi / tol_lo).  Case 2
at band threshold ``cap`` (f_crit = cap min f_T, band cap 1; Eq. 39-41) is the
same LP as "band cap h = cap, f~_T = 1" after the joint rescaling of f~_T and
the band cap by cap (Sec. 2.6.2): v* is unchanged and y is cap times larger.
Stage 2 is posed that way, so the stage-1 projections are a feasible starting
point for it without any rescaling.

The h_min LP (general LP with w = (1, 0)) gives the smallest band threshold for
which Case 2 is feasible at all; it needs no stage-1 result and runs in the
stage-1 batch.
"""
from __future__ import annotations

import math
import time

from . import binding as _b


def _levels(plan, f_target, labels):
    """min_gel f_T and the general-units normalised target f~_T = f_T / min_gel f_T as a per-voxel
    array (graded targets) or None (single-level targets, where f~_T = 1 on the gel)."""
    fmin, level = _b.target_levels(plan, f_target, labels)
    return fmin, level(1.0 / fmin)


def h_min_lp(plan, labels, act, f_min, ftn=None):
    """General LP with w = (1, 0): min u s.t. D <= u on band, D >= f~_T on gel (v free, unpriced)."""
    return _b.LP(plan, labels, act, _b.GENERAL, 1, 1, 1.0, 0.0, 1.0, 1.0, 1.0, lo_arr=ftn, hi_arr=ftn, f_crit=f_min)


def case2_lp(plan, labels, act, f_min, cap, ftn=None):
    """Case 2 (Eq. 40-45) at band threshold ``cap`` in general units: band cap h = cap, D = f~_T on the
    gel's lower rows and D <= v f~_T on its upper rows, w = (0, 1)."""
    return _b.LP(plan, labels, act, _b.CASE2, 0, 1, 0.0, 1.0, float(cap), 1.0, 1.0, lo_arr=ftn, hi_arr=ftn,
                 f_crit=f_min)


def transfer_cap(u1, margin):
    """Band threshold handed to stage 2: the stage-1 bound widened by a relative margin."""
    return float(u1) * (1.0 + float(margin))


def _metrics(lp, f_min, ftn=None):
    if lp.dose is None:
        return None
    return lp.plan.evaluate(lp.dose, lp.labels, f_target_norm=ftn, f_t_scalar=1.0, f_crit=f_min)


def two_stage(items, band_width=10.0, tol_lo=0.9, tol_hi=1.0, margin=0.02, opts=None, warm=True,
              with_h_min=True, workspace=None, times=None):
    """Run the two-stage workflow on every (plan, f_target) in ``items``.

    Stage 1: Case 1 on the window [tol_lo, tol_hi] f_T for every item (and the
    h_min LP when ``with_h_min``), one batched solve.  Stage 2: Case 2 at
    cap = u1 (1 + margin) for every item whose stage 1 is optimal, one batched
    solve, warm-started from the stage-1 projections (feasible for stage 2,
    with v = tol_hi / tol_lo) when ``warm``.

    Returns one dict per item: ``stage1`` / ``stage2`` / ``h_min`` solver
    results, ``u1``, ``cap``, ``f_min``, ``metrics1`` / ``metrics2`` (scale-
    invariant metrics of each stage's dose in general units) and the LP
    objects ``lp1`` / ``lp2`` holding y, duals and doses.  ``times``, if a
    dict, receives the wall-clock seconds of each stage's batched solve.
    """
    opts = _b.pdhg_options() if opts is None else opts
    lp1s, hms, fmins, ftns = [], [], [], []
    for plan, f in items:
        lp1 = _b.LP.build(plan, f, _b.CASE1, band_width=band_width, tol_lo=tol_lo, tol_hi=tol_hi)
        fmin = lp1.f_crit / tol_lo
        ftn = lp1.lo_arr          # f~_T per voxel for graded targets (Case 1's L is f_T / min f_T)
        lp1s.append(lp1)
        fmins.append(fmin)
        ftns.append(ftn)
        if with_h_min:
            hms.append(h_min_lp(plan, lp1.labels, lp1.act, fmin, ftn))
    t0 = time.perf_counter()
    res_a = _b.solve(lp1s + hms, opts, workspace=workspace)
    if times is not None:
        times["stage1"] = time.perf_counter() - t0
    res1, resh = res_a[:len(lp1s)], res_a[len(lp1s):]
    out = []
    lp2s = []
    for k, (lp1, r1, fmin) in enumerate(zip(lp1s, res1, fmins)):
        d = {"stage1": r1, "lp1": lp1, "f_min": fmin, "u1": math.nan, "cap": math.nan, "stage2": None,
             "lp2": None, "h_min": resh[k]["u"] if with_h_min and resh[k]["status_name"] == "optimal" else math.nan,
             "h_min_result": resh[k] if with_h_min else None, "metrics1": _metrics(lp1, fmin, ftns[k]),
             "metrics2": None, "ftn": ftns[k]}
        if r1["status_name"] == "optimal":
            d["u1"] = r1["u"]
            d["cap"] = transfer_cap(r1["u"], margin)
            lp2 = case2_lp(lp1.plan, lp1.labels, lp1.act, fmin, d["cap"], ftns[k])
            if warm:
                lp2.y.copy_(lp1.y)
                lp2.v0 = tol_hi / tol_lo
            d["lp2"] = lp2
            lp2s.append((k, lp2))
        out.append(d)
    if lp2s:
        t0 = time.perf_counter()
        res_b = _b.solve([lp for _, lp in lp2s], opts, workspace=workspace)
        if times is not None:
            times["stage2"] = time.perf_counter() - t0
        for (k, lp2), r2 in zip(lp2s, res_b):
            out[k]["stage2"] = r2
            out[k]["metrics2"] = _metrics(lp2, out[k]["f_min"], out[k]["ftn"])
    return out


def sweep(plan, f_target, weights, band_widths, opts=None, f_min=None, workspace=None):
    """General LP over every (w1, w2) in ``weights`` and band width in ``band_widths`` as one batched solve.

    ``math.inf`` (or None) in ``band_widths`` is the band-free configuration
    (every non-gel vial voxel is band, Sec. 3.2).  Region labels are computed
    once per band width and the active rays once.  Returns a list of dicts
    (band width major, weight pair minor) with the solver ``result``, the
    ``metrics`` of the dose and the ``lp`` object.
    """
    opts = _b.pdhg_options() if opts is None else opts
    act = plan.active_rays(f_target)
    lps, keys = [], []
    for bw in band_widths:
        labels = plan.regions(f_target, bw)
        fmin, ftn = _levels(plan, f_target, labels)
        if f_min is not None:
            fmin = float(f_min)
        for w1, w2 in weights:
            lps.append(_b.LP(plan, labels, act, _b.GENERAL, 1, 1, float(w1), float(w2), 1.0, 1.0, 1.0, lo_arr=ftn,
                             hi_arr=ftn, f_crit=fmin))
            keys.append((math.inf if bw is None else bw, float(w1), float(w2), fmin, ftn))
    res = _b.solve(lps, opts, workspace=workspace)
    return [{"band_width": bw, "w1": w1, "w2": w2, "result": r, "lp": lp, "metrics": _metrics(lp, fmin, ftn)}
            for (bw, w1, w2, fmin, ftn), r, lp in zip(keys, res, lps)]


def case2_screened(items, caps, band_width=10.0, opts=None, h_min_opts=None, workspace=None, times=None):
    """Case 2 at given band thresholds, screened by the h_min LP.

    ``caps[k]`` is item k's band threshold as a fraction of min gel f_T (the
    paper's Case-2 parameter, Eq. 39).  Stage A solves the h_min LP of every
    item in one batch (``h_min_opts``, default ``opts``).  Stage B solves every
    Case 2 in one batch, posed in general units (band cap h = cap).  An item
    whose cap lies below its h_min estimate starts from the h_min multipliers:
    those form a Farkas ray for it (band multipliers summing to 1, gel lower
    multipliers summing to h_min > cap), and the solver's own test accepts them
    at iteration 0 when they are accurate to its infeas_tol.  Other items start
    cold.  Returns one dict per item: ``h_min``, ``h_min_result``, ``result``,
    ``screened`` (started from the h_min multipliers) and ``lp``.
    """
    opts = _b.pdhg_options() if opts is None else opts
    h_min_opts = opts if h_min_opts is None else h_min_opts
    hms, fmins, ftns = [], [], []
    for plan, f in items:
        labels = plan.regions(f, band_width)
        act = plan.active_rays(f)
        fmin, ftn = _levels(plan, f, labels)
        hms.append(h_min_lp(plan, labels, act, fmin, ftn))
        fmins.append(fmin)
        ftns.append(ftn)
    t0 = time.perf_counter()
    rh = _b.solve(hms, h_min_opts, want_dose=False, workspace=workspace)
    if times is not None:
        times["h_min"] = time.perf_counter() - t0
    lps, screened = [], []
    for hm, r, fmin, cap, ftn in zip(hms, rh, fmins, caps, ftns):
        lp = case2_lp(hm.plan, hm.labels, hm.act, fmin, cap, ftn)
        below = r["status_name"] in ("optimal", "iter_limit") and float(cap) < r["u"]
        if below:
            lp.lam_up.copy_(hm.lam_up)
            lp.lam_lo.copy_(hm.lam_lo)
        lps.append(lp)
        screened.append(below)
    t0 = time.perf_counter()
    res = _b.solve(lps, opts, workspace=workspace)
    if times is not None:
        times["case2"] = time.perf_counter() - t0
    return [{"h_min": r["u"] if r["status_name"] == "optimal" else math.nan, "h_min_result": r, "result": rc,
             "screened": s, "lp": lp} for r, rc, s, lp in zip(rh, res, screened, lps)]

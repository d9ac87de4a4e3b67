"""Two-stage Case 1 -> Case 2 design and trade-off sweeps (Sec. 3.2) -- oracle side.

TEST INFRASTRUCTURE ONLY: exact LP solves (HiGHS) composed in the order the
paper describes; small instances.

Units.  Every stage is posed in the normalisation of the general LP, where
f_crit = min_gel f_T and the gel lower bound is L = f_T / f_crit (Case 1 with
window [tol_lo, tol_hi] f_T has the same L, since its f_crit = tol_lo min f_T
scales f_L = tol_lo f_T by the same factor).  In these units

  * ``h_min`` is the smallest band dose any y >= 0 reaches while every gel
    voxel meets L: the general LP with w = (1, 0) (v free and unpriced, so the
    gel has no upper bound);
  * Case 1 gives u1 = min band dose subject to L <= D <= (tol_hi / tol_lo) L;
  * Case 2 with band threshold ``cap`` (f_crit = cap min f_T, band cap 1,
    Eq. 39-41) is, after the joint rescaling of f~_T and the band cap by cap
    (the scale gauge of Sec. 2.6.2), the LP "min v s.t. D <= cap on band,
    L <= D <= v L on gel"; v* does not depend on the rescaling and y differs
    by the factor cap.  Case 2 is feasible iff cap >= h_min.

The two-stage workflow: stage 1 solves Case 1 and reads off the process bound
u1 it achieves; stage 2 solves Case 2 at cap = u1 (1 + margin).  The Case-1
optimum is feasible for stage 2 (band <= u1 <= cap, gel inside the window), so
stage 2 is feasible by construction, attains v2* <= tol_hi / tol_lo, and keeps
the separation: its gel minimum over band maximum is at least 1 / cap.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import lp as _lp


def case2_in_general_units(proj, f_target, cap, taps=None, band_width=10.0) -> _lp.LPProblem:
    """Case 2 (Eq. 40-45) at band threshold ``cap``, posed with f_crit = min f_T: band cap h = cap."""
    base = _lp.build(proj, f_target, _lp.GENERAL, taps=taps, band_width=band_width)
    return _lp.LPProblem(base.proj, base.taps, base.labels, base.act, base.lo, base.hi, False, True, 0.0, 1.0,
                         float(cap), _lp.CASE2, base.f_crit, {"cap": float(cap)})


def h_min(proj, f_target, taps=None, band_width=10.0) -> float:
    """Smallest feasible Case-2 band threshold, as a fraction of min gel f_T."""
    prob = _lp.build(proj, f_target, _lp.GENERAL, taps=taps, band_width=band_width, w1=1.0, w2=0.0)
    s = _lp.solve_highs(prob)
    if s.status != "optimal":
        raise RuntimeError(f"h_min LP: {s.status}")
    return float(s.u)


@dataclass
class TwoStage:
    stage1: _lp.LPSolution
    u1: float                   # process bound reached by Case 1 (general units)
    cap: float                  # band threshold handed to Case 2
    stage2: _lp.LPSolution      # None when stage 1 is infeasible
    prob1: _lp.LPProblem
    prob2: _lp.LPProblem


def transfer_cap(u1: float, margin: float) -> float:
    """Band threshold for stage 2: the stage-1 bound widened by a relative margin."""
    return float(u1) * (1.0 + float(margin))


def two_stage(proj, f_target, taps=None, band_width=10.0, tol_lo=0.9, tol_hi=1.0, margin=0.0) -> TwoStage:
    """Stage 1: Case 1 on the window [tol_lo, tol_hi] f_T.  Stage 2: Case 2 at the bound stage 1 reached."""
    p1 = _lp.build(proj, f_target, _lp.CASE1, taps=taps, band_width=band_width, tol_lo=tol_lo, tol_hi=tol_hi)
    s1 = _lp.solve_highs(p1)
    if s1.status != "optimal":
        return TwoStage(s1, math.nan, math.nan, None, p1, None)
    cap = transfer_cap(s1.u, margin)
    p2 = case2_in_general_units(proj, f_target, cap, taps=taps, band_width=band_width)
    s2 = _lp.solve_highs(p2)
    return TwoStage(s1, float(s1.u), cap, s2, p1, p2)


def case2_bound_by_bisection(proj, f_target, ratio, lo, hi, taps=None, band_width=10.0, steps=40) -> float:
    """Smallest cap in [lo, hi] whose Case-2 optimum v*(cap) <= ratio, by bisection over Case-2 solves.

    This is the parameter sweep the two-stage workflow replaces: v*(cap) is
    non-increasing in cap, so the threshold is the Case-1 bound u1 of the
    window ratio tol_hi / tol_lo.
    """
    def ok(c):
        s = _lp.solve_highs(case2_in_general_units(proj, f_target, c, taps=taps, band_width=band_width))
        return s.status == "optimal" and s.v <= ratio * (1.0 + 1e-9)
    if not ok(hi):
        raise ValueError("upper end of the bracket is not admissible")
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi


def sweep(proj, f_target, weights, band_widths, taps=None):
    """General LP over every (w1, w2) in ``weights`` and band width in ``band_widths`` (inf = band-free).

    Returns a list of (band_width, w1, w2, LPProblem, LPSolution) in the order
    band width major, weight pair minor.  Parity unpinned as a unit; each
    instance is one exact LP solve, and the tests pin the trade-off structure
    the sweep exposes (weighted-sum monotonicity, band nesting, agreement of
    general-LP points with Case 1 and Case 2 at the same bounds).
    """
    out = []
    for bw in band_widths:
        for w1, w2 in weights:
            p = _lp.build(proj, f_target, _lp.GENERAL, taps=taps, band_width=bw, w1=w1, w2=w2)
            out.append((bw, w1, w2, p, _lp.solve_highs(p)))
    return out


def separation(prob: _lp.LPProblem, y: np.ndarray) -> float:
    """min over gel of D / L divided by max over band of D (in the problem's units); inf with no band dose."""
    D = prob.dose(y)
    g, b = prob.gel, prob.band
    gmin = float(np.min(D[g] / prob.lo[g])) if g.any() else math.nan
    bmax = float(np.max(D[b])) if b.any() else 0.0
    return gmin / bmax if bmax > 0 else math.inf

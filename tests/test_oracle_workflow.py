"""Pins for the two-stage workflow, the h_min feasibility threshold and trade-off sweeps (Sec. 3.2).

Each pin ties one oracle construction to another that does not share its
arithmetic: the paper's own Case-2 builder (f_crit = cap min f_T, band cap 1)
against the general-units form, Case 1 and Case 2 against the general LP's
Pareto points, and the two-stage result against the cap sweep it replaces.
"""
import math

import numpy as np
import pytest

from oracle import lp, workflow
from oracle.geometry import make_geometry
from oracle.projector import Projector
from sipo_inputs import ellipses_target

N, ANGLES, BAND = 12, 16, 2.0


def setup(seed):
    P = Projector(make_geometry(N, ANGLES, atten=1.0))
    return P, ellipses_target(N, seed)


@pytest.mark.parametrize("seed", [1, 3])
def test_h_min_is_the_case2_feasibility_threshold(seed):
    # the paper's Case-2 builder at cap just below / above h_min: infeasible / feasible (Sec. 2.7.2)
    P, f = setup(seed)
    hm = workflow.h_min(P, f, band_width=BAND)
    assert 0.0 < hm < 1.0
    below = lp.solve_highs(lp.build(P, f, lp.CASE2, band_width=BAND, cap=hm * (1 - 1e-3)))
    above = lp.solve_highs(lp.build(P, f, lp.CASE2, band_width=BAND, cap=hm * (1 + 1e-3)))
    assert below.status == "infeasible"
    assert above.status == "optimal"


def test_case2_general_units_is_the_papers_case2_rescaled():
    # joint rescaling of f~_T and the band cap by cap keeps v* and scales y by cap (Sec. 2.6.2)
    P, f = setup(1)
    cap = 0.85
    paper = lp.solve_highs(lp.build(P, f, lp.CASE2, band_width=BAND, cap=cap))
    gen = lp.solve_highs(workflow.case2_in_general_units(P, f, cap, band_width=BAND))
    assert paper.status == gen.status == "optimal"
    assert gen.v == pytest.approx(paper.v, rel=1e-8)
    p2 = workflow.case2_in_general_units(P, f, cap, band_width=BAND)
    # the paper-units optimum, multiplied by cap, is optimal in general units
    assert p2.violation(paper.y * cap, cap, paper.v) < 1e-8


@pytest.mark.parametrize("seed", [1, 3])
def test_two_stage_is_feasible_and_keeps_the_separation(seed):
    P, f = setup(seed)
    res = workflow.two_stage(P, f, band_width=BAND, margin=1e-3)
    assert res.stage1.status == "optimal" and res.stage2.status == "optimal"
    hm = workflow.h_min(P, f, band_width=BAND)
    assert res.u1 >= hm * (1 - 1e-9)
    assert res.cap == pytest.approx(res.u1 * 1.001, rel=1e-12)
    # the Case-1 optimum is a feasible point of stage 2
    assert res.prob2.violation(res.stage1.y, res.cap, 1.0 / 0.9) < 1e-9
    # so stage 2 reaches at most the window ratio, and its separation is at least 1 / cap
    assert res.stage2.v <= (1.0 / 0.9) * (1 + 1e-9)
    assert workflow.separation(res.prob2, res.stage2.y) >= (1.0 / res.cap) * (1 - 1e-7)
    # stage 1 separation is 1 / u1 (gel floor at L, band max at u1)
    assert workflow.separation(res.prob1, res.stage1.y) == pytest.approx(1.0 / res.u1, rel=1e-6)


def test_two_stage_bound_matches_the_cap_sweep_it_replaces():
    # bisection over Case-2 caps for v*(cap) <= tol_hi / tol_lo lands on the Case-1 bound u1
    P, f = setup(1)
    res = workflow.two_stage(P, f, band_width=BAND, margin=0.0)
    hm = workflow.h_min(P, f, band_width=BAND)
    c = workflow.case2_bound_by_bisection(P, f, 1.0 / 0.9, hm, 1.0, band_width=BAND, steps=40)
    assert c == pytest.approx(res.u1, rel=1e-6)


def test_general_lp_pareto_points_agree_with_case1_and_case2():
    # a weighted-sum optimum (u_g, v_g) with w1, w2 > 0 is Pareto optimal: Case 2 at cap u_g attains
    # v_g, and Case 1 with window ratio v_g attains u_g (Eq. 19-24 vs Eq. 32-37 and 40-45)
    P, f = setup(3)
    for w1, w2 in [(1.0, 1.0), (3.0, 1.0), (1.0, 4.0)]:
        g = lp.solve_highs(lp.build(P, f, lp.GENERAL, band_width=BAND, w1=w1, w2=w2))
        assert g.status == "optimal"
        c2 = lp.solve_highs(workflow.case2_in_general_units(P, f, g.u, band_width=BAND))
        assert c2.v == pytest.approx(g.v, rel=1e-6)
        c1 = lp.solve_highs(lp.build(P, f, lp.CASE1, band_width=BAND, tol_lo=1.0, tol_hi=g.v))
        assert c1.u == pytest.approx(g.u, rel=1e-6)


def test_sweep_trade_off_structure():
    P, f = setup(1)
    weights = [(0.25, 1.0), (1.0, 1.0), (4.0, 1.0), (16.0, 1.0)]
    bands = [1.0, 2.0, 4.0, math.inf]
    out = workflow.sweep(P, f, weights, bands)
    assert len(out) == len(weights) * len(bands)
    assert [(r[0], r[1], r[2]) for r in out] == [(b, w1, w2) for b in bands for w1, w2 in weights]
    grid = {(b, w1): r[4] for b, w1, w2, _, r in [(r[0], r[1], r[2], r[3], r) for r in out]}
    for b in bands:
        sols = [grid[(b, w1)] for w1, _ in weights]
        assert all(s.status == "optimal" for s in sols)
        # pricing u more pushes u down and v up (weighted-sum monotonicity)
        us, vs = [s.u for s in sols], [s.v for s in sols]
        assert all(us[k + 1] <= us[k] * (1 + 1e-7) + 1e-9 for k in range(len(us) - 1))
        assert all(vs[k + 1] >= vs[k] * (1 - 1e-7) - 1e-9 for k in range(len(vs) - 1))
    # bands are nested (inf = every non-gel vial voxel), so the optimum never improves as the band widens
    labels = [out[k * len(weights)][3].labels for k in range(len(bands))]
    for a, b in zip(labels, labels[1:]):
        assert np.all((a == 1) <= (b == 1)) and np.array_equal(a == 2, b == 2)
    for w1, _ in weights:
        objs = [grid[(b, w1)].objective for b in bands]
        assert all(objs[k + 1] >= objs[k] * (1 - 1e-9) for k in range(len(objs) - 1))

"""Pins for the oracle LP (Eq. 19-45), simplex, KKT checker and PDHG (Sec. 2.8)."""
import json
import os

import numpy as np
import pytest

from oracle import lp, simplex, kkt, pdhg, metrics, blur
from oracle.geometry import make_geometry
from oracle.projector import Projector
from sipo_inputs import ellipses_target, ellipsoids_target

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def tiny(case, seed=1, n=12, angles=16, band=2.0, **kw):
    g = make_geometry(n, angles, atten=1.0)
    P = Projector(g)
    f = ellipses_target(n, seed)
    return lp.build(P, f, case, band_width=band, **kw)


def tiny3d(case, seed=2, **kw):
    g = make_geometry(8, 10, nz=6, atten=1.0)
    P = Projector(g)
    f = ellipsoids_target(8, seed, count=2, nz=6)
    return lp.build(P, f, case, taps=blur.psf_taps((1.0, 1.0, 1.0)), band_width=2.0, **kw)


CASES = [lp.GENERAL, lp.CASE1, lp.CASE2]


def test_builders_follow_the_paper_cases():
    facts = json.load(open(GOLDEN))["cases"]
    p1, p2 = tiny(lp.CASE1), tiny(lp.CASE2)
    assert [p1.w1, p1.w2] == facts["case1_weights"] and p1.u_free and not p1.v_free
    assert [p2.w1, p2.w2] == facts["case2_weights"] and p2.v_free and not p2.u_free
    assert p2.h == facts["case2_band_cap"]
    gel = p1.gel
    np.testing.assert_allclose(p1.lo[gel], 1.0)
    np.testing.assert_allclose(p1.hi[gel], 1.0 / 0.9)
    np.testing.assert_allclose(p2.lo[gel], 1.0 / 0.7)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [1, 4])
def test_dense_simplex_matches_highs(case, seed):
    prob = tiny(case, seed=seed)
    asm = lp.assemble(prob)
    ref = lp.solve_highs(prob)
    got = simplex.solve(asm.c, asm.G.toarray(), asm.h)
    assert got["status"] == ref.status
    if ref.status == "optimal":
        assert got["objective"] == pytest.approx(ref.objective, rel=1e-9, abs=1e-12)
        # the simplex multipliers also satisfy KKT
        y, u, v, lu, ll = lp.unpack(prob, asm, got["x"], got["lam"])
        assert kkt.residuals(prob, y, u, v, lu, ll).rel < 1e-8


def test_dense_simplex_matches_highs_3d_with_blur():
    for case in CASES:
        prob = tiny3d(case)
        asm = lp.assemble(prob)
        ref = lp.solve_highs(prob)
        got = simplex.solve(asm.c, asm.G.toarray(), asm.h)
        assert got["status"] == ref.status
        if ref.status == "optimal":
            assert got["objective"] == pytest.approx(ref.objective, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_kkt_checker_accepts_optimum_and_rejects_perturbations(case):
    prob = tiny(case)
    s = lp.solve_highs(prob)
    assert s.status == "optimal"
    k = kkt.residuals(prob, s.y, s.u, s.v, s.lam_up, s.lam_lo)
    assert k.rel < 1e-8
    assert abs(k.primal_obj - s.objective) < 1e-9
    bad_y = kkt.residuals(prob, 1.1 * s.y, s.u, s.v, s.lam_up, s.lam_lo)
    bad_l = kkt.residuals(prob, s.y, s.u, s.v, 1.3 * s.lam_up, s.lam_lo)
    assert bad_y.rel > 1e-4 and bad_l.rel > 1e-4


def test_general_lp_optimum_equals_the_fractional_objective():
    # Charnes-Cooper (Eq. 18-22): at y*, min gel ratio = 1 and the LP value equals
    # the linear-fractional objective of Eq. 9 evaluated at y*.
    for seed in (1, 2, 3):
        prob = tiny(lp.GENERAL, seed=seed, w1=1.0, w2=1.0)
        s = lp.solve_highs(prob)
        D = prob.dose(s.y)
        ft = prob.lo
        gel, band = prob.gel, prob.band
        ratio = D[gel] / ft[gel]
        assert ratio.min() == pytest.approx(1.0, rel=1e-8)
        lfp = (prob.w1 * D[band].max() + prob.w2 * ratio.max()) / ratio.min()
        assert lfp == pytest.approx(s.objective, rel=1e-8)
        # and equals w1 DSR + w2 DTVR (Eq. 8, f_crit-normalised target)
        assert prob.w1 * metrics.dsr(D, ft, prob.labels) + prob.w2 * metrics.dtvr(D, ft, prob.labels) \
            == pytest.approx(s.objective, rel=1e-8)


def test_case2_value_invariant_under_joint_rescaling():
    # scaling f~_T and the band cap together by c scales y by c and keeps v* (Sec. 2.6.2 scale gauge)
    base = tiny(lp.CASE2, seed=5, cap=0.9)
    s0 = lp.solve_highs(base)
    assert s0.status == "optimal"
    c = 3.7
    sc = tiny(lp.CASE2, seed=5, cap=0.9)
    sc.lo = sc.lo * c
    sc.hi = sc.hi * c
    sc.h = sc.h * c
    s1 = lp.solve_highs(sc)
    assert s1.objective == pytest.approx(s0.objective, rel=1e-8)


def h_min(seed):
    prob = tiny(lp.GENERAL, seed=seed, w1=1.0, w2=0.0)
    return lp.solve_highs(prob).objective


def test_infeasible_instances_and_farkas_certificates():
    # Case 1 with U < L and Case 2 with a cap below h_min are infeasible (Sec. 2.7)
    p1 = tiny(lp.CASE1, seed=2, tol_lo=1.0, tol_hi=0.95)
    hm = h_min(3)
    p2 = tiny(lp.CASE2, seed=3, cap=0.5 * hm)
    p2ok = tiny(lp.CASE2, seed=3, cap=min(1.0, 1.5 * hm))
    for p in (p1, p2):
        asm = lp.assemble(p)
        assert simplex.solve(asm.c, asm.G.toarray(), asm.h)["status"] == "infeasible"
        assert lp.solve_highs(p).status == "infeasible"
        r = pdhg.pdhg_restarted(p, tol=1e-8, max_iters=20000)
        assert r.status == pdhg.PRIMAL_INFEASIBLE
        assert kkt.farkas_check(p, *r.certificate, tol=1e-7)["valid"]
    assert lp.solve_highs(p2ok).status == "optimal"


def test_farkas_check_rejects_non_certificates():
    p = tiny(lp.CASE1, seed=2)
    s = lp.solve_highs(p)
    assert s.status == "optimal"
    assert not kkt.farkas_check(p, s.lam_up, s.lam_lo)["valid"]


def test_power_norm_matches_largest_singular_value():
    for case in CASES:
        prob = tiny(case)
        asm = lp.assemble(prob)
        want = np.linalg.norm(asm.G.toarray(), 2)
        assert pdhg.power_norm(prob, iters=400) == pytest.approx(want, rel=1e-6)


def test_diagonal_scaling_matches_explicit_abs_sums():
    for case in CASES:
        prob = tiny3d(case) if case == lp.CASE1 else tiny(case)
        asm = lp.assemble(prob)
        G = abs(asm.G).toarray()
        sc = pdhg.diagonal_scaling(prob)
        col = G.sum(axis=0)
        row = G.sum(axis=1)
        np.testing.assert_allclose(sc.T.ravel()[asm.act_idx], 1.0 / col[:asm.n_y], rtol=1e-12)
        k = asm.n_y
        if prob.u_free:
            assert sc.Tu == pytest.approx(1.0 / col[k], rel=1e-12); k += 1
        if prob.v_free:
            assert sc.Tv == pytest.approx(1.0 / col[k], rel=1e-12)
        nb, ng = len(asm.band_idx), len(asm.gel_idx)
        np.testing.assert_allclose(sc.S_up.ravel()[asm.band_idx], 1.0 / row[:nb], rtol=1e-12)
        np.testing.assert_allclose(sc.S_up.ravel()[asm.gel_idx], 1.0 / row[nb:nb + ng], rtol=1e-12)
        np.testing.assert_allclose(sc.S_lo.ravel()[asm.gel_idx], 1.0 / row[nb + ng:], rtol=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_restarted_pdhg_reaches_the_lp_value(case):
    prob = tiny(case, seed=1)
    ref = lp.solve_highs(prob)
    r = pdhg.pdhg_restarted(prob, tol=1e-6, max_iters=40000)
    assert r.status == pdhg.OPTIMAL
    assert r.kkt.primal_obj == pytest.approx(ref.objective, rel=2e-5, abs=1e-8)
    assert prob.violation(r.state.y, r.state.u, r.state.v) < 1e-5


def test_plain_pdhg_approaches_the_lp_value():
    prob = tiny(lp.CASE1, seed=1)
    ref = lp.solve_highs(prob)
    r = pdhg.pdhg_plain(prob, iters=6000)
    assert r.kkt.primal_obj == pytest.approx(ref.objective, rel=2e-2)
    assert r.kkt.rel < 1e-2

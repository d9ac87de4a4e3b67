"""The solve at the benchmarked size (256^3 volume, 360 views, blur sigma 1.5, Case 1, FP32) checked
against the oracle: regions, active rays and the full relative KKT residuals of the returned state,
plus the sign and support structure every returned state has.  Degenerate LPs (empty band, empty
target) and the solve's argument checks are covered at small sizes."""
import numpy as np
import pytest
import torch

from oracle import lp as olp, kkt as okkt, blur as oblur
from oracle.geometry import make_geometry
from oracle.projector import Projector
from sipo_inputs import ellipsoids_target, ellipses_target, angles_uniform

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda", 0)


def test_full_size_solve_state_matches_oracle_kkt():
    import paper_2604_08997_amd as sipo
    n, na, sigma = 256, 360, (1.5, 1.5, 1.5)
    ang = angles_uniform(na)
    f = ellipsoids_target(n, 3000)
    plan = sipo.Plan(n, list(ang), nz=n, atten=1.0, sigma=sigma, dtype=torch.float32, device=dev())
    plan.autotune()
    lp = sipo.LP.build(plan, torch.as_tensor(f, dtype=torch.float32, device=dev()), sipo.CASE1, band_width=10.0,
                       f_min=1.0)
    # ten KKT checks of the restarted solver, in the configuration the benchmark times
    r = sipo.solve(lp, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=640, tol=1e-12, check_every=64))
    assert r["status_name"] == "iter_limit" and r["iters"] == 640
    y = lp.y.double().cpu().numpy()
    lu = lp.lam_up.double().cpu().numpy()
    ll = lp.lam_lo.double().cpu().numpy()
    lab = lp.labels.cpu().numpy()
    act = lp.act.cpu().numpy().astype(bool)
    del lp
    torch.cuda.empty_cache()
    op = olp.build(Projector(make_geometry(n, ang, nz=n, atten=1.0)), f, olp.CASE1, taps=oblur.psf_taps(sigma),
                   band_width=10.0)
    np.testing.assert_array_equal(lab, op.labels)
    np.testing.assert_array_equal(act, op.act)
    # structure of any returned state
    assert y.min() >= 0.0 and not y[~act].any()
    assert lu.min() >= 0.0 and ll.min() >= 0.0
    assert not lu[lab == 0].any() and not ll[lab != 2].any()
    # the residuals the solver reports are the oracle's residuals of the state it returns
    k = okkt.residuals(op, y, r["u"], r["v"], lu, ll)
    assert k.primal_obj == pytest.approx(r["primal_obj"], rel=1e-6)
    assert k.dual_obj == pytest.approx(r["dual_obj"], rel=1e-4, abs=1e-6)
    for got, want in ((r["rel_primal"], k.eps_p), (r["rel_dual"], k.eps_d), (r["rel_gap"], k.eps_gap)):
        assert got == pytest.approx(want, rel=2e-2, abs=1e-7), (got, want)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_empty_band_gives_zero_band_bound(dtype):
    # band width 0 without blur leaves no band voxels: Case 1 then has u* = 0 (u >= 0, no band rows)
    import paper_2604_08997_amd as sipo
    n, na = 24, 20
    f = ellipses_target(n, 51)
    plan = sipo.Plan(n, list(angles_uniform(na)), dtype=dtype, device=dev())
    lp = sipo.LP.build(plan, torch.as_tensor(f, dtype=dtype, device=dev()), sipo.CASE1, band_width=0.0, f_min=1.0)
    assert not bool((lp.labels == 1).any())
    op = olp.build(Projector(make_geometry(n, angles_uniform(na), atten=1.0)), f, olp.CASE1, band_width=0.0)
    ref = olp.solve_highs(op)
    assert ref.status == "optimal" and ref.objective == pytest.approx(0.0, abs=1e-12)
    r = sipo.solve(lp, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=50000,
                                         tol=1e-6 if dtype == torch.float64 else 2e-5))
    assert r["status_name"] == "optimal", r
    assert abs(r["u"]) <= 1e-6 and abs(r["primal_obj"]) <= 1e-6
    y = lp.y.double().cpu().numpy()
    assert op.violation(y, r["u"], r["v"]) <= 1e-4 * (1.0 + float(np.abs(op.hi).max()))


def test_empty_target_is_a_trivial_lp():
    # no gel, no band, no active ray: every case is solved by y = 0 with zero objective
    import paper_2604_08997_amd as sipo
    n, na = 16, 12
    plan = sipo.Plan(n, list(angles_uniform(na)), dtype=torch.float64, device=dev())
    f = torch.zeros(plan.vol_shape, dtype=torch.float64, device=dev())
    for case in (sipo.GENERAL, sipo.CASE1, sipo.CASE2):
        lp = sipo.LP.build(plan, f, case, band_width=3.0, f_min=1.0)
        assert not bool(lp.labels.any()) and not bool(lp.act.any())
        r = sipo.solve(lp, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=1000, tol=1e-8))
        assert r["status_name"] == "optimal", (case, r)
        assert r["primal_obj"] == pytest.approx(0.0, abs=1e-12)
        assert not bool(lp.y.any())


def test_solve_rejects_invalid_arguments_before_launching():
    import paper_2604_08997_amd as sipo
    from paper_2604_08997_amd import SipoError
    n, na = 16, 12
    f = ellipses_target(n, 52)
    p64 = sipo.Plan(n, list(angles_uniform(na)), dtype=torch.float64, device=dev())
    p32 = sipo.Plan(n, list(angles_uniform(na)), dtype=torch.float32, device=dev())
    a = sipo.LP.build(p64, torch.as_tensor(f, device=dev()), sipo.CASE1, band_width=2.0, f_min=1.0)
    b = sipo.LP.build(p32, torch.as_tensor(f, dtype=torch.float32, device=dev()), sipo.CASE1, band_width=2.0, f_min=1.0)
    y0 = a.y.clone()
    bad_opts = [dict(max_iters=0), dict(eta=1.0), dict(mode=7), dict(check_every=0), dict(scalar_weight=-1.0),
                dict(profile=1, use_graph=1), dict(progress_every=-1)]
    for kw in bad_opts:
        with pytest.raises(SipoError):
            sipo.solve(a, sipo.pdhg_options(**kw))
    with pytest.raises(SipoError):          # mixed precisions in one batch
        sipo.solve([a, b])
    a.w1 = -1.0
    with pytest.raises(SipoError):          # negative objective weight
        sipo.solve(a)
    assert torch.equal(a.y, y0)             # nothing ran


def test_progress_lines_report_the_checks(capfd):
    # progress_every = 2: one line per unfinished instance at every second KKT check (64 iterations apart)
    import paper_2604_08997_amd as sipo
    n, na = 16, 12
    f = ellipses_target(n, 53)
    plan = sipo.Plan(n, list(angles_uniform(na)), dtype=torch.float64, device=dev())
    lps = [sipo.LP.build(plan, torch.as_tensor(f, device=dev()), sipo.CASE1, band_width=2.0, f_min=1.0)
           for _ in range(2)]
    r = sipo.solve(lps, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=512, tol=1e-14, check_every=64,
                                          progress_every=2))
    assert [x["iters"] for x in r] == [512, 512]
    lines = [ln for ln in capfd.readouterr().err.splitlines() if ln.startswith("[sipo] instance")]
    assert len(lines) == 2 * 4
    for k, ln in enumerate(lines):
        assert ln.startswith(f"[sipo] instance {k % 2}: iteration {128 * (k // 2 + 1)}, relative KKT ")

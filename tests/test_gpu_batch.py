"""Batched PDHG solves of uneven instances: one set of launches for all instances.

A batch must give every instance what a solve of that instance alone gives:
same arithmetic per instance (identical segment partition and reduction
order), so plain-mode iterates agree to the last bit, and restarted solves
reach the oracle's LP value or certify infeasibility per instance.
"""
import numpy as np
import pytest
import torch

from oracle import lp as olp, kkt as okkt
from oracle.geometry import make_geometry
from oracle.projector import Projector
from sipo_inputs import ellipses_target, ellipsoids_target, angles_uniform

pytestmark = pytest.mark.gpu

# (n, views, case, seed): uneven grids, view counts (odd ones unpaired) and LP cases
SMALL = [(20, 12, 1, 31), (28, 24, 2, 32), (36, 18, 0, 33), (24, 15, 1, 34), (32, 30, 2, 35)]


def dev():
    return torch.device("cuda", 0)


def build(spec, dtype, band=3.0):
    import paper_2604_08997_amd as sipo
    n, na, case, seed = spec
    f = ellipses_target(n, seed)
    kw = {"cap": 0.9} if case == 2 else {}
    plan = sipo.Plan(n, list(angles_uniform(na)), dtype=dtype, device=dev())
    lp = sipo.LP.build(plan, torch.as_tensor(f, dtype=dtype, device=dev()), case, band_width=band, f_min=1.0, **kw)
    op = olp.build(Projector(make_geometry(n, angles_uniform(na), atten=1.0)), f, case, band_width=band, **kw)
    return lp, op


def state(lp):
    return [t.double().cpu().numpy().copy() for t in (lp.y, lp.lam_up, lp.lam_lo)]


def test_plain_fp64_batch_equals_individual_solves():
    import paper_2604_08997_amd as sipo
    opts = sipo.pdhg_options(mode=sipo.PLAIN, max_iters=300, power_iters=50)
    alone = []
    for spec in SMALL:
        lp, _ = build(spec, torch.float64)
        r = sipo.solve(lp, opts)
        alone.append((r, state(lp)))
    lps = [build(spec, torch.float64)[0] for spec in SMALL]
    res = sipo.solve(lps, opts)
    for (ra, sa), rb, lp in zip(alone, res, lps):
        assert rb["tau"] == ra["tau"]
        for a, b in zip(sa, state(lp)):
            np.testing.assert_array_equal(a, b)
        assert rb["primal_obj"] == ra["primal_obj"] and rb["rel_dual"] == ra["rel_dual"]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_restarted_batch_reaches_each_lp_value(dtype):
    import paper_2604_08997_amd as sipo
    built = [build(spec, dtype) for spec in SMALL]
    tol = 1e-6 if dtype == torch.float64 else 1e-5
    res = sipo.solve([b[0] for b in built], sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=100000, tol=tol))
    for (lp, op), r, spec in zip(built, res, SMALL):
        ref = olp.solve_highs(op)
        if ref.status == "infeasible":
            assert r["status_name"] == "infeasible", (spec, r)
            _, lu, ll = state(lp)
            assert okkt.farkas_check(op, lu, ll, tol=1e-6 if dtype == torch.float64 else 1e-4)["valid"], spec
            continue
        assert r["status_name"] == "optimal", (spec, r)
        assert abs(r["primal_obj"] - ref.objective) <= 1e-4 * (1 + abs(ref.objective)), (spec, r, ref.objective)
        y, lu, ll = state(lp)
        assert okkt.residuals(op, y, r["u"], r["v"], lu, ll).rel <= 5 * tol, spec
        # max constraint violation in normalised dose units
        assert op.violation(y, r["u"], r["v"]) <= 1e-4, spec


def test_batch_with_an_infeasible_instance_certifies_it_and_solves_the_rest():
    import paper_2604_08997_amd as sipo
    import paper_2604_08997_amd.binding as B
    good = [build(spec, torch.float64) for spec in SMALL[:2]]
    n, na = 24, 30
    f = ellipses_target(n, 2)
    plan = sipo.Plan(n, list(angles_uniform(na)), dtype=torch.float64, device=dev())
    bad = sipo.LP.build(plan, torch.as_tensor(f, device=dev()), sipo.CASE1, band_width=3.0, f_min=1.0,
                        tol_lo=1.0, tol_hi=0.95)
    op_bad = olp.build(Projector(make_geometry(n, angles_uniform(na), atten=1.0)), f, olp.CASE1, band_width=3.0,
                       tol_lo=1.0, tol_hi=0.95)
    assert olp.solve_highs(op_bad).status == "infeasible"
    res = sipo.solve([good[0][0], bad, good[1][0]],
                     sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=60000, tol=1e-6, infeas_tol=1e-7))
    assert res[1]["status_name"] == "infeasible"
    _, lu, ll = state(bad)
    assert okkt.farkas_check(op_bad, lu, ll, tol=1e-6)["valid"]
    for (lp, op), r in zip(good, (res[0], res[2])):
        ref = olp.solve_highs(op)
        if ref.status == "optimal":
            assert r["status_name"] == "optimal"
            assert abs(r["primal_obj"] - ref.objective) <= 1e-4 * (1 + abs(ref.objective))
    assert B.STATUS_NAMES[B.PRIMAL_INFEASIBLE] == "infeasible"


def test_graph_captured_batch_matches_eager_batch():
    import paper_2604_08997_amd as sipo
    s = torch.cuda.Stream()
    out = []
    for use_graph in (0, 1):
        lps = [build(spec, torch.float32)[0] for spec in SMALL]
        with torch.cuda.stream(s):
            res = sipo.solve(lps, sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=5000, tol=1e-5,
                                                    use_graph=use_graph))
        s.synchronize()
        out.append((res, [state(lp) for lp in lps]))
    (ra, sa), (rb, sb) = out
    for a, b in zip(ra, rb):
        assert (a["status"], a["iters"], a["restarts"]) == (b["status"], b["iters"], b["restarts"])
        assert a["primal_obj"] == b["primal_obj"]
    for x, y in zip(sa, sb):
        for a, b in zip(x, y):
            np.testing.assert_array_equal(a, b)


def test_mixed_3d_and_2d_batch_equals_individual_solves():
    # a blurred 3D instance (plan operators, internal layouts) next to 2D instances
    import paper_2604_08997_amd as sipo
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=640, tol=1e-12, check_every=64)

    def make():
        n, na, sigma = 16, 12, (1.0, 1.0, 1.0)
        f3 = ellipsoids_target(n, 5, count=2)
        p3 = sipo.Plan(n, list(angles_uniform(na)), nz=f3.shape[0], sigma=sigma, dtype=torch.float64, device=dev())
        l3 = sipo.LP.build(p3, torch.as_tensor(f3, device=dev()), sipo.CASE1, band_width=2.0, f_min=1.0)
        return [l3] + [build(spec, torch.float64)[0] for spec in SMALL[:2]]

    alone = []
    for lp in make():
        r = sipo.solve(lp, opts)
        alone.append((r, state(lp)))
    lps = make()
    res = sipo.solve(lps, opts)
    for (ra, sa), rb, lp in zip(alone, res, lps):
        assert (ra["status"], ra["iters"], ra["restarts"]) == (rb["status"], rb["iters"], rb["restarts"])
        for a, b in zip(sa, state(lp)):
            np.testing.assert_array_equal(a, b)


def test_fp32_3d_instances_after_a_2d_one_equal_individual_solves():
    # two blurred FP32 3D instances of different ragged sizes behind a 2D one, so every per-instance
    # field of the masked 3D path (projector input, blur and transpose flags, live segments, the
    # primal step fused into the projector) sits at a nonzero offset of the batch workspace
    import paper_2604_08997_amd as sipo
    opts = sipo.pdhg_options(mode=sipo.RESTARTED, max_iters=640, tol=1e-12, check_every=64)

    def make():
        out = [build(SMALL[0], torch.float32)[0]]
        for n, na, nz, seed in ((24, 16, 12, 9), (40, 18, 20, 31)):
            f3 = ellipsoids_target(n, seed, count=2, nz=nz)
            p3 = sipo.Plan(n, list(angles_uniform(na)), nz=nz, sigma=(1.0, 1.0, 1.5), dtype=torch.float32,
                           device=dev())
            out.append(sipo.LP.build(p3, torch.as_tensor(f3, dtype=torch.float32, device=dev()), sipo.CASE1,
                                     band_width=2.0, f_min=1.0))
        return out

    alone = []
    for lp in make():
        r = sipo.solve(lp, opts)
        alone.append((r, state(lp)))
    lps = make()
    res = sipo.solve(lps, opts)
    for (ra, sa), rb, lp in zip(alone, res, lps):
        assert (ra["status"], ra["iters"], ra["restarts"]) == (rb["status"], rb["iters"], rb["restarts"])
        assert ra["primal_obj"] == rb["primal_obj"]
        for a, b in zip(sa, state(lp)):
            np.testing.assert_array_equal(a, b)

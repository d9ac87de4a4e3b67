"""Pins of the oracle parts whose earlier tests could not catch a plausible mistake.

Each pin is a check function applied to the oracle as it stands (it must hold) and to
planted variants with one typical mistake each (it must fail).  The expected values come
from the paper's formulas evaluated by hand, or from brute-force loops, never from the
function under test:

* the Richards response M (Eq. 4) and its inverse (Eq. 5): values at f0 and at
  f0 + ln 3 / beta, the two asymptotes, and the slope at f0;
* the active-ray rule of Sec. 2.2 (rays with P f_T above 1e-6 of its maximum), against
  ray sums from the ray-first brute-force entries, on a field built so that the
  "!= 0" reading, a 1e-3 threshold and P K f_T (blur before projecting) all differ;
* plain PDHG (Chambolle-Pock, primal first, theta = 1): three iterations stepped by hand
  on a 2 x 2 grid with one view, where the LP has the variables y0, y1 (masked) and u.
"""
import math

import numpy as np
import pytest

from oracle import blur, lp, metrics, pdhg, regions
from oracle.geometry import make_geometry
from oracle.projector import Projector, brute_force_entries
from sipo_inputs import ellipses_target


# ----------------------------------------------------------------- Richards (Eq. 4-5)
RES = dict(a=0.1, k=0.9, beta=4.0, gamma=2.0, f0=0.5)


def richards_pin_holds(M) -> bool:
    a, k, beta, gamma, f0 = RES["a"], RES["k"], RES["beta"], RES["gamma"], RES["f0"]
    ok = True
    # at f = f0 the bracket is 1 + e^0 = 2: M = a + (k - a) 2^(-1/gamma) = 0.1 + 0.8 / sqrt(2)
    ok &= abs(M(f0, **RES) - 0.6656854249492381) < 1e-12
    # at f = f0 + ln 3 / beta the bracket is 1 + 1/3 = 4/3: M = 0.1 + 0.8 (3/4)^(1/2)
    ok &= abs(M(f0 + math.log(3.0) / beta, **RES) - 0.7928203230275509) < 1e-12
    # asymptotes: a below, k above
    ok &= abs(M(f0 - 40.0, **RES) - a) < 1e-12 and abs(M(f0 + 40.0, **RES) - k) < 1e-12
    # slope at f0: (k - a) (beta / gamma) e^0 2^(-1/gamma - 1) = 0.8 * 2 * 2^(-1.5)
    h = 1e-6
    slope = (M(f0 + h, **RES) - M(f0 - h, **RES)) / (2 * h)
    ok &= abs(slope - 0.565685424949238) < 1e-7
    # gamma = 1 is the plain logistic: M(f0 + ln 3 / beta) = a + 3/4 (k - a)
    p1 = dict(RES, gamma=1.0)
    ok &= abs(M(f0 + math.log(3.0) / beta, **p1) - 0.7) < 1e-12
    return bool(ok)


def richards_inverse_pin_holds(Minv) -> bool:
    beta, f0 = RES["beta"], RES["f0"]
    ok = abs(Minv(0.6656854249492381, **RES) - f0) < 1e-12
    ok &= abs(Minv(0.7928203230275509, **RES) - (f0 + math.log(3.0) / beta)) < 1e-12
    ok &= abs(Minv(0.7, **dict(RES, gamma=1.0)) - (f0 + math.log(3.0) / beta)) < 1e-12
    return bool(ok)


def test_richards_matches_eq4_hand_values():
    assert richards_pin_holds(metrics.richards)
    assert richards_inverse_pin_holds(metrics.richards_inverse)


def test_richards_pins_catch_planted_mistakes():
    def exp_gamma(f, a, k, beta, gamma, f0):           # exponent gamma instead of 1/gamma
        return a + (k - a) / (1.0 + np.exp(-beta * (f - f0))) ** gamma

    def sign_beta(f, a, k, beta, gamma, f0):           # growth-rate sign flipped
        return a + (k - a) / (1.0 + np.exp(beta * (f - f0))) ** (1.0 / gamma)

    def swapped(f, a, k, beta, gamma, f0):             # asymptotes swapped
        return k + (a - k) / (1.0 + np.exp(-beta * (f - f0))) ** (1.0 / gamma)

    for bad in (exp_gamma, sign_beta, swapped):
        assert not richards_pin_holds(bad), bad.__name__

    def inv_exp(m, a, k, beta, gamma, f0):             # 1/gamma in the inverse
        return f0 - np.log(((k - a) / (m - a)) ** (1.0 / gamma) - 1.0) / beta

    def inv_sign(m, a, k, beta, gamma, f0):
        return f0 + np.log(((k - a) / (m - a)) ** gamma - 1.0) / beta

    for bad in (inv_exp, inv_sign):
        assert not richards_inverse_pin_holds(bad), bad.__name__


# ------------------------------------------------------------ active rays (Sec. 2.2)
def brute_force_ray_sums(g, f):
    """P f by the ray-first entry loops, slice by slice (P_3D = I_z (x) P_2D)."""
    ent = brute_force_entries(g)
    out = np.zeros(g.sino_shape)
    for (i, a, b), w in ent.items():
        r, c = divmod(i, g.n)
        for z in range(g.nz):
            out[a, z, b] += w * f[z, r, c]
    return out


def graded_field():
    """2D field whose rays fall in all three classes: one voxel at 1, one at 1e-4 and one at
    1e-9.  Rays meeting only the 1e-4 voxel lie between 1e-6 and 1e-3 of the maximum; rays
    meeting only the 1e-9 voxel lie above zero but below 1e-6 of it."""
    f = np.zeros((1, 8, 8))
    f[0, 3, 3] = 1.0
    f[0, 5, 2] = 1e-4
    f[0, 2, 6] = 1e-9
    return f


def active_pin_holds(active_fn) -> bool:
    g = make_geometry(8, 12, atten=1.0)
    P = Projector(g)
    f = graded_field()
    ref = brute_force_ray_sums(g, f)
    m = ref.max()
    want = ref > 1e-6 * m
    # the field separates the readings: some rays in (1e-6, 1e-3] m, some in (0, 1e-6] m
    assert ((ref > 1e-6 * m) & (ref <= 1e-3 * m)).any()
    assert ((ref > 0) & (ref <= 1e-6 * m)).any()
    got = active_fn(P, f)
    return bool(got.shape == want.shape and (got == want).all())


def active_pin_3d_holds(build) -> bool:
    """In 3D with a blur PSF the mask uses P f_T, not P K f_T (Sec. 2.2): a target confined to
    one slice leaves every other slice without an active ray, although K f_T reaches them."""
    g = make_geometry(8, 6, nz=5, atten=1.0)
    P = Projector(g)
    f = np.zeros((5, 8, 8))
    f[2] = ellipses_target(8, 4)[0]
    assert f[2].any()
    taps = blur.psf_taps((1.0, 1.0, 1.0))
    act = build(P, f, lp.CASE1, taps=taps, band_width=2.0).act
    ref = brute_force_ray_sums(g, f)
    want = ref > 1e-6 * ref.max()
    assert not want[:, [0, 1, 3, 4], :].any()
    return bool((act == want).all())


def test_active_rays_match_brute_force_threshold():
    assert active_pin_holds(regions.active_rays)
    assert active_pin_3d_holds(lp.build)


def test_active_ray_pins_catch_planted_mistakes(monkeypatch):
    def nonzero(P, f):                                  # the literal "!= 0" reading
        return P.project(f) > 0.0

    def loose(P, f):                                    # threshold 1e-3 instead of 1e-6
        pf = P.project(f)
        return pf > 1e-3 * pf.max()

    for bad in (nonzero, loose):
        assert not active_pin_holds(bad), bad.__name__

    taps = blur.psf_taps((1.0, 1.0, 1.0))
    real = regions.active_rays

    def blurred(P, f):                                  # P K f_T instead of P f_T
        return real(P, blur.apply(f, taps))
    monkeypatch.setattr(lp._regions, "active_rays", blurred)
    assert not active_pin_3d_holds(lp.build)


# ----------------------------------------------------- plain PDHG, stepped by hand
TAU, SIGMA = 0.3, 0.2


def two_by_two_case1():
    """2 x 2 grid, one view at theta = 0, no attenuation.  Voxel rows sit at y = -1/2 and 1/2, so
    u = y + 1/2 lands exactly on bins 0 and 1 with weight 1: D(r, c) = y_r.  Target = voxel (0, 0)
    (gel); band width 1 makes (0, 1) and (1, 0) band; bin 1 sees no target and is masked.  Case 1
    (L = 1, U = 1/0.9, v = 1) with w1 lowered to 0.01 so that u moves within three steps."""
    g = make_geometry(2, [0.0], atten=0.0)
    f = np.zeros((1, 2, 2))
    f[0, 0, 0] = 1.0
    prob = lp.build(Projector(g), f, lp.CASE1, band_width=1.0)
    prob.w1 = 0.01
    assert prob.labels.tolist() == [[[2, 1], [1, 0]]]
    assert prob.act[:, 0, :].tolist() == [[True, False]]
    return prob


# State after iterations 1..3, by hand (module docstring of oracle.pdhg for the step):
#  it 1: q = 0, y0 = 0, u = max(0, -0.3 * 0.01) = 0, D = 0, lambda3 = sigma (L - 0) = 0.2.
#  it 2: z(gel) = -0.2, q(bin 0) = -0.2, y0 = 0.3 * 0.2 = 0.06, u = 0; D(row 0) = 0.06,
#        Dbar = 0.12; lambda1(0, 1) = 0.2 * 0.12 = 0.024; lambda2 = max(0, 0.2 (0.12 - 1/0.9)) = 0;
#        lambda3 = 0.2 + 0.2 (1 - 0.12) = 0.376.
#  it 3: q(bin 0) = 0.024 - 0.376 = -0.352, y0 = 0.06 + 0.3 * 0.352 = 0.1656;
#        u = max(0, -0.3 (0.01 - 0.024)) = 0.0042, ubar = 0.0084; Dbar = 2 * 0.1656 - 0.06 = 0.2712;
#        lambda1(0, 1) = 0.024 + 0.2 (0.2712 - 0.0084) = 0.07656, lambda1(1, 0) = 0;
#        lambda2 = 0; lambda3 = 0.376 + 0.2 (1 - 0.2712) = 0.52176.
HAND = {
    1: dict(y0=0.0, u=0.0, l1=(0.0, 0.0), l2=0.0, l3=0.2),
    2: dict(y0=0.06, u=0.0, l1=(0.024, 0.0), l2=0.0, l3=0.376),
    3: dict(y0=0.1656, u=0.0042, l1=(0.07656, 0.0), l2=0.0, l3=0.52176),
}


def plain_pin_holds(run) -> bool:
    prob = two_by_two_case1()
    for k, h in HAND.items():
        st = run(prob, k)
        got = [st.y[0, 0, 0], st.y[0, 0, 1], st.u, st.lam_up[0, 0, 1], st.lam_up[0, 1, 0],
               st.lam_up[0, 0, 0], st.lam_lo[0, 0, 0]]
        want = [h["y0"], 0.0, h["u"], h["l1"][0], h["l1"][1], h["l2"], h["l3"]]
        if not np.allclose(got, want, rtol=0, atol=1e-14):
            return False
    return True


def oracle_run(prob, k):
    return pdhg.pdhg_plain(prob, iters=k, tau=TAU, sigma=SIGMA).state


def test_plain_pdhg_matches_three_hand_steps():
    assert plain_pin_holds(oracle_run)


def _dual_update(prob, st, D_new, ubar, tau_lam):
    band, gel = prob.band, prob.gel
    Dbar = 2.0 * D_new - st.D
    lu, ll = st.lam_up.copy(), st.lam_lo.copy()
    lu[band] = np.maximum(0.0, lu[band] + tau_lam * (Dbar[band] - ubar))
    lu[gel] = np.maximum(0.0, lu[gel] + tau_lam * (Dbar[gel] - prob.hi[gel]))
    ll[gel] = np.maximum(0.0, ll[gel] + tau_lam * (prob.lo[gel] - Dbar[gel]))
    return lu, ll


def test_plain_pdhg_pin_catches_planted_mistakes():
    from oracle import kkt

    def dual_first(prob, k):
        # dual step on the current dose first, then the primal step with the new multipliers
        st = pdhg.initial_state(prob)
        for _ in range(k):
            band = prob.band
            lu = st.lam_up.copy(); ll = st.lam_lo.copy()
            lu[band] = np.maximum(0.0, lu[band] + SIGMA * (st.D[band] - st.u))
            lu[prob.gel] = np.maximum(0.0, lu[prob.gel] + SIGMA * (st.D[prob.gel] - prob.hi[prob.gel]))
            ll[prob.gel] = np.maximum(0.0, ll[prob.gel] + SIGMA * (prob.lo[prob.gel] - st.D[prob.gel]))
            q = prob.adjoint(kkt.z_of(prob, lu, ll))
            y = np.where(prob.act, np.maximum(0.0, st.y - TAU * q), 0.0)
            u = max(0.0, st.u - TAU * (prob.w1 - float(lu[band].sum())))
            st = pdhg.State(y, u, 1.0, lu, ll, prob.dose(y))
        return st

    def no_extrapolation(prob, k):
        # dual step on D+ instead of 2 D+ - D
        st = pdhg.initial_state(prob)
        for _ in range(k):
            q = prob.adjoint(kkt.z_of(prob, st.lam_up, st.lam_lo))
            y = np.where(prob.act, np.maximum(0.0, st.y - TAU * q), 0.0)
            u = max(0.0, st.u - TAU * (prob.w1 - float(st.lam_up[prob.band].sum())))
            D = prob.dose(y)
            half = pdhg.State(st.y, st.u, 1.0, st.lam_up, st.lam_lo, D)   # so that 2D - D = D
            lu, ll = _dual_update(prob, half, D, 2.0 * u - st.u, SIGMA)
            st = pdhg.State(y, u, 1.0, lu, ll, D)
        return st

    def scalar_not_extrapolated(prob, k):
        # ubar = u+ instead of 2 u+ - u
        st = pdhg.initial_state(prob)
        for _ in range(k):
            q = prob.adjoint(kkt.z_of(prob, st.lam_up, st.lam_lo))
            y = np.where(prob.act, np.maximum(0.0, st.y - TAU * q), 0.0)
            u = max(0.0, st.u - TAU * (prob.w1 - float(st.lam_up[prob.band].sum())))
            D = prob.dose(y)
            lu, ll = _dual_update(prob, st, D, u, SIGMA)
            st = pdhg.State(y, u, 1.0, lu, ll, D)
        return st

    def ascent_sign(prob, k):
        # y + tau q instead of y - tau q
        st = pdhg.initial_state(prob)
        for _ in range(k):
            q = prob.adjoint(kkt.z_of(prob, st.lam_up, st.lam_lo))
            y = np.where(prob.act, np.maximum(0.0, st.y + TAU * q), 0.0)
            u = max(0.0, st.u - TAU * (prob.w1 - float(st.lam_up[prob.band].sum())))
            D = prob.dose(y)
            lu, ll = _dual_update(prob, st, D, 2.0 * u - st.u, SIGMA)
            st = pdhg.State(y, u, 1.0, lu, ll, D)
        return st

    def correct(prob, k):
        # the same hand-written loop without a mistake passes, so the variants fail for their
        # mistake alone
        st = pdhg.initial_state(prob)
        for _ in range(k):
            q = prob.adjoint(kkt.z_of(prob, st.lam_up, st.lam_lo))
            y = np.where(prob.act, np.maximum(0.0, st.y - TAU * q), 0.0)
            u = max(0.0, st.u - TAU * (prob.w1 - float(st.lam_up[prob.band].sum())))
            D = prob.dose(y)
            lu, ll = _dual_update(prob, st, D, 2.0 * u - st.u, SIGMA)
            st = pdhg.State(y, u, 1.0, lu, ll, D)
        return st

    assert plain_pin_holds(correct)
    for bad in (dual_first, no_extrapolation, scalar_not_extrapolated, ascent_sign):
        assert not plain_pin_holds(bad), bad.__name__

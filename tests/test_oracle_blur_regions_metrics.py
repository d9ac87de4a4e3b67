"""Pins for the oracle blur K, the region partition and the metrics."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage
from scipy.optimize import minimize_scalar

from oracle import blur, regions, metrics
from oracle.geometry import make_geometry, in_vial
from oracle.projector import Projector
from sipo_inputs import uniform_field, ellipses_target, ellipsoids_target

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def test_blur_matches_scipy_convolve_with_explicit_3d_kernel():
    taps = blur.psf_taps((1.0, 1.5, 2.0))
    vol = uniform_field((9, 10, 11), 7)
    k3 = taps[2][:, None, None] * taps[1][None, :, None] * taps[0][None, None, :]
    want = ndimage.convolve(vol, k3, mode="constant", cval=0.0)
    np.testing.assert_allclose(blur.apply(vol, taps), want, rtol=1e-13, atol=1e-15)


def test_blur_is_symmetric_and_unit_sum_inside():
    taps = blur.psf_taps((1.5, 1.5, 1.5))
    a = uniform_field((12, 13, 14), 1)
    b = uniform_field((12, 13, 14), 2)
    lhs = (blur.apply(a, taps) * b).sum()
    rhs = (a * blur.apply(b, taps)).sum()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    one = blur.apply(np.ones((12, 13, 14)), taps)
    np.testing.assert_allclose(one[3:-3, 3:-3, 3:-3], 1.0, rtol=1e-14)


def test_psf_support_matches_paper_set_up():
    facts = json.load(open(GOLDEN))["psf"]
    t = blur.gaussian_taps(facts["sigma"])
    assert len(t) == facts["populated_taps_per_axis"]
    assert abs(t.sum() - 1.0) < 1e-15
    assert len(blur.gaussian_taps(1.5)) == 7 and len(blur.gaussian_taps(2.0)) == 9
    # the populated part sits inside the paper's larger kernel box
    assert len(t) <= facts["kernel_size"]


@pytest.mark.parametrize("w", [0.0, 1.0, 2.5, 3.0])
def test_band_partition_matches_brute_force_2d(w):
    f = ellipses_target(20, 17)
    np.testing.assert_array_equal(regions.labels(f, band_width=w), regions.labels_brute_force(f, w))


def test_band_partition_matches_brute_force_3d():
    f = ellipsoids_target(10, 4, count=2, nz=8)
    np.testing.assert_array_equal(regions.labels(f, band_width=2.0), regions.labels_brute_force(f, 2.0))


def test_band_free_and_blur_support():
    f = ellipses_target(24, 3)
    lab = regions.labels(f, band_width=np.inf)
    vial = in_vial(24)[None]
    assert ((lab == regions.BAND) == ((f == 0) & vial)).all()
    # w = 0 and K != I: band is exactly the box dilation of gel minus gel
    taps = blur.psf_taps((1.0, 1.0, 1.0))
    f3 = ellipsoids_target(12, 9, count=2, nz=12)
    lab3 = regions.labels(f3, band_width=0.0, taps=taps)
    gel = f3 != 0
    dil = ndimage.binary_dilation(gel, structure=np.ones((5, 5, 5), bool))
    want = dil & ~gel & np.broadcast_to(in_vial(12), f3.shape)
    assert ((lab3 == regions.BAND) == want).all()


def test_every_gel_voxel_keeps_an_active_ray_in_every_view():
    n = 32
    g = make_geometry(n, 24)
    P = Projector(g)
    f = ellipses_target(n, 5)
    act = regions.active_rays(P, f)
    PT = P.PT.tocsr()
    gel_idx = np.nonzero(f.ravel() != 0)[0]
    for i in gel_idx:
        row = PT.getrow(i).toarray().ravel().reshape(g.n_angles, g.n_bins)
        for a in range(g.n_angles):
            b = int(np.argmax(row[a]))
            assert act[a, 0, b]


def test_metrics_scale_invariance_and_hand_example():
    lab = np.array([[[2, 2, 2, 1, 0]]], dtype=np.uint8)
    D = np.array([[[1.0, 2.0, 1.5, 0.5, 9.0]]])
    ft = np.ones_like(D)
    assert metrics.dtvr(D, ft, lab) == pytest.approx(2.0)
    assert metrics.dsr(D, ft, lab) == pytest.approx(0.5)
    assert metrics.psr(D, lab) == pytest.approx(2.0)
    rng = np.random.default_rng(0)
    D = rng.uniform(0.2, 2.0, size=(1, 6, 6))
    lab = rng.integers(0, 3, size=(1, 6, 6)).astype(np.uint8)
    lab[0, 0, 0], lab[0, 0, 1] = 2, 1
    ft = rng.uniform(0.5, 1.5, size=D.shape)
    base = (metrics.dtvr(D, ft, lab), metrics.dsr(D, ft, lab), metrics.psr(D, lab))
    for c in (1e-3, 1.0, 7.5, 1e3):
        got = (metrics.dtvr(c * D, ft, lab), metrics.dsr(c * D, ft, lab), metrics.psr(c * D, lab))
        np.testing.assert_allclose(got, base, rtol=1e-12)


def test_alpha_star_is_the_least_squares_minimiser_and_case2_downscales():
    rng = np.random.default_rng(3)
    lab = np.full((1, 5, 5), 2, dtype=np.uint8)
    ft = rng.uniform(0.5, 1.0, size=lab.shape)
    fn = ft / 0.7 * rng.uniform(1.0, 1.2, size=lab.shape)   # normalised dose >= f~_T (Case 2)
    w = rng.uniform(0.1, 1.0, size=lab.shape)
    a = metrics.alpha_star(fn, ft, lab, w)
    phi = lambda al: float((w * (al * fn - ft) ** 2).sum())
    best = minimize_scalar(phi, bounds=(0.0, 5.0), method="bounded", options={"xatol": 1e-12})
    assert a == pytest.approx(best.x, rel=1e-7)
    assert a <= 0.7 + 1e-15             # alpha* <= f_crit when f~* >= f~_T


def test_richards_inverse_round_trip():
    p = dict(a=0.05, k=0.95, beta=8.0, gamma=0.7, f0=0.5)
    m = np.linspace(0.1, 0.9, 17)
    np.testing.assert_allclose(metrics.richards(metrics.richards_inverse(m, **p), **p), m, rtol=1e-12)


def test_alpha_m_recovers_the_generating_scale_and_beats_a_dense_scan():
    # Eq. 28: when m_T is exactly M(alpha0 f~*) on the gel, the calibration returns alpha0
    resin = (0.02, 0.98, 6.0, 0.8, 1.1)
    rng = np.random.default_rng(11)
    lab = rng.integers(0, 3, size=(2, 6, 6)).astype(np.uint8)
    lab[0, 0, 0] = 2
    fn = rng.uniform(0.8, 1.3, size=lab.shape)
    alpha0 = 1.37
    mt = metrics.richards(alpha0 * fn, *resin)
    assert metrics.alpha_m(fn, mt, lab, resin) == pytest.approx(alpha0, rel=1e-8)
    # perturbed targets: no alpha on a dense scan does better (brute force)
    mt2 = mt * rng.uniform(0.95, 1.05, size=mt.shape)
    w = rng.uniform(0.2, 1.0, size=lab.shape)
    am = metrics.alpha_m(fn, mt2, lab, resin, w)
    f_best = metrics.phi_m(am, fn, mt2, lab, resin, w)
    scan = [metrics.phi_m(a, fn, mt2, lab, resin, w) for a in np.linspace(0.5, 3.0, 5001)]
    assert f_best <= min(scan) + 1e-12
    # DTVR_m of the generating dose is exactly 1
    assert metrics.dtvr_m(alpha0 * fn, mt, lab, resin) == pytest.approx(1.0, abs=1e-12)

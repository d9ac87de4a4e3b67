"""GPU response map, metrics and post-scaling (Eq. 4-8, 25-28, 46) against the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import metrics as om

pytestmark = pytest.mark.gpu

# synthetic resin constants (the paper prints none): lower/upper asymptote, rate, shape, location
RESIN = (0.02, 0.98, 6.0, 0.8, 1.1)


def dev():
    return torch.device("cuda", 0)


def plan(dtype, n=40, nz=3):
    import paper_2604_08997_amd as sipo
    return sipo.Plan(n, 8, nz=nz, dtype=dtype, device=dev())


def data(p, seed):
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 3, size=p.vol_shape).astype(np.uint8)
    D = rng.uniform(0.6, 1.6, size=p.vol_shape)
    ftn = rng.uniform(0.9, 1.2, size=p.vol_shape)
    w = rng.uniform(0.2, 1.0, size=p.vol_shape)
    return lab, D, ftn, w


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_response_and_inverse(dtype):
    p = plan(dtype)
    rng = np.random.default_rng(1)
    f = rng.uniform(0.0, 2.5, size=p.vol_shape)
    t = torch.as_tensor(f, dtype=dtype, device=dev())
    m = p.response(t, RESIN).double().cpu().numpy()
    want = om.richards(torch.as_tensor(f, dtype=dtype).double().numpy(), *RESIN)
    tol = 1e-13 if dtype == torch.float64 else 1e-6
    np.testing.assert_allclose(m, want, rtol=tol, atol=tol)
    mm = np.clip(want, 0.05, 0.95)
    back = p.response(torch.as_tensor(mm, dtype=dtype, device=dev()), RESIN, inverse=True).double().cpu().numpy()
    np.testing.assert_allclose(back, om.richards_inverse(torch.as_tensor(mm, dtype=dtype).double().numpy(), *RESIN),
                               rtol=10 * tol, atol=10 * tol)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_metrics_and_post_scaling_match_oracle(dtype):
    p = plan(dtype)
    lab, D, ftn, w = data(p, 2)
    # values as the device holds them
    Dd, fd, wd = (torch.as_tensor(a, dtype=dtype, device=dev()) for a in (D, ftn, w))
    D, ftn, w = (a.double().cpu().numpy() for a in (Dd, fd, wd))
    f_crit = 0.8
    m_t = om.richards(1.3 * D, *RESIN) * np.random.default_rng(3).uniform(0.97, 1.03, size=D.shape)
    md = torch.as_tensor(m_t, dtype=dtype, device=dev())
    m_t = md.double().cpu().numpy()
    r = p.evaluate(Dd, torch.as_tensor(lab, device=dev()), fd, f_crit=f_crit, weights=wd, resin=RESIN, m_target=md)
    assert r["dtvr"] == pytest.approx(om.dtvr(D, ftn, lab), rel=1e-13)
    assert r["dsr"] == pytest.approx(om.dsr(D, ftn, lab), rel=1e-13)
    assert r["psr_f"] == pytest.approx(om.psr(D, lab), rel=1e-13)
    assert r["alpha_f"] == pytest.approx(om.alpha_star(D, f_crit * ftn, lab, w), rel=1e-11)
    am = om.alpha_m(D, m_t, lab, RESIN, w)
    assert r["alpha_m"] == pytest.approx(am, rel=1e-6)
    # objective at the GPU's alpha is as good as the oracle's (to rounding)
    assert om.phi_m(r["alpha_m"], D, m_t, lab, RESIN, w) <= om.phi_m(am, D, m_t, lab, RESIN, w) * (1 + 1e-9)
    assert r["psr_m"] == pytest.approx(om.psr(om.richards(r["alpha_m"] * D, *RESIN), lab), rel=1e-10)
    assert r["dtvr_m"] == pytest.approx(om.dtvr_m(r["alpha_m"] * D, m_t, lab, RESIN), rel=1e-10)
    assert r["n_gel"] == int((lab == 2).sum()) and r["n_band"] == int((lab == 1).sum())


def test_empty_band_and_zero_gel_minimum():
    p = plan(torch.float64, n=16, nz=1)
    lab = np.zeros(p.vol_shape, dtype=np.uint8)
    lab[0, 5:9, 5:9] = 2
    D = np.ones(p.vol_shape)
    r = p.evaluate(torch.as_tensor(D, device=dev()), torch.as_tensor(lab, device=dev()), None, f_t_scalar=1.0)
    assert math.isnan(r["dsr"]) and math.isnan(r["psr_f"]) and r["dtvr"] == 1.0
    D[0, 6, 6] = 0.0
    lab[0, 0, 8] = 1
    r = p.evaluate(torch.as_tensor(D, device=dev()), torch.as_tensor(lab, device=dev()), None, f_t_scalar=1.0)
    assert math.isinf(r["dtvr"]) and math.isinf(r["dsr"])

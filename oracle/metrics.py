"""Scale-invariant metrics, post-scaling and the material response (Sec. 2.4-2.6, 3).

  DTVR  = max_gel(D / f~_T) / min_gel(D / f~_T)                      (Eq. 6, 8)
  DSR   = max_band D / min_gel(D / f~_T)                             (Eq. 8)
  PSR_f = min_gel D / max_band D                                     (Eq. 46)
  PSR_m = min_gel M(D) / max_band M(D)                               (Eq. 46)
  alpha* = <f~*, f_T>_W / <f~*, f~*>_W   (weighted least squares)     (Eq. 27)
  alpha_m = argmin_{alpha > 0} sum_gel w (M(alpha f~*) - m_T)^2       (Eq. 28)
  M(f)   = a + (k - a) / [1 + exp(-beta (f - f0))]^(1/gamma)          (Eq. 4)
  M^-1(m) = f0 - (1/beta) ln[((k - a)/(m - a))^gamma - 1]            (Eq. 5)

Empty band: DSR and PSR are NaN.  min over gel of zero: DTVR = +inf.
The paper prints no resin constants, so M is exercised only with constants
passed in by the caller.
"""
from __future__ import annotations

import numpy as np

from .regions import BAND, GEL


def dtvr(D, f_t_norm, labels) -> float:
    gel = labels == GEL
    r = D[gel] / f_t_norm[gel]
    lo = r.min()
    return float(r.max() / lo) if lo > 0 else float("inf")


def dsr(D, f_t_norm, labels) -> float:
    gel, band = labels == GEL, labels == BAND
    if not band.any():
        return float("nan")
    lo = (D[gel] / f_t_norm[gel]).min()
    return float(D[band].max() / lo) if lo > 0 else float("inf")


def psr(values, labels) -> float:
    gel, band = labels == GEL, labels == BAND
    if not band.any():
        return float("nan")
    hi = values[band].max()
    return float(values[gel].min() / hi) if hi > 0 else float("inf")


def alpha_star(f_norm, f_target, labels, weights=None) -> float:
    gel = labels == GEL
    w = np.ones(int(gel.sum())) if weights is None else np.asarray(weights)[gel]
    a, b = f_norm[gel], f_target[gel]
    return float((w * a * b).sum() / (w * a * a).sum())


def richards(f, a, k, beta, gamma, f0):
    return a + (k - a) / (1.0 + np.exp(-beta * (np.asarray(f) - f0))) ** (1.0 / gamma)


def richards_inverse(m, a, k, beta, gamma, f0):
    return f0 - np.log(((k - a) / (np.asarray(m) - a)) ** gamma - 1.0) / beta


def phi_m(alpha, f_norm, m_target, labels, resin, weights=None) -> float:
    """Response-domain calibration functional of Eq. 28 at one alpha (resin = (a, k, beta, gamma, f0))."""
    gel = labels == GEL
    w = np.ones(int(gel.sum())) if weights is None else np.asarray(weights)[gel]
    m = richards(alpha * f_norm[gel], *resin)
    return float((w * (m - np.asarray(m_target)[gel]) ** 2).sum())


def alpha_m(f_norm, m_target, labels, resin, weights=None) -> float:
    """argmin over alpha > 0 of phi_m (Eq. 28): the paper calls it a cheap scalar problem and gives
    no method.  Reading: search log(alpha) over [alpha_f / 100, alpha_f * 100] around the dose-domain
    factor on a 41-point scan, then a bounded Brent refinement inside the best scan bracket."""
    from scipy.optimize import minimize_scalar
    with np.errstate(invalid="ignore", divide="ignore"):
        f_t_dose = richards_inverse(np.asarray(m_target), *resin)   # NaN where m_T leaves (a, k)
    a0 = alpha_star(f_norm, f_t_dose, labels, weights)
    a0 = a0 if np.isfinite(a0) and a0 > 0 else 1.0
    grid = np.linspace(np.log(a0) - np.log(100.0), np.log(a0) + np.log(100.0), 41)
    vals = [phi_m(np.exp(g), f_norm, m_target, labels, resin, weights) for g in grid]
    i = int(np.argmin(vals))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    r = minimize_scalar(lambda g: phi_m(np.exp(g), f_norm, m_target, labels, resin, weights), bounds=(lo, hi),
                        method="bounded", options={"xatol": 1e-13})
    return float(np.exp(r.x))


def dtvr_m(f_phys, m_target, labels, resin) -> float:
    """max_gel(M(f)/m_T) / min_gel(M(f)/m_T): in-part response uniformity (Sec. 3.4)."""
    gel = labels == GEL
    q = richards(f_phys[gel], *resin) / np.asarray(m_target)[gel]
    return float(q.max() / q.min())

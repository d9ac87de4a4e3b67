"""Scale-invariant metrics, post-scaling and the material response (Sec. 2.4-2.6, 3).

  DTVR  = max_gel(D / f~_T) / min_gel(D / f~_T)                      (Eq. 6, 8)
  DSR   = max_band D / min_gel(D / f~_T)                             (Eq. 8)
  PSR_f = min_gel D / max_band D                                     (Eq. 46)
  PSR_m = min_gel M(D) / max_band M(D)                               (Eq. 46)
  alpha* = <f~*, f_T>_W / <f~*, f~*>_W   (weighted least squares)     (Eq. 27)
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

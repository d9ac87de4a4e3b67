"""KKT residuals and infeasibility certificates (Supp. 6.1, Eq. 47-51).

For the unified LP  min c^T x  s.t.  G x <= h,  x >= 0,  y_mask = 0  (see
``lp``) with multipliers lambda = (lambda1 on band, lambda2, lambda3 on gel):

  stationarity (Eq. 48-51): reduced costs
      q   = P K z,  z = lambda1[band] + lambda2[gel] - lambda3[gel]   >= 0 on act
      r_u = w1 - sum(lambda1)          >= 0   (u free; Eq. 48 with u >= 0)
      r_v = w2 - sum(U lambda2)        >= 0   (v free; Eq. 49 with v >= 0)
  primal feasibility: the rows of G x <= h (Sec. 6.1.3)
  dual objective:  d = sum_gel L lambda3 - [u fixed] h sum lambda1
                       - [v fixed] sum_gel U lambda2

Relative residuals (l2):
  eps_p   = ||(G x - h)^+|| / (1 + ||h||)
  eps_d   = ||[min(q, 0) on act, min(r_u, 0), min(r_v, 0)]|| / (1 + ||c||)
  eps_gap = |p - d| / (1 + |p| + |d|)

Lambda arrays are voxel-shaped: lam_up holds lambda1 on band and lambda2 on
gel; lam_lo holds lambda3 on gel.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .lp import LPProblem


@dataclass
class KKT:
    eps_p: float
    eps_d: float
    eps_gap: float
    primal_obj: float
    dual_obj: float
    r_p: float        # absolute ||(Gx - h)^+||
    r_d: float        # absolute dual residual norm
    gap: float        # p - d

    @property
    def rel(self) -> float:
        return max(self.eps_p, self.eps_d, self.eps_gap)


def h_norm(prob: LPProblem) -> float:
    band, gel = prob.band, prob.gel
    s = float((prob.lo[gel] ** 2).sum())
    if not prob.u_free:
        s += float(band.sum()) * prob.h ** 2
    if not prob.v_free:
        s += float((prob.hi[gel] ** 2).sum())
    return float(np.sqrt(s))


def c_norm(prob: LPProblem) -> float:
    return float(np.hypot(prob.w1 if prob.u_free else 0.0, prob.w2 if prob.v_free else 0.0))


def z_of(prob: LPProblem, lam_up, lam_lo) -> np.ndarray:
    band, gel = prob.band, prob.gel
    z = np.zeros(prob.labels.shape)
    z[band] = lam_up[band]
    z[gel] = lam_up[gel] - lam_lo[gel]
    return z


def dual_objective(prob: LPProblem, lam_up, lam_lo) -> float:
    band, gel = prob.band, prob.gel
    d = float((prob.lo[gel] * lam_lo[gel]).sum())
    if not prob.u_free:
        d -= prob.h * float(lam_up[band].sum())
    if not prob.v_free:
        d -= float((prob.hi[gel] * lam_up[gel]).sum())
    return d


def residuals(prob: LPProblem, y, u, v, lam_up, lam_lo, D=None, q=None) -> KKT:
    band, gel = prob.band, prob.gel
    y = np.asarray(y, dtype=np.float64)
    D = prob.dose(y) if D is None else D
    ub = prob.upper_bound(u, v)
    rp = np.concatenate([np.maximum(D[band] - ub[band], 0.0),
                         np.maximum(D[gel] - ub[gel], 0.0),
                         np.maximum(prob.lo[gel] - D[gel], 0.0),
                         np.minimum(y[prob.act], 0.0),
                         y[~prob.act]])
    if q is None:
        q = prob.adjoint(z_of(prob, lam_up, lam_lo))
    rd = [np.minimum(q[prob.act], 0.0)]
    if prob.u_free:
        rd.append(np.array([min(prob.w1 - float(lam_up[band].sum()), 0.0)]))
    if prob.v_free:
        rd.append(np.array([min(prob.w2 - float((prob.hi[gel] * lam_up[gel]).sum()), 0.0)]))
    rd = np.concatenate(rd)
    p = prob.objective(u, v)
    d = dual_objective(prob, lam_up, lam_lo)
    r_p = float(np.linalg.norm(rp))
    r_d = float(np.linalg.norm(rd))
    return KKT(eps_p=r_p / (1.0 + h_norm(prob)), eps_d=r_d / (1.0 + c_norm(prob)),
               eps_gap=abs(p - d) / (1.0 + abs(p) + abs(d)), primal_obj=p, dual_obj=d,
               r_p=r_p, r_d=r_d, gap=p - d)


def farkas_check(prob: LPProblem, lam_up, lam_lo, tol: float = 1e-9) -> dict:
    """Verify an approximate Farkas certificate of primal infeasibility.

    A dual ray lambda >= 0 with G^T lambda >= 0 on the x >= 0 columns and
    h^T lambda < 0 proves G x <= h, x >= 0 has no solution.  The ray is scaled
    to -h^T lambda = 1; then every reduced-cost violation must be <= tol.
    Components: q = P K z >= 0 on act; -sum(lambda1) >= 0 if u is free;
    -sum(U lambda2) >= 0 if v is free.
    """
    band, gel = prob.band, prob.gel
    lu = np.where(band | gel, np.maximum(lam_up, 0.0), 0.0)
    ll = np.where(gel, np.maximum(lam_lo, 0.0), 0.0)
    ray_obj = dual_objective(prob, lu, ll)           # = -h^T lambda
    if not ray_obj > 0.0:
        return {"valid": False, "reason": "dual ray objective not positive", "ray_obj": ray_obj}
    lu, ll = lu / ray_obj, ll / ray_obj
    q = prob.adjoint(z_of(prob, lu, ll))
    viol = [float(-np.minimum(q[prob.act], 0.0).min(initial=0.0))]
    if prob.u_free:
        viol.append(float(lu[band].sum()))
    if prob.v_free:
        viol.append(float((prob.hi[gel] * lu[gel]).sum()))
    worst = max(viol)
    return {"valid": worst <= tol, "worst": worst, "ray_obj": ray_obj}

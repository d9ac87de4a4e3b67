"""The Charnes-Cooper linear program (Sec. 2.6-2.7) in one unified form.

After the Charnes-Cooper change of variables y = t g, u~ = t u, v~ = t v
(Eq. 18) the general problem is (Eq. 19-24)

    minimise    w1 u + w2 v
    subject to  (A^T y)_i - u       <= 0   i in band           (Eq. 20)
                (A^T y)_i - v f~_T,i <= 0   i in gel            (Eq. 21)
                f~_T,i - (A^T y)_i   <= 0   i in gel            (Eq. 22)
                y_j >= 0 (act),  y_j = 0 (mask)                 (Eq. 23-24)

with A^T = K P^T (Eq. 3).  Case 1 (Eq. 32-37) fixes v = 1 with per-voxel
bounds f~_L <= A^T y <= f~_U on gel and w = (1, 0); Case 2 (Eq. 40-45) fixes
the band cap u = 1 and w = (0, 1).  All three are one LP

    min  w1 u + w2 v   s.t.   D - u_bar <= 0 (band),  D - v_bar U <= 0 (gel),
                              L - D <= 0 (gel),  y >= 0,  y_mask = 0,
    where D = K P^T y, u_bar = u if u is free else h, v_bar = v if v is free else 1.

Free scalars carry the bound u, v >= 0.  Any feasible point has u >= max band
dose >= 0 and v >= 1, so this only matters when the band is empty, where it
makes u* = 0 instead of unbounded.

Explicit assembly (``assemble``) is for small instances; the matrix-free
operators serve every size.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog

from . import blur as _blur
from . import regions as _regions
from .projector import Projector

GENERAL, CASE1, CASE2 = 0, 1, 2


@dataclass
class LPProblem:
    proj: Projector
    taps: object                 # (tx, ty, tz) or None for K = I
    labels: np.ndarray           # uint8 [nz][n][n]: 0 ext, 1 band, 2 gel
    act: np.ndarray              # bool sinogram mask
    lo: np.ndarray               # L_i (used on gel)
    hi: np.ndarray               # U_i (used on gel)
    u_free: bool
    v_free: bool
    w1: float
    w2: float
    h: float = 1.0               # band cap when u is fixed
    case: int = GENERAL
    f_crit: float = 1.0
    meta: dict = field(default_factory=dict)

    # ------------------------------------------------------------ operators
    @property
    def band(self):
        return self.labels == _regions.BAND

    @property
    def gel(self):
        return self.labels == _regions.GEL

    def dose(self, y: np.ndarray) -> np.ndarray:
        """D = K P^T y (Eq. 2-3)."""
        return _blur.apply(self.proj.backproject(y), self.taps)

    def adjoint(self, z: np.ndarray) -> np.ndarray:
        """q = P K z, the adjoint of ``dose`` (K symmetric, Eq. 51)."""
        return self.proj.project(_blur.apply(z, self.taps))

    def upper_bound(self, u: float, v: float) -> np.ndarray:
        """Per-voxel right-hand side of the upper rows: u_bar on band, v_bar U on gel."""
        ub = np.zeros(self.labels.shape)
        ub[self.band] = u if self.u_free else self.h
        ub[self.gel] = (v if self.v_free else 1.0) * self.hi[self.gel]
        return ub

    def objective(self, u: float, v: float) -> float:
        return (self.w1 * u if self.u_free else 0.0) + (self.w2 * v if self.v_free else 0.0)

    def violation(self, y, u, v) -> float:
        """Max constraint violation in normalised dose units."""
        D = self.dose(y)
        ub = self.upper_bound(u, v)
        m = self.band | self.gel
        viol = 0.0
        if m.any():
            viol = max(viol, float(np.max(np.maximum(D[m] - ub[m], 0.0))))
        g = self.gel
        if g.any():
            viol = max(viol, float(np.max(np.maximum(self.lo[g] - D[g], 0.0))))
        yy = np.asarray(y)
        viol = max(viol, float(np.max(np.maximum(-yy, 0.0))) if yy.size else 0.0)
        viol = max(viol, float(np.max(np.abs(yy[~self.act]))) if (~self.act).any() else 0.0)
        return viol


def build(proj: Projector, f_target: np.ndarray, case: int, taps=None, band_width: float = 10.0,
          w1: float = 1.0, w2: float = 1.0, tol_lo: float = 0.9, tol_hi: float = 1.0,
          cap: float = 0.7) -> LPProblem:
    """Problem construction (Fig. 1 a-c) for a target dose f_T.

    general: f_crit = min over gel of f_T (Sec. 2.5); L = U = f~_T; u, v free.
    case 1:  f_L = tol_lo f_T, f_U = tol_hi f_T (the dose-domain tolerance
             window), f_crit = min f_L (Eq. 30), L = f_L / f_crit,
             U = f_U / f_crit (Eq. 31); w = (1, 0); v fixed.
    case 2:  f_crit = cap * min f_T (the inhibition threshold as a fraction of
             the target dose), f~_T = f_T / f_crit (Eq. 39); band cap h = 1
             (Eq. 41); w = (0, 1); u fixed.
    """
    f = np.asarray(f_target, dtype=np.float64)
    lab = _regions.labels(f, band_width=band_width, taps=taps)
    act = _regions.active_rays(proj, f)
    gel = lab == _regions.GEL
    fmin = float(f[gel].min()) if gel.any() else 1.0
    if case == GENERAL:
        fc = fmin
        lo = hi = f / fc
        return LPProblem(proj, taps, lab, act, lo, hi, True, True, w1, w2, 1.0, GENERAL, fc)
    if case == CASE1:
        fl, fu = tol_lo * f, tol_hi * f
        fc = tol_lo * fmin
        return LPProblem(proj, taps, lab, act, fl / fc, fu / fc, True, False, 1.0, 0.0, 1.0, CASE1, fc)
    if case == CASE2:
        fc = cap * fmin
        ft = f / fc
        return LPProblem(proj, taps, lab, act, ft, ft, False, True, 0.0, 1.0, 1.0, CASE2, fc)
    raise ValueError(f"unknown case {case}")


# ---------------------------------------------------------------- assembly
def dose_matrix(prob: LPProblem) -> sp.csr_matrix:
    """Explicit A^T = K P^T over the full volume and sinogram (small instances)."""
    g = prob.proj.geom
    n2 = g.n * g.n
    PT = prob.proj.PT.tocoo()                      # (n2, A*B) slice matrix
    blocks_r, blocks_c, blocks_v = [], [], []
    for z in range(g.nz):
        a, b = np.divmod(PT.col, g.n_bins)
        blocks_r.append(z * n2 + PT.row)
        blocks_c.append(a * (g.nz * g.n_bins) + z * g.n_bins + b)
        blocks_v.append(PT.data)
    PT3 = sp.coo_matrix((np.concatenate(blocks_v), (np.concatenate(blocks_r), np.concatenate(blocks_c))),
                        shape=(g.nz * n2, g.n_angles * g.nz * g.n_bins)).tocsr()
    if prob.taps is None:
        return PT3
    tx, ty, tz = prob.taps

    def conv1d(n, t):
        r = (len(t) - 1) // 2
        return sp.diags([np.full(n - abs(k), t[k + r]) for k in range(-r, r + 1) if n - abs(k) > 0],
                        [k for k in range(-r, r + 1) if n - abs(k) > 0], shape=(n, n))
    K = sp.kron(sp.kron(conv1d(g.nz, tz), conv1d(g.n, ty)), conv1d(g.n, tx)).tocsr()
    return (K @ PT3).tocsr()


@dataclass
class Assembled:
    G: sp.csr_matrix
    h: np.ndarray
    c: np.ndarray
    act_idx: np.ndarray
    band_idx: np.ndarray
    gel_idx: np.ndarray
    n_y: int


def assemble(prob: LPProblem) -> Assembled:
    """G x <= h, x >= 0 with x = (y on act, [u], [v])."""
    AT = dose_matrix(prob)
    act_idx = np.nonzero(prob.act.ravel())[0]
    band_idx = np.nonzero(prob.band.ravel())[0]
    gel_idx = np.nonzero(prob.gel.ravel())[0]
    ATa = AT[:, act_idx]
    ny = len(act_idx)
    U = prob.hi.ravel()[gel_idx]
    L = prob.lo.ravel()[gel_idx]
    nb, ng = len(band_idx), len(gel_idx)
    extra = []
    if prob.u_free:
        extra.append(sp.vstack([sp.csr_matrix(-np.ones((nb, 1))), sp.csr_matrix((2 * ng, 1))]))
    if prob.v_free:
        extra.append(sp.vstack([sp.csr_matrix((nb, 1)), sp.csr_matrix(-U.reshape(-1, 1)),
                                sp.csr_matrix((ng, 1))]))
    Gy = sp.vstack([ATa[band_idx], ATa[gel_idx], -ATa[gel_idx]])
    G = sp.hstack([Gy] + extra).tocsr()
    h = np.concatenate([np.full(nb, 0.0 if prob.u_free else prob.h),
                        np.zeros(ng) if prob.v_free else U,
                        -L])
    c = np.concatenate([np.zeros(ny)] + ([np.array([prob.w1])] if prob.u_free else [])
                       + ([np.array([prob.w2])] if prob.v_free else []))
    return Assembled(G, h, c, act_idx, band_idx, gel_idx, ny)


@dataclass
class LPSolution:
    status: str                  # "optimal" | "infeasible" | other
    objective: float
    y: np.ndarray
    u: float
    v: float
    lam_up: np.ndarray
    lam_lo: np.ndarray


def unpack(prob: LPProblem, asm: Assembled, x: np.ndarray, lam: np.ndarray):
    """Map (x, lambda) of the assembled LP back to (y, u, v, lam_up, lam_lo)."""
    g = prob.proj.geom
    y = np.zeros(int(np.prod(g.sino_shape)))
    y[asm.act_idx] = x[:asm.n_y]
    k = asm.n_y
    u = v = 0.0
    if prob.u_free:
        u = float(x[k]); k += 1
    else:
        u = prob.h
    if prob.v_free:
        v = float(x[k]); k += 1
    else:
        v = 1.0
    nb, ng = len(asm.band_idx), len(asm.gel_idx)
    lam_up = np.zeros(int(np.prod(g.vol_shape)))
    lam_lo = np.zeros_like(lam_up)
    lam_up[asm.band_idx] = lam[:nb]
    lam_up[asm.gel_idx] = lam[nb:nb + ng]
    lam_lo[asm.gel_idx] = lam[nb + ng:]
    return (y.reshape(g.sino_shape), u, v, lam_up.reshape(g.vol_shape), lam_lo.reshape(g.vol_shape))


def solve_highs(prob: LPProblem) -> LPSolution:
    """Exact LP solution with HiGHS (scipy.optimize.linprog), small instances."""
    asm = assemble(prob)
    res = linprog(asm.c, A_ub=asm.G, b_ub=asm.h, bounds=(0, None), method="highs")
    g = prob.proj.geom
    if res.status == 2:
        z = np.zeros(g.vol_shape)
        return LPSolution("infeasible", np.nan, np.zeros(g.sino_shape), np.nan, np.nan, z, z)
    if res.status != 0:
        raise RuntimeError(f"HiGHS failed: {res.message}")
    lam = -np.asarray(res.ineqlin.marginals)
    y, u, v, lu, ll = unpack(prob, asm, res.x, lam)
    return LPSolution("optimal", float(res.fun), y, u, v, lu, ll)

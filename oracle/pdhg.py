"""Matrix-free PDHG for the unified Charnes-Cooper LP (Sec. 2.8) -- FP64 oracle.

The paper states only that the LP is solved by a matrix-free primal-dual
hybrid gradient method whose primal descent and dual ascent follow the KKT
system of Supp. 6.1 (Eq. 47-51).  The iteration below is the standard
Chambolle-Pock form of that saddle problem

    min_{x in X} max_{lambda >= 0}  c^T x + lambda^T (G x - h),
    X = {y >= 0 on act, y = 0 on mask, u >= 0, v >= 0},

written with the dose operator D = K P^T y (Eq. 3) and its adjoint
q = P K z (Eq. 51):

    z      = lambda1[band] + lambda2[gel] - lambda3[gel]
    y+     = act ? max(0, y - tau_y * P K z) : 0                      (Eq. 50-51)
    u+     = max(0, u - tau_u (w1 - sum lambda1))          if u free  (Eq. 48)
    v+     = max(0, v - tau_v (w2 - sum U lambda2))        if v free  (Eq. 49)
    D+     = K P^T y+                 (one backprojection per iteration)
    Dbar   = 2 D+ - D,  ubar = 2 u+ - u,  vbar = 2 v+ - v
    lambda1 <- max(0, lambda1 + s (Dbar - ubar))        on band (ubar = h if u fixed)
    lambda2 <- max(0, lambda2 + s (Dbar - vbar U))      on gel  (vbar = 1 if v fixed)
    lambda3 <- max(0, lambda3 + s (L - Dbar))           on gel

``pdhg_plain`` uses scalar steps tau = sigma = 0.9 / ||G|| (100 power
iterations from the all-ones vector on the act columns and free scalars).

``pdhg_restarted`` is a restarted reflected Halpern PDHG (prior art: the
Halpern-iteration and restart schemes for PDHG on LPs of Lu and Yang, and
PDLP by Applegate et al.), arranged here as: diagonal Pock-Chambolle steps
(alpha = 1) T_j = 1 / sum_i |G_ij|, S_i = 1 / sum_j |G_ij| from P K w (w = 1 on
band, 2 on gel) and K P^T 1_act; a primal weight omega (tau = eta T / omega,
sigma = eta omega S); the Halpern anchor at the last restart; a KKT check
every ``check_every`` iterations on the PDHG output; restarts under the
sufficient (0.2) / necessary (0.8) / artificial (0.36) rules; omega updated
from the movement between restarts; and Farkas tests of two dual
differences (one step, and one check window).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import kkt as _kkt
from .lp import LPProblem

OPTIMAL, PRIMAL_INFEASIBLE, ITER_LIMIT, NUMERICAL = 0, 1, 2, 3


@dataclass
class State:
    y: np.ndarray
    u: float
    v: float
    lam_up: np.ndarray
    lam_lo: np.ndarray
    D: np.ndarray

    def copy(self):
        return State(self.y.copy(), self.u, self.v, self.lam_up.copy(), self.lam_lo.copy(), self.D.copy())


@dataclass
class Result:
    status: int
    iters: int
    state: State
    kkt: object
    restarts: int = 0
    tau: float = 0.0
    sigma: float = 0.0
    omega: float = 1.0
    history: list = field(default_factory=list)
    certificate: tuple | None = None


def initial_state(prob: LPProblem) -> State:
    g = prob.proj.geom
    return State(np.zeros(g.sino_shape), 0.0 if prob.u_free else prob.h, 0.0 if prob.v_free else 1.0,
                 np.zeros(g.vol_shape), np.zeros(g.vol_shape), np.zeros(g.vol_shape))


# ------------------------------------------------------------------ G, G^T
def apply_G(prob: LPProblem, y, u, v):
    """Row blocks (band, gel-up, gel-lo) of G x for x = (y, [u], [v])."""
    D = prob.dose(y)
    band, gel = prob.band, prob.gel
    rb = D[band] - (u if prob.u_free else 0.0)
    ru = D[gel] - (v * prob.hi[gel] if prob.v_free else 0.0)
    rl = -D[gel]
    return rb, ru, rl


def apply_GT(prob: LPProblem, rb, ru, rl):
    band, gel = prob.band, prob.gel
    z = np.zeros(prob.labels.shape)
    z[band] = rb
    z[gel] = ru - rl
    gy = prob.adjoint(z) * prob.act
    gu = -float(rb.sum()) if prob.u_free else 0.0
    gv = -float((prob.hi[gel] * ru).sum()) if prob.v_free else 0.0
    return gy, gu, gv


def power_norm(prob: LPProblem, iters: int = 100) -> float:
    """||G||_2 on the act y-columns and free scalar columns, by power iteration on G^T G."""
    y = prob.act.astype(np.float64)
    u = 1.0 if prob.u_free else 0.0
    v = 1.0 if prob.v_free else 0.0
    nrm = np.sqrt((y * y).sum() + u * u + v * v)
    y, u, v = y / nrm, u / nrm, v / nrm
    lam = 0.0
    for _ in range(iters):
        gy, gu, gv = apply_GT(prob, *apply_G(prob, y, u, v))
        lam = np.sqrt((gy * gy).sum() + gu * gu + gv * gv)
        if lam == 0.0:
            return 0.0
        y, u, v = gy / lam, gu / lam, gv / lam
    return float(np.sqrt(lam))


# ------------------------------------------------------------- one step
def step(prob: LPProblem, st: State, tau_y, tau_u, tau_v, s_up, s_lo) -> State:
    """One Chambolle-Pock iteration (see module docstring); steps may be arrays."""
    band, gel = prob.band, prob.gel
    z = _kkt.z_of(prob, st.lam_up, st.lam_lo)
    q = prob.adjoint(z)
    y = np.where(prob.act, np.maximum(0.0, st.y - tau_y * q), 0.0)
    if prob.u_free:
        u = max(0.0, st.u - tau_u * (prob.w1 - float(st.lam_up[band].sum())))
        ubar = 2.0 * u - st.u
    else:
        u = ubar = prob.h
    if prob.v_free:
        v = max(0.0, st.v - tau_v * (prob.w2 - float((prob.hi[gel] * st.lam_up[gel]).sum())))
        vbar = 2.0 * v - st.v
    else:
        v = vbar = 1.0
    D = prob.dose(y)
    Dbar = 2.0 * D - st.D
    lu = st.lam_up.copy()
    ll = st.lam_lo.copy()
    su = s_up[band] if np.ndim(s_up) else s_up
    lu[band] = np.maximum(0.0, lu[band] + su * (Dbar[band] - ubar))
    su = s_up[gel] if np.ndim(s_up) else s_up
    lu[gel] = np.maximum(0.0, lu[gel] + su * (Dbar[gel] - vbar * prob.hi[gel]))
    sl = s_lo[gel] if np.ndim(s_lo) else s_lo
    ll[gel] = np.maximum(0.0, ll[gel] + sl * (prob.lo[gel] - Dbar[gel]))
    return State(y, u, v, lu, ll, D)


def pdhg_plain(prob: LPProblem, iters: int, tau: float | None = None, sigma: float | None = None,
               record_every: int = 0) -> Result:
    """Plain Chambolle-Pock: theta = 1, primal first, no restarts or averaging."""
    if tau is None or sigma is None:
        nrm = power_norm(prob)
        tau = sigma = 0.9 / nrm
    st = initial_state(prob)
    hist = []
    for k in range(1, iters + 1):
        st = step(prob, st, tau, tau, tau, sigma, sigma)
        if record_every and k % record_every == 0:
            hist.append((k, _kkt.residuals(prob, st.y, st.u, st.v, st.lam_up, st.lam_lo, D=st.D)))
    res = _kkt.residuals(prob, st.y, st.u, st.v, st.lam_up, st.lam_lo, D=st.D)
    return Result(ITER_LIMIT, iters, st, res, 0, tau, sigma, 1.0, hist)


# ------------------------------------------------------ restarted variant
@dataclass
class Scaling:
    T: np.ndarray       # per-ray primal scaling (0 on mask)
    Tu: float
    Tv: float
    S_up: np.ndarray    # per-voxel dual scaling of the upper rows
    S_lo: np.ndarray    # per-voxel dual scaling of the lower rows


def diagonal_scaling(prob: LPProblem) -> Scaling:
    """Pock-Chambolle alpha = 1: inverse absolute column / row sums of G."""
    band, gel = prob.band, prob.gel
    w = band.astype(np.float64) + 2.0 * gel
    col = prob.adjoint(w)
    T = np.where(prob.act & (col > 0), 1.0 / np.where(col > 0, col, 1.0), 0.0)
    nband = float(band.sum())
    Tu = 1.0 / nband if (prob.u_free and nband > 0) else 0.0
    sU = float(prob.hi[gel].sum())
    Tv = 1.0 / sU if (prob.v_free and sU > 0) else 0.0
    R = prob.dose(prob.act.astype(np.float64))
    rs_up = R + (band * (1.0 if prob.u_free else 0.0)) + (gel * (prob.hi if prob.v_free else 0.0))
    S_up = np.where((band | gel) & (rs_up > 0), 1.0 / np.where(rs_up > 0, rs_up, 1.0), 0.0)
    S_lo = np.where(gel & (R > 0), 1.0 / np.where(R > 0, R, 1.0), 0.0)
    return Scaling(T, Tu, Tv, S_up, S_lo)


def _merit(k: _kkt.KKT, omega: float = 1.0, kind: str = "relative") -> float:
    if kind == "weighted":
        return float(np.sqrt(omega ** 2 * k.r_p ** 2 + k.r_d ** 2 / omega ** 2 + k.gap ** 2))
    return float(np.sqrt(k.eps_p ** 2 + k.eps_d ** 2 + k.eps_gap ** 2))


def _wnorm(a, w):
    m = w > 0
    return float(np.sqrt((a[m] ** 2 / w[m]).sum()))


def infeasibility_ray(prob: LPProblem, d_up, d_lo, tol: float):
    """Test a dual iterate difference as a Farkas ray; returns (valid, lam_up, lam_lo)."""
    chk = _kkt.farkas_check(prob, d_up, d_lo, tol=tol)
    return chk["valid"], chk


def _combine(w: float, rho: float, t: State, z: State, anchor: State) -> State:
    """Reflected Halpern update: w ((1 + rho) t - rho z) + (1 - w) anchor."""
    def c(a, b, an):
        return w * ((1.0 + rho) * a - rho * b) + (1.0 - w) * an
    return State(c(t.y, z.y, anchor.y), c(t.u, z.u, anchor.u), c(t.v, z.v, anchor.v),
                 c(t.lam_up, z.lam_up, anchor.lam_up), c(t.lam_lo, z.lam_lo, anchor.lam_lo),
                 c(t.D, z.D, anchor.D))


def pdhg_restarted(prob: LPProblem, tol: float = 1e-4, max_iters: int = 20000, check_every: int = 64,
                   eta: float = 0.95, omega0: float = 1.0, infeas_tol: float = 1e-7,
                   beta_suff: float = 0.2, beta_nec: float = 0.8, beta_art: float = 0.36,
                   rho: float = 1.0) -> Result:
    """Restarted reflected Halpern PDHG with diagonal steps and a primal weight.

    z_{k+1} = w_k ((1 + rho) T(z_k) - rho z_k) + (1 - w_k) z_0,  w_k = (k + 1)/(k + 2),
    where T is one Chambolle-Pock step (``step``) with tau = eta T / omega,
    sigma = eta omega S, k counts iterations since the last restart and z_0 is
    the restart point.  Every ``check_every`` iterations the PDHG output
    t = T(z) (which satisfies the bounds) is checked: termination on its
    relative KKT error, a Farkas test of the dual one-step difference
    lambda(t) - lambda(z) and of the window difference lambda(t) - lambda(t at
    the previous check), and the restart rules on the l2 merit of the relative
    residuals (sufficient 0.2, necessary 0.8 with no progress, artificial
    0.36 of all iterations).  A restart moves z to t, makes it the new z_0 and
    updates omega from the primal / dual movement since the previous restart
    (scaled norms, geometric smoothing 1/2).
    """
    sc = diagonal_scaling(prob)
    omega = omega0
    z = initial_state(prob)
    anchor = z.copy()
    last = z.copy()
    k_in = 0
    k0 = _kkt.residuals(prob, z.y, z.u, z.v, z.lam_up, z.lam_lo, D=z.D)
    m_anchor = _merit(k0)
    m_prev = np.inf
    k_restart = 0
    restarts = 0
    snap = None
    hist = []
    t = z
    kc = k0
    for k in range(1, max_iters + 1):
        t = step(prob, z, eta * sc.T / omega, eta * sc.Tu / omega, eta * sc.Tv / omega,
                 eta * omega * sc.S_up, eta * omega * sc.S_lo)
        w = (k_in + 1.0) / (k_in + 2.0)
        check = k % check_every == 0
        if check:
            fx = (t.lam_up - z.lam_up, t.lam_lo - z.lam_lo)
        z = _combine(w, rho, t, z, anchor)
        k_in += 1
        if not check:
            continue
        if not (np.isfinite(t.y).all() and np.isfinite(t.lam_up).all()):
            return Result(NUMERICAL, k, t, None, restarts, omega=omega, history=hist)
        kc = _kkt.residuals(prob, t.y, t.u, t.v, t.lam_up, t.lam_lo, D=t.D)
        hist.append((k, kc.rel, omega))
        if kc.rel <= tol:
            return Result(OPTIMAL, k, t, kc, restarts, omega=omega, history=hist)
        for cand in ([fx] + ([(t.lam_up - snap[0], t.lam_lo - snap[1])] if snap is not None else [])):
            ok, _ = infeasibility_ray(prob, cand[0], cand[1], infeas_tol)
            if ok:
                return Result(PRIMAL_INFEASIBLE, k, t, kc, restarts, omega=omega, history=hist, certificate=cand)
        snap = (t.lam_up.copy(), t.lam_lo.copy())
        m = _merit(kc)
        if not (m <= beta_suff * m_anchor or (m <= beta_nec * m_anchor and m > m_prev)
                or (k - k_restart) >= beta_art * k):
            m_prev = m
            continue
        dx = np.sqrt(_wnorm((t.y - last.y).ravel(), sc.T.ravel()) ** 2
                     + ((t.u - last.u) ** 2 / sc.Tu if sc.Tu > 0 else 0.0)
                     + ((t.v - last.v) ** 2 / sc.Tv if sc.Tv > 0 else 0.0))
        dl = np.sqrt(_wnorm((t.lam_up - last.lam_up).ravel(), sc.S_up.ravel()) ** 2
                     + _wnorm((t.lam_lo - last.lam_lo).ravel(), sc.S_lo.ravel()) ** 2)
        if dx > 1e-10 and dl > 1e-10:
            omega = float(np.exp(0.5 * np.log(dl / dx) + 0.5 * np.log(omega)))
        z = t.copy()
        anchor = t.copy()
        last = t.copy()
        k_in = 0
        m_anchor = m
        m_prev = np.inf
        k_restart = k
        restarts += 1
    return Result(ITER_LIMIT, max_iters, t, kc, restarts, omega=omega, history=hist)

"""Dense two-phase revised simplex with Bland's rule -- an independent exact LP solver.

Solves  min c^T x  s.t.  G x <= h,  x >= 0  for tiny dense instances, so the
LP value of the Charnes-Cooper problem (Eq. 19-24 and the two cases) can be
checked against a solver that shares nothing with HiGHS or PDHG.  Slacks make
the rows equalities; rows with a negative right-hand side are negated and get
an artificial variable for phase 1.  Every iteration re-solves with the basis
matrix taken from the original data (no tableau updates), so rounding does
not accumulate.  Degenerate ties are broken by solving with a tiny random
perturbation of the right-hand side; the final basis is then re-evaluated on
the exact data and accepted only if it is primal feasible there.  Returns status, x, objective and the multipliers
lambda >= 0 of the <= rows.
"""
from __future__ import annotations

import numpy as np


def _iterate(A, b, cost, basis, allowed, eps, piv_tol, max_iter):
    m = A.shape[0]
    for _ in range(max_iter):
        B = A[:, basis]
        xb = np.linalg.solve(B, b)
        pi = np.linalg.solve(B.T, cost[basis])
        red = cost - A.T @ pi
        cand = np.nonzero((red < -eps) & allowed)[0]
        if len(cand) == 0:
            return "optimal", xb, red
        e = int(cand[0])                                   # Bland: smallest index enters
        d = np.linalg.solve(B, A[:, e])
        pos = d > piv_tol
        if not pos.any():
            return "unbounded", xb, red
        ratios = np.full(m, np.inf)
        ratios[pos] = np.maximum(xb[pos], 0.0) / d[pos]
        best = ratios.min()
        ties = np.nonzero(ratios <= best + 1e-12 * max(1.0, best))[0]
        r = int(min(ties, key=lambda i: basis[i]))         # Bland: smallest index leaves
        basis[r] = e
    return "iteration_limit", None, None


def solve(c, G, h, eps: float = 1e-10, piv_tol: float = 1e-9, max_iter: int = 200000):
    c = np.asarray(c, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    m, n = G.shape
    neg = h < 0
    n_art = int(neg.sum())
    N = n + m + n_art
    A = np.zeros((m, N))
    sgn = np.where(neg, -1.0, 1.0)
    A[:, :n] = sgn[:, None] * G
    A[np.arange(m), n + np.arange(m)] = sgn
    b_exact = sgn * h
    pert = np.random.default_rng(12345).uniform(0.0, 1.0, m)
    b = b_exact + 1e-9 * (1.0 + np.abs(b_exact)) * pert
    basis = []
    k = 0
    for i in range(m):
        if neg[i]:
            A[i, n + m + k] = 1.0
            basis.append(n + m + k)
            k += 1
        else:
            basis.append(n + i)
    allowed = np.ones(N, dtype=bool)
    if n_art:
        cost1 = np.zeros(N)
        cost1[n + m:] = 1.0
        st, xb, _ = _iterate(A, b, cost1, basis, allowed, eps, piv_tol, max_iter)
        if st != "optimal":
            return {"status": st}
        if cost1[basis] @ xb > 1e-9 * max(1.0, np.abs(h).max()):
            return {"status": "infeasible"}
        # pivot zero-level artificials out of the basis where a usable column exists
        for r in range(m):
            if basis[r] >= n + m:
                B = A[:, basis]
                row = np.linalg.solve(B.T, np.eye(m)[r]) @ A[:, :n + m]
                cand = [j for j in np.nonzero(np.abs(row) > 1e-7)[0] if j not in basis]
                if cand:
                    basis[r] = int(cand[0])
        allowed[n + m:] = False
    cost2 = np.zeros(N)
    cost2[:n] = c
    st, xb, red = _iterate(A, b, cost2, basis, allowed, eps, piv_tol, max_iter)
    if st != "optimal":
        return {"status": st}
    xb = np.linalg.solve(A[:, basis], b_exact)
    if xb.min() < -1e-8 * max(1.0, np.abs(h).max()):
        return {"status": "perturbation_failed"}
    x = np.zeros(N)
    x[basis] = np.maximum(xb, 0.0)
    # the reduced cost of slack i is lambda_i (a negated row flips both the
    # row multiplier and the slack column, so no sign change is needed)
    lam = red[n:n + m]
    return {"status": "optimal", "x": x[:n], "objective": float(c @ x[:n]), "lam": np.maximum(lam, 0.0)}

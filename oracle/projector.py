"""Explicit sparse backprojector P^T and forward projector P (Eq. 2-3, Sec. 2.3).

The paper defines the dose model f = A^T g with A^T = K P^T, P^T the discrete
backprojection and P its adjoint (Eq. 2-3), and allows the operator to carry
attenuation (Sec. 1).  It does not say how P^T is discretised.  Reading used
here (voxel-driven linear interpolation, parallel beam):

  for voxel i with centre (x, y) inside the vial and view theta:
      s = -x sin(theta) + y cos(theta)      detector coordinate
      t =  x cos(theta) + y sin(theta)      depth along the ray
      u = (s + 1) / ds - 1/2,  b = floor(u),  f = u - b      (ds = 2 / n_bins)
      a = exp(-atten * (t + sqrt(1 - s^2)))  Beer-Lambert factor: light enters
                                             the unit disk at t = -sqrt(1 - s^2)
      P^T[i, (theta, b)]     += a (1 - f)   if 0 <= b < n_bins
      P^T[i, (theta, b + 1)] += a f         if 0 <= b + 1 < n_bins

No angular or detector-pitch factor is applied (unit weights).  P is the exact
transpose.  In 3D the views are perpendicular to the rotation axis z and each
detector row sees one slice, so P_3D = I_z (x) P_2D: the same slice matrix is
applied to every z column.

Array layouts: volume [nz][n][n] (x fastest), sinogram [n_angles][nz][n_bins].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Geometry, plane_coords, in_vial


def slice_matrix(geom: Geometry, voxels=None) -> sp.csr_matrix:
    """P^T for one slice: shape (n*n, n_angles*n_bins), CSR, float64.

    ``voxels`` (flat slice indices) restricts the build to those rows; the
    other rows are left empty (used to sample large operators row by row).
    """
    n, nb = geom.n, geom.n_bins
    X, Y = plane_coords(n)
    inside = in_vial(n).ravel()
    if voxels is not None:
        sel = np.zeros(n * n, dtype=bool)
        sel[np.asarray(voxels)] = True
        inside = inside & sel
    vox = np.nonzero(inside)[0]
    x = X.ravel()[vox]
    y = Y.ravel()[vox]
    ds = 2.0 / nb
    rows, cols, vals = [], [], []
    for k, th in enumerate(geom.angles):
        sn, cs = np.sin(th), np.cos(th)
        s = -x * sn + y * cs
        t = x * cs + y * sn
        u = (s + 1.0) / ds - 0.5
        b = np.floor(u)
        f = u - b
        b = b.astype(np.int64)
        a = np.exp(-geom.atten * (t + np.sqrt(np.maximum(0.0, 1.0 - s * s))))
        for tap, w in ((b, a * (1.0 - f)), (b + 1, a * f)):
            ok = (tap >= 0) & (tap < nb)
            rows.append(vox[ok])
            cols.append(k * nb + tap[ok])
            vals.append(w[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n * n, geom.n_angles * nb))
    return m.tocsr()


class Projector:
    """P and P^T for a geometry, built once as an explicit sparse matrix."""

    def __init__(self, geom: Geometry):
        self.geom = geom
        self.PT = slice_matrix(geom)          # (n*n, A*B)
        self.P = self.PT.T.tocsr()            # (A*B, n*n)

    def backproject(self, sino: np.ndarray) -> np.ndarray:
        """vol = P^T sino; sino [A][nz][B] -> vol [nz][n][n]."""
        g = self.geom
        sino = np.asarray(sino, dtype=np.float64).reshape(g.sino_shape)
        cols = sino.transpose(0, 2, 1).reshape(g.n_angles * g.n_bins, g.nz)   # [(a,b)][z]
        out = self.PT @ cols                                                   # [i][z]
        return np.ascontiguousarray(out.T).reshape(g.vol_shape)

    def project(self, vol: np.ndarray) -> np.ndarray:
        """sino = P vol; vol [nz][n][n] -> sino [A][nz][B]."""
        g = self.geom
        vol = np.asarray(vol, dtype=np.float64).reshape(g.vol_shape)
        cols = vol.reshape(g.nz, g.n * g.n).T                                 # [i][z]
        out = self.P @ cols                                                    # [(a,b)][z]
        return np.ascontiguousarray(out.reshape(g.n_angles, g.n_bins, g.nz).transpose(0, 2, 1))


def brute_force_entries(geom: Geometry) -> dict:
    """Entry dictionary {(voxel, angle, bin): value} built ray-first with plain loops.

    Independent loop order from ``slice_matrix`` (for tiny grids only): for each
    view and bin, visit every voxel and add its hat-function weight
    a * max(0, 1 - |u - bin|), which equals the two interpolation taps.
    """
    import math
    n, nb = geom.n, geom.n_bins
    ds = 2.0 / nb
    out = {}
    for k, th in enumerate(geom.angles):
        sn, cs = math.sin(th), math.cos(th)
        for b in range(nb):
            for r in range(n):
                yv = -1.0 + (r + 0.5) * (2.0 / n)
                for c in range(n):
                    xv = -1.0 + (c + 0.5) * (2.0 / n)
                    if xv * xv + yv * yv > 1.0:
                        continue
                    s = -xv * sn + yv * cs
                    t = xv * cs + yv * sn
                    u = (s + 1.0) / ds - 0.5
                    w = 1.0 - abs(u - b)
                    if w <= 0.0:
                        continue
                    a = math.exp(-geom.atten * (t + math.sqrt(max(0.0, 1.0 - s * s))))
                    out[(r * n + c, k, b)] = out.get((r * n + c, k, b), 0.0) + a * w
    return out

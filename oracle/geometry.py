"""Discretisation of the object and projection domains (Sec. 2.2, Fig. 2).

The paper fixes only the index sets: an N x N object grid, N_angle views and
N_beam = N beamlets per view (Fig. 2 equations).  Readings used here (the
paper is silent on them):

  * the grid covers [-1, 1]^2 with pitch h = 2/N and centres -1 + (c + 1/2) h;
    3D stacks nz slices along the rotation axis z;
  * voxels whose centre lies outside the unit disk (the vial) are outside the
    object domain: they receive no dose and their projector column is zero;
  * n_bins detector bins cover [-1, 1] with pitch 2/n_bins;
  * a view at angle theta sends light along e = (cos t, sin t); the detector
    axis is n = (-sin t, cos t).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geometry:
    n: int              # grid is n x n per slice
    nz: int             # number of slices (1 in 2D)
    n_bins: int         # detector bins per row
    angles: tuple       # view angles, radians
    atten: float = 1.0  # Beer-Lambert coefficient in units of 1/vial radius (0 = none)

    @property
    def n_angles(self) -> int:
        return len(self.angles)

    @property
    def vol_shape(self):
        return (self.nz, self.n, self.n)

    @property
    def sino_shape(self):
        return (self.n_angles, self.nz, self.n_bins)


def make_geometry(n, n_angles_or_angles, n_bins=None, nz=1, atten=1.0) -> Geometry:
    if np.isscalar(n_angles_or_angles):
        k = np.arange(int(n_angles_or_angles), dtype=np.float64)
        ang = 2.0 * np.pi * k / int(n_angles_or_angles)
    else:
        ang = np.asarray(n_angles_or_angles, dtype=np.float64)
    return Geometry(n=int(n), nz=int(nz), n_bins=int(n if n_bins is None else n_bins),
                    angles=tuple(float(a) for a in ang), atten=float(atten))


def centres(n: int) -> np.ndarray:
    """Voxel (or bin) centre coordinates on [-1, 1]."""
    return -1.0 + (np.arange(n, dtype=np.float64) + 0.5) * (2.0 / n)


def plane_coords(n: int):
    """X[r, c] = x_c and Y[r, c] = y_r for the slice grid (row r is y, column c is x)."""
    c = centres(n)
    return np.meshgrid(c, c, indexing="xy")


def in_vial(n: int) -> np.ndarray:
    """Boolean [n, n] mask of voxels whose centre lies in the closed unit disk."""
    X, Y = plane_coords(n)
    return (X * X + Y * Y) <= 1.0

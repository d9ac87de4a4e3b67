"""Partition of the object and projection domains (Sec. 2.2, Fig. 2).

Object space (Fig. 2a):
  gel  = {i : f_T,i != 0}
  band = {i : f_T,i == 0, (K f_T)_i != 0}
  ext  = the rest.
With K = I the paper's band is empty, yet its experiments use a band of
width 10 voxels around the part and a band-free option in which every
non-target voxel is band (Sec. 3.2, 3.4).  Reading used here:
  band = {non-gel i in the vial : Euclidean centre distance to the nearest
          gel voxel <= w (in voxel units)}  union  (supp(K f_T) minus gel),
with w = inf meaning band-free.  Voxels outside the vial are never gel or
band (their dose is identically zero).

Projection space (Fig. 2b): act = {j : (P f_T)_j != 0}.  The test "!= 0" is
read as (P f_T)_j > 1e-6 * max_j (P f_T)_j so that rays grazing the part with
negligible weight are masked identically in every precision.

Label codes: 0 = exterior (or outside the vial), 1 = band, 2 = gel.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

from . import blur as _blur
from .geometry import in_vial

EXT, BAND, GEL = 0, 1, 2
ACT_REL_THRESHOLD = 1e-6


def labels(f_target: np.ndarray, band_width: float = 10.0, taps=None) -> np.ndarray:
    """uint8 label volume [nz][n][n] from the target dose f_T."""
    f = np.asarray(f_target, dtype=np.float64)
    nz, n, _ = f.shape
    vial = np.broadcast_to(in_vial(n), f.shape)
    gel = (f != 0.0) & vial
    out = np.zeros(f.shape, dtype=np.uint8)
    if gel.any():
        if np.isinf(band_width):
            near = np.ones(f.shape, dtype=bool)
        else:
            if nz == 1:
                d = ndimage.distance_transform_edt(~gel[0])[None]
            else:
                d = ndimage.distance_transform_edt(~gel)
            near = d <= band_width
        band = near & ~gel & vial
        if taps is not None:
            band |= _blur.support_dilate(gel, taps) & ~gel & vial
        out[band] = BAND
    out[gel] = GEL
    return out


def labels_brute_force(f_target: np.ndarray, band_width: float) -> np.ndarray:
    """Same partition (K = I) by explicit pairwise distances -- tiny grids only."""
    f = np.asarray(f_target, dtype=np.float64)
    nz, n, _ = f.shape
    vial = np.broadcast_to(in_vial(n), f.shape)
    gel = (f != 0.0) & vial
    out = np.zeros(f.shape, dtype=np.uint8)
    gz, gy, gx = np.nonzero(gel)
    for z in range(nz):
        for r in range(n):
            for c in range(n):
                if gel[z, r, c]:
                    out[z, r, c] = GEL
                elif vial[z, r, c] and len(gz):
                    d2 = (gz - z) ** 2 + (gy - r) ** 2 + (gx - c) ** 2
                    if np.sqrt(d2.min()) <= band_width:
                        out[z, r, c] = BAND
    return out


def active_rays(projector, f_target: np.ndarray) -> np.ndarray:
    """bool sinogram mask act = (P f_T) > 1e-6 * max (P f_T)."""
    pf = projector.project(f_target)
    m = pf.max() if pf.size else 0.0
    if m <= 0.0:
        return np.zeros(pf.shape, dtype=bool)
    return pf > ACT_REL_THRESHOLD * m

"""Object-space PSF operator K (Eq. 1-3; 3D set-up of Sec. 3).

The paper's only example is a Gaussian of standard deviation 1 voxel whose
populated support is 5 taps per axis (Sec. 3, 3D Thinker set-up), i.e. a
radius of 2 sigma.  Reading used here for any sigma:

  * per axis: radius r = ceil(2 sigma), taps w_k proportional to
    exp(-k^2 / (2 sigma^2)) for |k| <= r, normalised to sum 1;
  * K is the separable product of the three 1D kernels, "same" output size,
    zero outside the volume;
  * the kernel is symmetric, so K^T = K.
A sigma of 0 (or None) on an axis means the identity along that axis.
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_taps(sigma) -> np.ndarray:
    if sigma is None or sigma <= 0:
        return np.ones(1)
    r = int(math.ceil(2.0 * sigma))
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def psf_taps(sigma_xyz):
    """(taps_x, taps_y, taps_z) for sigmas given in (x, y, z) order; None -> identity."""
    if sigma_xyz is None:
        return None
    sx, sy, sz = sigma_xyz
    return gaussian_taps(sx), gaussian_taps(sy), gaussian_taps(sz)


def _conv_axis(vol: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    """out[i] = sum_k taps[k + r] * in[i + k] along ``axis``, zero outside."""
    r = (len(taps) - 1) // 2
    if r == 0:
        return vol * taps[0]
    out = np.zeros_like(vol)
    n = vol.shape[axis]
    for k in range(-r, r + 1):
        w = taps[k + r]
        lo, hi = max(0, -k), min(n, n - k)           # output indices i with 0 <= i+k < n
        if lo >= hi:
            continue
        dst = [slice(None)] * vol.ndim
        src = [slice(None)] * vol.ndim
        dst[axis] = slice(lo, hi)
        src[axis] = slice(lo + k, hi + k)
        out[tuple(dst)] += w * vol[tuple(src)]
    return out


def apply(vol: np.ndarray, taps) -> np.ndarray:
    """K vol for a volume [nz][ny][nx]; ``taps`` = (tx, ty, tz) or None for identity."""
    vol = np.asarray(vol, dtype=np.float64)
    if taps is None:
        return vol.copy()
    tx, ty, tz = taps
    out = _conv_axis(vol, tx, 2)
    out = _conv_axis(out, ty, 1)
    out = _conv_axis(out, tz, 0)
    return out


def support_dilate(mask: np.ndarray, taps) -> np.ndarray:
    """supp(K m) for a nonnegative indicator m: box dilation by the tap radii (all taps > 0)."""
    if taps is None:
        return mask.copy()
    tx, ty, tz = taps
    out = mask.astype(bool)
    for axis, t in ((2, tx), (1, ty), (0, tz)):
        r = (len(t) - 1) // 2
        acc = out.copy()
        n = out.shape[axis]
        for k in range(-r, r + 1):
            lo, hi = max(0, -k), min(n, n - k)
            if lo >= hi:
                continue
            dst = [slice(None)] * 3
            src = [slice(None)] * 3
            dst[axis] = slice(lo, hi)
            src[axis] = slice(lo + k, hi + k)
            acc[tuple(dst)] |= out[tuple(src)]
        out = acc
    return out

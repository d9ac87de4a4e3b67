"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module produces *inputs only*: angle tables, binary target doses f_T and
random fields.  It holds none of the method's arithmetic (no projector, no
blur, no region partition, no LP), so both the CPU oracle and the HIP path can
consume the same arrays without sharing any of the computation they check.

Conventions of the arrays produced here
  * volumes are C-ordered ``[nz][ny][nx]`` (x fastest); a 2D slice has nz = 1;
  * the square object grid covers [-1, 1]^2 with voxel centres
    ``-1 + (c + 1/2) * 2/N``; z slices use the same rule over [-1, 1];
  * the vial is the unit disk in (x, y) (a cylinder along z in 3D);
  * every generator takes an integer seed and uses ``numpy.random.Generator``
    with ``PCG64(seed)``; config ``c`` instance ``k`` uses seed ``1000*c + k``.

The target shapes stand in for the paper's own targets (a 512^2 logo and a
128x128x130 figure, Sec. 3), which are not available: random ellipses, an
annulus with disks, random ellipsoids and a jittered open-cell lattice.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng", "angles_uniform", "ellipses_target", "annulus_disks_target",
    "ellipsoids_target", "lattice_target", "uniform_field", "signed_field", "graded_levels",
    "BatchInstance", "batch_instances", "CONFIGS", "Config",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def angles_uniform(n_angles: int) -> np.ndarray:
    """theta_k = 2*pi*k/n_angles, k = 0..n-1 (uniform over 360 degrees)."""
    return 2.0 * math.pi * np.arange(n_angles, dtype=np.float64) / n_angles


def _centres(n: int) -> np.ndarray:
    return -1.0 + (np.arange(n, dtype=np.float64) + 0.5) * (2.0 / n)


def _plane(n: int):
    c = _centres(n)
    X, Y = np.meshgrid(c, c, indexing="xy")  # X[r, c] = x_c, Y[r, c] = y_r
    return X, Y


def _rotation_from_quaternion(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipses_target(n: int, seed: int, count: int = 3, g: np.random.Generator | None = None) -> np.ndarray:
    """Binary union of ``count`` random ellipses, shape [1, n, n] (float64).

    Centres area-uniform in r < 0.6, semi-axes U[0.1, 0.3], orientation
    U[0, pi); membership tested at voxel centres.
    """
    g = rng(seed) if g is None else g
    X, Y = _plane(n)
    inside = np.zeros((n, n), dtype=bool)
    for _ in range(count):
        r = 0.6 * math.sqrt(g.uniform())
        phi = 2.0 * math.pi * g.uniform()
        cx, cy = r * math.cos(phi), r * math.sin(phi)
        a, b = g.uniform(0.1, 0.3), g.uniform(0.1, 0.3)
        psi = g.uniform(0.0, math.pi)
        dx, dy = X - cx, Y - cy
        p = (dx * math.cos(psi) + dy * math.sin(psi)) / a
        q = (-dx * math.sin(psi) + dy * math.cos(psi)) / b
        inside |= (p * p + q * q) <= 1.0
    inside &= (X * X + Y * Y) <= 1.0
    return inside.astype(np.float64)[None]


def annulus_disks_target(n: int, seed: int) -> np.ndarray:
    """Annulus about the origin (inner U[0.2,0.3], outer U[0.45,0.6]) plus 4 disks.

    Disk radius U[0.05, 0.12], centre area-uniform in r < 0.85 - radius.
    Shape [1, n, n], float64 in {0, 1}.
    """
    g = rng(seed)
    X, Y = _plane(n)
    R2 = X * X + Y * Y
    r_in, r_out = g.uniform(0.2, 0.3), g.uniform(0.45, 0.6)
    inside = (R2 >= r_in * r_in) & (R2 <= r_out * r_out)
    for _ in range(4):
        rad = g.uniform(0.05, 0.12)
        rc = (0.85 - rad) * math.sqrt(g.uniform())
        phi = 2.0 * math.pi * g.uniform()
        cx, cy = rc * math.cos(phi), rc * math.sin(phi)
        inside |= ((X - cx) ** 2 + (Y - cy) ** 2) <= rad * rad
    inside &= R2 <= 1.0
    return inside.astype(np.float64)[None]


def _ellipsoid_mask(P: np.ndarray, centre, axes, Rm) -> np.ndarray:
    d = P - np.asarray(centre)[:, None]
    local = Rm.T @ d
    return ((local / np.asarray(axes)[:, None]) ** 2).sum(axis=0) <= 1.0


def _box(n: int, nz: int, lo, hi):
    """Index ranges (z, y, x slices) of the voxel centres inside the box [lo, hi] (x, y, z order)."""
    out = []
    for m, l, h in ((nz, lo[2], hi[2]), (n, lo[1], hi[1]), (n, lo[0], hi[0])):
        i0 = max(0, int(np.floor((l + 1.0) * m / 2.0 - 0.5)) - 1)
        i1 = min(m, int(np.ceil((h + 1.0) * m / 2.0 - 0.5)) + 2)
        out.append(slice(i0, max(i0, i1)))
    return tuple(out)


def _paint(inside: np.ndarray, n: int, nz: int, lo, hi, test) -> None:
    """inside[box] |= test(P) for the voxel-centre points P (3 x m, x/y/z rows) of the box [lo, hi]."""
    sz, sy, sx = _box(n, nz, lo, hi)
    if sz.start >= sz.stop or sy.start >= sy.stop or sx.start >= sx.stop:
        return
    c, cz = _centres(n), _centres(nz)
    Z, Y, X = np.meshgrid(cz[sz], c[sy], c[sx], indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    inside[sz, sy, sx] |= test(P).reshape(Z.shape)


def _vial(n: int, nz: int) -> np.ndarray:
    c = _centres(n)
    return np.broadcast_to((c[None, :] ** 2 + c[:, None] ** 2) <= 1.0, (nz, n, n))


def ellipsoids_target(n: int, seed: int, count: int = 6, nz: int | None = None) -> np.ndarray:
    """Union of ``count`` random ellipsoids, shape [nz, n, n] (float64 in {0,1}).

    Centres uniform in the ball r < 0.7, semi-axes U[0.1, 0.3], uniformly
    random rotation (random unit quaternion), clipped to the vial cylinder.
    Each ellipsoid is tested only inside its bounding box.
    """
    nz = n if nz is None else nz
    g = rng(seed)
    inside = np.zeros((nz, n, n), dtype=bool)
    for _ in range(count):
        while True:
            c = g.uniform(-0.7, 0.7, size=3)
            if c @ c < 0.49:
                break
        axes = g.uniform(0.1, 0.3, size=3)
        Rm = _rotation_from_quaternion(g.normal(size=4))
        r = float(axes.max())
        _paint(inside, n, nz, c - r, c + r, lambda P, c=c, axes=axes, Rm=Rm: _ellipsoid_mask(P, c, axes, Rm))
    inside &= _vial(n, nz)
    return inside.astype(np.float64)


def lattice_target(n: int, seed: int, nz: int | None = None) -> np.ndarray:
    """Jittered open-cell lattice, shape [nz, n, n] (float64 in {0,1}).

    3x3x3 node centres at {-0.4, 0, 0.4}^3 jittered by U[-0.04, 0.04]^3;
    nodes are ellipsoids with semi-axes U[0.06, 0.10] and random rotation;
    54 cylinders of radius 0.04 join axis-adjacent nodes.  Each primitive is
    tested only inside its bounding box.
    """
    nz = n if nz is None else nz
    g = rng(seed)
    grid = np.array([-0.4, 0.0, 0.4])
    nodes = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                nodes[i, j, k] = np.array([grid[i], grid[j], grid[k]]) + g.uniform(-0.04, 0.04, 3)
    inside = np.zeros((nz, n, n), dtype=bool)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                axes = g.uniform(0.06, 0.10, size=3)
                Rm = _rotation_from_quaternion(g.normal(size=4))
                c = nodes[i, j, k]
                r = float(axes.max())
                _paint(inside, n, nz, c - r, c + r, lambda P, c=c, axes=axes, Rm=Rm: _ellipsoid_mask(P, c, axes, Rm))
    rad = 0.04
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for di, dj, dk in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    a, b, c = i + di, j + dj, k + dk
                    if a > 2 or b > 2 or c > 2:
                        continue
                    p0, p1 = nodes[i, j, k], nodes[a, b, c]
                    seg = p1 - p0
                    L2 = seg @ seg

                    def cyl(P, p0=p0, seg=seg, L2=L2):
                        t = np.clip(((P - p0[:, None]) * seg[:, None]).sum(0) / L2, 0.0, 1.0)
                        closest = p0[:, None] + t[None] * seg[:, None]
                        return ((P - closest) ** 2).sum(0) <= rad * rad

                    _paint(inside, n, nz, np.minimum(p0, p1) - rad, np.maximum(p0, p1) + rad, cyl)
    inside &= _vial(n, nz)
    return inside.astype(np.float64)


def graded_levels(shape, seed: int, lo: float = 0.5, hi: float = 1.0, waves: int = 4) -> np.ndarray:
    """Smooth seeded field with values in [lo, hi] over a volume [nz][n][n] on [-1, 1]^3.

    A grayscale target is a binary target times this field (Sec. 3.3 designs for
    graded in-part doses): the mean of ``waves`` plane cosines with directions
    uniform on the sphere, wave numbers U[2, 6] and phases U[0, 2 pi), mapped
    affinely from [-1, 1] onto [lo, hi].
    """
    g = rng(seed)
    nz, ny, nx = shape
    z = _centres(nz) if nz > 1 else np.zeros(1)
    Z, Y, X = np.meshgrid(z, _centres(ny), _centres(nx), indexing="ij")
    acc = np.zeros(shape)
    for _ in range(waves):
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        k = g.uniform(2.0, 6.0)
        ph = g.uniform(0.0, 2.0 * math.pi)
        acc += np.cos(k * (d[0] * X + d[1] * Y + d[2] * Z) + ph)
    acc /= waves
    return lo + (hi - lo) * 0.5 * (acc + 1.0)


def uniform_field(shape, seed: int) -> np.ndarray:
    """U[0, 1) float64 field of the given shape."""
    return rng(seed).uniform(0.0, 1.0, size=shape)


def signed_field(shape, seed: int) -> np.ndarray:
    """U[-1, 1) float64 field of the given shape."""
    return rng(seed).uniform(-1.0, 1.0, size=shape)


@dataclass
class BatchInstance:
    """One instance of the uneven 2D batch: grid N, angle count, LP case, target."""
    seed: int
    n: int
    n_angles: int
    case: int
    target: np.ndarray = field(repr=False)


def batch_instances(count: int = 64, seed0: int = 2000, sizes=(128, 192, 256, 384, 512),
                    angle_counts=(180, 360, 720)) -> list[BatchInstance]:
    """The uneven batch: per instance k, seed = seed0 + k draws N, angles, case, then 3 ellipses."""
    out = []
    for k in range(count):
        s = seed0 + k
        g = rng(s)
        n = int(sizes[g.integers(len(sizes))])
        na = int(angle_counts[g.integers(len(angle_counts))])
        case = int(1 + g.integers(2))
        tgt = ellipses_target(n, s, g=g)
        out.append(BatchInstance(seed=s, n=n, n_angles=na, case=case, target=tgt))
    return out


@dataclass(frozen=True)
class Config:
    """A named workload: grid, angles, detector, blur and LP case."""
    name: str
    n: int
    nz: int
    n_angles: int
    n_bins: int
    sigma: tuple | None      # blur standard deviations (x, y, z) in voxels, None = identity
    cases: tuple             # LP cases exercised (1 = spillage, 2 = conformity)
    dtype: str


CONFIGS = {
    "slice64": Config("2D slice 64x64, 180 angles, ellipses, FP64", 64, 1, 180, 64, None, (1,), "f64"),
    "slice256": Config("2D slice 256x256, 360 angles, annulus+disks, FP32", 256, 1, 360, 256, None, (1, 2), "f32"),
    "batch64": Config("64 uneven 2D instances, N in {128..512}, angles in {180,360,720}", 0, 1, 0, 0, None, (1, 2), "f32"),
    "vol256": Config("3D 256^3, 360 angles, 256x256 detector, blur sigma 1.5", 256, 256, 360, 256, (1.5, 1.5, 1.5), (1,), "f32"),
    "vol512": Config("3D 512^3, 720 angles, 512x512 detector, blur sigma (1,1,2)", 512, 512, 720, 512, (1.0, 1.0, 2.0), (2,), "f32"),
}

"""Pins for the oracle projector (Eq. 2-3): brute force, closed forms, invariants."""
import math

import numpy as np
import pytest

from oracle.geometry import make_geometry, centres, in_vial
from oracle.projector import Projector, slice_matrix, brute_force_entries
from sipo_inputs import uniform_field


def test_brute_force_two_loop_orders_8x8():
    # voxel-first vectorised build vs ray-first scalar loops over the same entry rule
    angs = [0.0, 0.3, 1.0, math.pi / 2, 2.5, math.pi, 4.0, 5.9]
    g = make_geometry(8, angs, atten=1.0)
    PT = slice_matrix(g).tocoo()
    mat = {}
    for r, c, v in zip(PT.row, PT.col, PT.data):
        mat[(int(r), int(c) // g.n_bins, int(c) % g.n_bins)] = mat.get((int(r), int(c) // g.n_bins, int(c) % g.n_bins), 0.0) + v
    bf = brute_force_entries(g)
    keys = {k for k, v in mat.items() if v != 0.0} | set(bf)
    assert keys
    for k in keys:
        assert abs(mat.get(k, 0.0) - bf.get(k, 0.0)) <= 1e-14, k


def test_brute_force_non_square_detector():
    g = make_geometry(8, [0.2, 1.3, 3.9], n_bins=11, atten=0.7)
    PT = slice_matrix(g).tocoo()
    mat = {}
    for r, c, v in zip(PT.row, PT.col, PT.data):
        key = (int(r), int(c) // g.n_bins, int(c) % g.n_bins)
        mat[key] = mat.get(key, 0.0) + v
    bf = brute_force_entries(g)
    for k in set(mat) | set(bf):
        assert abs(mat.get(k, 0.0) - bf.get(k, 0.0)) <= 1e-14


@pytest.mark.parametrize("n", [16, 17])
def test_axis_aligned_views_are_attenuated_row_and_column_sums(n):
    alpha = 1.0
    g = make_geometry(n, [0.0, math.pi / 2, math.pi, 3 * math.pi / 2], atten=alpha)
    P = Projector(g)
    x = uniform_field((1, n, n), 11)
    x[0][~in_vial(n)] = 0.0
    s = P.project(x)[:, 0, :]
    c = centres(n)
    vial = in_vial(n)
    exp0 = np.zeros(n); exp1 = np.zeros(n); exp2 = np.zeros(n); exp3 = np.zeros(n)
    for b in range(n):
        for k in range(n):
            # theta = 0: light along +x, detector coordinate s = y -> bin = row
            if vial[b, k]:
                exp0[b] += math.exp(-alpha * (c[k] + math.sqrt(1 - c[b] ** 2))) * x[0, b, k]
            # theta = 90 deg: light along +y, s = -x -> bin = n-1-column
            col = n - 1 - b
            if vial[k, col]:
                exp1[b] += math.exp(-alpha * (c[k] + math.sqrt(1 - c[col] ** 2))) * x[0, k, col]
            # theta = 180 deg: light along -x, s = -y -> bin = n-1-row
            row = n - 1 - b
            if vial[row, k]:
                exp2[b] += math.exp(-alpha * (-c[k] + math.sqrt(1 - c[row] ** 2))) * x[0, row, k]
            # theta = 270 deg: light along -y, s = x -> bin = column
            if vial[k, b]:
                exp3[b] += math.exp(-alpha * (-c[k] + math.sqrt(1 - c[b] ** 2))) * x[0, k, b]
    for got, want in zip(s, (exp0, exp1, exp2, exp3)):
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_mass_identity_without_attenuation():
    # each voxel's two taps sum to 1 when no tap leaves the detector
    n = 32
    g = make_geometry(n, 37, atten=0.0)
    P = Projector(g)
    x = uniform_field((1, n, n), 5)
    cc = centres(n)
    X, Y = np.meshgrid(cc, cc, indexing="xy")
    x[0][X * X + Y * Y > 0.85 ** 2] = 0.0
    per_view = P.project(x)[:, 0, :].sum(axis=1)
    np.testing.assert_allclose(per_view, x.sum(), rtol=1e-13)


def test_attenuated_uniform_disk_converges_to_closed_form():
    # continuum limit of P 1 at detector coordinate s: (1/h) * (1 - exp(-2 sqrt(1-s^2))) / alpha
    errs = []
    for n in (64, 256):
        g = make_geometry(n, [0.37], atten=1.0)
        P = Projector(g)
        x = in_vial(n).astype(float)[None]
        s = P.project(x)[0, 0]
        sb = centres(n)
        interior = np.abs(sb) < 0.8
        want = (n / 2.0) * (1.0 - np.exp(-2.0 * np.sqrt(1.0 - sb ** 2)))
        errs.append(np.max(np.abs(s[interior] - want[interior]) / want[interior]))
    assert errs[1] < errs[0]
    assert errs[1] < 2e-2


def test_3d_is_block_diagonal_in_z_and_adjoint_layout():
    n, nz = 12, 3
    g3 = make_geometry(n, 10, nz=nz, atten=1.0)
    g2 = make_geometry(n, 10, nz=1, atten=1.0)
    P3, P2 = Projector(g3), Projector(g2)
    x = uniform_field((nz, n, n), 1)
    y = uniform_field((10, nz, n), 2)
    s3 = P3.project(x)
    b3 = P3.backproject(y)
    for z in range(nz):
        np.testing.assert_allclose(s3[:, z:z + 1, :], P2.project(x[z:z + 1]), rtol=1e-14)
        np.testing.assert_allclose(b3[z:z + 1], P2.backproject(y[:, z:z + 1, :]), rtol=1e-14)
    assert abs((s3 * y).sum() - (x * b3).sum()) <= 1e-12 * abs((s3 * y).sum())


def test_outside_vial_voxels_have_zero_columns():
    n = 16
    g = make_geometry(n, 9)
    PT = slice_matrix(g)
    outside = ~in_vial(n).ravel()
    assert PT[outside].nnz == 0
    assert (PT.data >= 0).all()


def test_planted_mistake_is_caught(monkeypatch):
    # a projector with the detector axis flipped must fail the theta = 0 closed form
    import oracle.projector as pj
    n = 8
    g = make_geometry(n, [0.0], atten=1.0)
    real = pj.plane_coords

    def flipped(m):
        X, Y = real(m)
        return X, -Y
    monkeypatch.setattr(pj, "plane_coords", flipped)
    P = pj.Projector(g)
    x = uniform_field((1, n, n), 3)
    x[0][~in_vial(n)] = 0
    s = P.project(x)[0, 0]
    c = centres(n)
    want = np.array([sum(math.exp(-(c[k] + math.sqrt(1 - c[b] ** 2))) * x[0, b, k]
                         for k in range(n) if in_vial(n)[b, k]) for b in range(n)])
    assert np.max(np.abs(s - want)) > 1e-3

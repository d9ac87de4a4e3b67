"""GPU parity of the HIP operators (P^T, P, K, regions, active rays) against the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import blur as oblur, regions as oregions
from oracle.geometry import make_geometry
from oracle.projector import Projector, slice_matrix
from sipo_inputs import uniform_field, signed_field, ellipses_target, ellipsoids_target, angles_uniform

pytestmark = pytest.mark.gpu

F32_NORM_TOL = 1e-5      # normwise relative error bound for FP32 projector outputs
F64_TOL = 1e-12


def dev():
    return torch.device("cuda", 0)


def plan_for(n, angles, nz=1, n_bins=None, atten=1.0, sigma=None, dtype=torch.float32):
    from paper_2604_08997_amd import Plan
    return Plan(n, angles, n_bins=n_bins, nz=nz, atten=atten, sigma=sigma, dtype=dtype, device=dev())


def to_gpu(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def rel_norm(got, want):
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


CASES = [
    # (n, angles, nz, n_bins, atten)
    (64, 180, 1, None, 1.0),       # 2D slice of the small FP64 workload
    (67, 37, 1, 70, 0.7),          # ragged grid, non-square detector, odd angle count
    (40, 23, 13, 41, 1.0),         # 3D with a slice count that is not a multiple of the z chunk
    (24, [0.0, math.pi / 2, math.pi, 1.5 * math.pi, 0.25 * math.pi], 3, None, 0.0),   # exact axis/diagonal views
    (64, 45, 36, None, 1.0),       # 3D with a slice count divisible by 4 (vector staging path)
    (16, 10, 4, 40, 1.0),          # 3D with a detector much finer than the grid (general fallback path)
    (70, 181, 8, 70, 1.0),         # odd view count, views on both sides of the 45 degree split
    (48, 60, 20, None, 1.0),       # 3D, every view has its opposite: the projector walks view pairs
    (33, 90, 11, 35, 0.7),         # view pairs with a ragged grid, slice count and detector
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", CASES)
def test_backproject_and_project_match_oracle(case, dtype):
    n, angles, nz, nb, atten = case
    ang = angles_uniform(angles) if isinstance(angles, int) else np.asarray(angles)
    g = make_geometry(n, ang, n_bins=nb, nz=nz, atten=atten)
    P = Projector(g)
    plan = plan_for(n, list(ang), nz=nz, n_bins=nb, atten=atten, dtype=dtype)
    sino = uniform_field(g.sino_shape, 101)
    vol = signed_field(g.vol_shape, 102)
    bp = plan.backproject(to_gpu(sino, dtype)).double().cpu().numpy()
    fp = plan.project(to_gpu(vol, dtype)).double().cpu().numpy()
    bp_ref, fp_ref = P.backproject(sino), P.project(vol)
    if dtype == torch.float64:
        np.testing.assert_allclose(bp, bp_ref, rtol=F64_TOL, atol=F64_TOL * np.abs(bp_ref).max())
        np.testing.assert_allclose(fp, fp_ref, rtol=F64_TOL, atol=F64_TOL * np.abs(fp_ref).max())
    else:
        assert rel_norm(bp, bp_ref) < F32_NORM_TOL
        assert rel_norm(fp, fp_ref) < F32_NORM_TOL


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_autotuned_plan_matches_oracle(dtype):
    # the autotuner only changes work splits: outputs stay within the parity bound
    n, nz, na = 40, 24, 36
    ang = angles_uniform(na)
    g = make_geometry(n, ang, nz=nz, atten=1.0)
    P = Projector(g)
    plan = plan_for(n, list(ang), nz=nz, sigma=(1.0, 1.0, 1.5), dtype=dtype).autotune()
    vol = signed_field(g.vol_shape, 7)
    fp = plan.project(to_gpu(vol, dtype)).double().cpu().numpy()
    kb = plan.blur(to_gpu(vol, dtype)).double().cpu().numpy()
    kb_ref = oblur.apply(vol, oblur.psf_taps((1.0, 1.0, 1.5)))
    if dtype == torch.float64:
        np.testing.assert_allclose(fp, P.project(vol), rtol=F64_TOL, atol=F64_TOL * np.abs(fp).max())
        np.testing.assert_allclose(kb, kb_ref, rtol=F64_TOL, atol=F64_TOL * np.abs(kb_ref).max())
    else:
        assert rel_norm(fp, P.project(vol)) < F32_NORM_TOL
        assert rel_norm(kb, kb_ref) < F32_NORM_TOL


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adjoint_identity_on_gpu(dtype):
    n, nz = 96, 5
    plan = plan_for(n, 90, nz=nz, dtype=dtype)
    x = to_gpu(uniform_field(plan.vol_shape, 3), dtype)
    y = to_gpu(signed_field(plan.sino_shape, 4), dtype)
    lhs = float((plan.project(x).double() * y.double()).sum())
    rhs = float((x.double() * plan.backproject(y).double()).sum())
    scale = float(plan.project(x).double().norm() * y.double().norm())
    tol = 1e-13 if dtype == torch.float64 else 1e-6
    assert abs(lhs - rhs) <= tol * scale


def test_accumulate_flag_adds_to_output():
    plan = plan_for(32, 20, nz=2)
    s = to_gpu(uniform_field(plan.sino_shape, 8), torch.float32)
    v0 = to_gpu(uniform_field(plan.vol_shape, 9), torch.float32)
    base = plan.backproject(s)
    acc = plan.backproject(s, out=v0.clone(), accumulate=True)
    torch.testing.assert_close(acc, base + v0, rtol=1e-6, atol=1e-6)
    x = to_gpu(uniform_field(plan.vol_shape, 10), torch.float32)
    y0 = to_gpu(uniform_field(plan.sino_shape, 11), torch.float32)
    torch.testing.assert_close(plan.project(x, out=y0.clone(), accumulate=True), plan.project(x) + y0,
                               rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("sigma,shape", [((1.5, 1.5, 1.5), (37, 70, 70)), ((1.0, 1.0, 2.0), (9, 33, 33)),
                                         ((0.6, 2.4, 0.0), (5, 20, 20))])
def test_blur_matches_oracle(sigma, shape, dtype):
    nz, n, _ = shape
    plan = plan_for(n, 4, nz=nz, sigma=sigma, dtype=dtype)
    vol = uniform_field(shape, 12)
    got = plan.blur(to_gpu(vol, dtype)).double().cpu().numpy()
    want = oblur.apply(vol, oblur.psf_taps(sigma))
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    np.testing.assert_allclose(got, want, rtol=tol, atol=tol)


@pytest.mark.parametrize("w", [0.0, 2.0, 3.5, 10.0, math.inf])
def test_regions_match_oracle_2d(w):
    n = 96
    f = ellipses_target(n, 21)
    plan = plan_for(n, 8, dtype=torch.float32)
    got = plan.regions(to_gpu(f, torch.float32), band_width=w).cpu().numpy()
    want = oregions.labels(f, band_width=w)
    np.testing.assert_array_equal(got, want)


def test_regions_match_oracle_3d_with_psf():
    f = ellipsoids_target(40, 5, count=3, nz=24)
    sigma = (1.0, 1.0, 2.0)
    plan = plan_for(40, 8, nz=24, sigma=sigma, dtype=torch.float64)
    for w in (0.0, 1.5, 4.0):
        got = plan.regions(to_gpu(f, torch.float64), band_width=w).cpu().numpy()
        want = oregions.labels(f, band_width=w, taps=oblur.psf_taps(sigma))
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_active_rays_match_oracle(dtype):
    n = 64
    g = make_geometry(n, 60, atten=1.0)
    P = Projector(g)
    f = ellipses_target(n, 33)
    plan = plan_for(n, 60, dtype=dtype)
    got = plan.active_rays(to_gpu(f, dtype)).cpu().numpy().astype(bool)
    want = oregions.active_rays(P, f)
    pf = P.project(f)
    thr = 1e-6 * pf.max()
    decided = np.abs(pf - thr) > 1e-5 * thr          # rays not within rounding of the threshold
    np.testing.assert_array_equal(got[decided], want[decided])


def test_full_size_3d_projector_sampled_outputs():
    # 256^3 volume, 360 views, 256 x 256 detector rows, FP32: sampled outputs vs the oracle
    n, nz, na = 256, 256, 360
    g = make_geometry(n, na, nz=nz, atten=1.0)
    plan = plan_for(n, na, nz=nz, dtype=torch.float32)
    rng = np.random.default_rng(7)
    vol = uniform_field((nz, n, n), 3002).astype(np.float32)
    sino = uniform_field((na, nz, n), 3001).astype(np.float32)
    fp = plan.project(to_gpu(vol, torch.float32)).cpu().numpy()
    bp = plan.backproject(to_gpu(sino, torch.float32)).cpu().numpy()
    PT = slice_matrix(g)                                   # (n*n, na*n)
    # sampled detector bins: (angle, z, bin)
    ia, iz, ib = rng.integers(0, na, 3000), rng.integers(0, nz, 3000), rng.integers(0, n, 3000)
    cols = PT[:, ia * n + ib].tocsc()
    want = np.array([cols[:, k].T @ vol[iz[k]].reshape(-1).astype(np.float64) for k in range(3000)]).ravel()
    got = fp[ia, iz, ib]
    assert rel_norm(got, want) < F32_NORM_TOL
    # sampled voxels
    vz, vr, vc = rng.integers(0, nz, 3000), rng.integers(0, n, 3000), rng.integers(0, n, 3000)
    rows = PT[vr * n + vc]
    s64 = sino.astype(np.float64)
    want_b = np.array([rows[k] @ s64[:, vz[k], :].reshape(-1) for k in range(3000)]).ravel()
    assert rel_norm(bp[vz, vr, vc], want_b) < F32_NORM_TOL


# 3D FP32 cases whose slice counts allow the asynchronous projector (nz % 4 == 0)
VARIANT_CASES = [
    (48, 60, 20, None),     # view pairs
    (40, 37, 24, None),     # odd view count: no pairing
    (33, 90, 12, 35),       # ragged grid and detector, view pairs
]


@pytest.mark.parametrize("case", VARIANT_CASES)
def test_every_projector_and_blur_variant_matches_oracle(case):
    # each work split the autotuner can choose, pinned through sipo_plan_set_tuning
    from paper_2604_08997_amd import SipoError
    n, na, nz, nb = case
    ang = angles_uniform(na)
    g = make_geometry(n, ang, n_bins=nb, nz=nz, atten=1.0)
    P = Projector(g)
    sigma = (1.0, 1.0, 1.5)
    plan = plan_for(n, list(ang), nz=nz, n_bins=nb, sigma=sigma)
    vol = signed_field(g.vol_shape, 11)
    vol_d = to_gpu(vol, torch.float32)
    fp_ref = P.project(vol)
    kb_ref = oblur.apply(vol, oblur.psf_taps(sigma))
    default = plan.tuning()
    ran_async = 0
    for zc in (8, 16, 32, 64):
        for dma, skip, cm in [(0, 0, 2), (1, 0, 1), (1, 0, 2), (1, 1, 1), (1, 1, 2)]:
            try:
                plan.set_tuning(p3d_zc=zc, p3d_dma=dma, p3d_skip=skip, p3d_cm=cm)
            except SipoError as e:
                assert (dma == 1 and not default["p3d_dma"]) or (zc == 64 and (dma == 0 or cm == 2)), (zc, dma, e)
                continue
            assert plan.tuning()["p3d_zc"] == zc and plan.tuning()["p3d_cm"] == cm
            fp = plan.project(vol_d).double().cpu().numpy()
            assert rel_norm(fp, fp_ref) < F32_NORM_TOL, (zc, dma, skip, cm)
            ran_async += dma
    assert ran_async == 14 or not default["p3d_dma"]
    sino = uniform_field(g.sino_shape, 12)
    bp_ref = P.backproject(sino)
    for bzc in (4, 8, 16, 32):
        plan.set_tuning(bp3d_zc=bzc)
        bp = plan.backproject(to_gpu(sino, torch.float32)).double().cpu().numpy()
        assert rel_norm(bp, bp_ref) < F32_NORM_TOL, bzc
    for bzc in (0, 8, 16, 32):
        if bzc > nz:
            with pytest.raises(SipoError):
                plan.set_tuning(blur_zc=bzc)
            continue
        plan.set_tuning(blur_zc=bzc)
        kb = plan.blur(vol_d).double().cpu().numpy()
        assert rel_norm(kb, kb_ref) < F32_NORM_TOL, bzc


def test_set_tuning_rejects_invalid_settings():
    from paper_2604_08997_amd import SipoError
    p64 = plan_for(24, 20, nz=8, dtype=torch.float64)
    before = p64.tuning()
    for bad in [dict(p3d_zc=32), dict(p3d_zc=64), dict(p3d_zc=12), dict(p3d_dma=1), dict(p3d_cm=3),
                dict(p3d_skip=1, p3d_dma=0), dict(blur_zc=16), dict(bp3d_zc=32), dict(bp3d_zc=2)]:
        with pytest.raises(SipoError):
            p64.set_tuning(**bad)
        assert p64.tuning() == before
    with pytest.raises(ValueError):
        p64.set_tuning(zc=16)
    p32 = plan_for(24, 20, nz=64, dtype=torch.float32)
    before = p32.tuning()
    for bad in [dict(p3d_zc=64, p3d_dma=0, p3d_skip=0), dict(p3d_zc=64, p3d_dma=1, p3d_cm=2)]:
        with pytest.raises(SipoError):
            p32.set_tuning(**bad)
        assert p32.tuning() == before


def test_plan_workspace_is_caller_memory():
    # the standalone operators run in a workspace the caller attaches to the plan; without one they
    # fail before launching, and with one a first call allocates no device memory
    import ctypes as C
    from paper_2604_08997_amd import binding as B
    n, nz, na = 128, 128, 90
    ang = angles_uniform(na)
    g = make_geometry(n, ang, nz=nz, atten=1.0)
    # a small 3D plan first loads the kernels' code, so the measurement below sees only the call
    small = plan_for(24, list(angles_uniform(10)), nz=8, dtype=torch.float32)
    small.backproject(small.project(torch.ones(small.vol_shape, dtype=torch.float32, device=dev())))
    plan = plan_for(n, list(ang), nz=nz, dtype=torch.float32)
    L, h = B.lib(), plan.handle
    need = int(L.sipo_plan_workspace_size(h))
    vb, sb = 4 * n * n * nz, 4 * na * nz * n
    assert need >= vb + sb
    assert 0 < plan.device_bytes < 16 << 20
    vol = to_gpu(signed_field(g.vol_shape, 5), torch.float32)
    sino = torch.empty(g.sino_shape, dtype=torch.float32, device=dev())
    stream = B._stream()
    assert L.sipo_plan_set_workspace(h, None, 0) == B.SIPO_OK
    assert L.sipo_project(h, B._ptr(vol), B._ptr(sino), 0, stream) == B.SIPO_E_WORKSPACE
    assert L.sipo_backproject(h, B._ptr(sino), B._ptr(vol), 0, stream) == B.SIPO_E_WORKSPACE
    ws = plan.workspace
    assert L.sipo_plan_set_workspace(h, B._ptr(ws), C.c_size_t(need - 1)) == B.SIPO_E_WORKSPACE
    assert L.sipo_plan_set_workspace(h, C.c_void_p(ws.data_ptr() + 64), C.c_size_t(need - 64)) == B.SIPO_E_INVALID
    assert L.sipo_plan_set_workspace(h, B._ptr(ws), C.c_size_t(need)) == B.SIPO_OK
    out, bp = plan.empty_sino(), plan.empty_vol()     # outputs allocated before the measurement
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev())[0]
    plan.project(vol, out=out)
    plan.backproject(out, out=bp)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(dev())[0]
    # the workspace-less allocation this replaced took a volume plus a sinogram (about 14 MB here)
    assert free0 - free1 < (vb + sb) // 2, (free0, free1)
    P = Projector(g)
    assert rel_norm(out.double().cpu().numpy(), P.project(vol.double().cpu().numpy())) < F32_NORM_TOL
    assert rel_norm(bp.double().cpu().numpy(), P.backproject(out.double().cpu().numpy())) < F32_NORM_TOL

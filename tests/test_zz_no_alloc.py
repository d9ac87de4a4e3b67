"""Allocation-free metric evaluation (sipo_evaluate_noalloc) against sipo_evaluate.

Both calls run the same kernels in the same order, so their results must agree bit for bit;
the no-allocation call must work with no plan workspace attached and must not change the
device's free memory.  Two calls in a row, the second on a smaller volume, check that the
shared library-held scratch carries nothing over from one call to the next."""
import ctypes as C
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

RESIN = (0.02, 0.98, 6.0, 0.8, 1.1)   # synthetic resin constants (the paper prints none)


def dev():
    return torch.device("cuda", 0)


def same(a, b):
    return (math.isnan(a) and math.isnan(b)) or a == b


def inputs(p, seed, dtype):
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 3, size=p.vol_shape).astype(np.uint8)
    D = rng.uniform(0.6, 1.6, size=p.vol_shape)
    ftn = rng.uniform(0.9, 1.2, size=p.vol_shape)
    w = rng.uniform(0.2, 1.0, size=p.vol_shape)
    mt = rng.uniform(0.3, 0.9, size=p.vol_shape)
    t = lambda a: torch.as_tensor(a, dtype=dtype, device=dev())
    return torch.as_tensor(lab, device=dev()), t(D), t(ftn), t(w), t(mt)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_evaluate_noalloc_matches_evaluate(dtype):
    import paper_2604_08997_amd as sipo
    from paper_2604_08997_amd import binding as B
    # larger volume first, then a smaller one (fewer reduction workgroups than the first call left)
    for n, nz, seed in ((160, 40, 1), (24, 3, 2)):
        p = sipo.Plan(n, 8, nz=nz, dtype=dtype, device=dev())
        lab, D, ftn, w, mt = inputs(p, seed, dtype)
        kw = dict(f_target_norm=ftn, f_crit=0.8, weights=w, resin=RESIN, m_target=mt)
        ref = p.evaluate(D, lab, **kw)
        ref_plain = p.evaluate(D, lab, f_t_scalar=1.1)
        # no workspace attached: the ordinary call refuses, the allocation-free call runs
        assert B.lib().sipo_plan_set_workspace(p.handle, None, 0) == B.SIPO_OK
        with pytest.raises(B.SipoError) as e:
            p.evaluate(D, lab, **kw)
        assert e.value.code == B.SIPO_E_WORKSPACE
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(dev())[0]
        got = p.evaluate(D, lab, noalloc=True, **kw)
        got_plain = p.evaluate(D, lab, f_t_scalar=1.1, noalloc=True)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(dev())[0]
        assert free1 == free0, (free0, free1)
        for k in ref:
            assert same(got[k], ref[k]), (n, k, got[k], ref[k])
            assert same(got_plain[k], ref_plain[k]), (n, k, got_plain[k], ref_plain[k])
        assert math.isfinite(got["alpha_m"]) and math.isnan(got_plain["alpha_m"])
        assert got["n_gel"] == int((lab == 2).sum().item())
        assert B.lib().sipo_plan_set_workspace(p.handle, B._ptr(p.workspace), C.c_size_t(p.workspace.numel())) == 0


def test_evaluate_noalloc_rejects_bad_arguments():
    import paper_2604_08997_amd as sipo
    from paper_2604_08997_amd import binding as B
    p = sipo.Plan(16, 8, nz=1, dtype=torch.float64, device=dev())
    lab, D, ftn, w, mt = inputs(p, 3, torch.float64)
    with pytest.raises(B.SipoError) as e:
        p.evaluate(D, lab, f_t_scalar=-1.0, noalloc=True)
    assert e.value.code == B.SIPO_E_INVALID
    with pytest.raises(B.SipoError) as e:
        p.evaluate(D, lab, ftn, f_crit=0.0, noalloc=True)
    assert e.value.code == B.SIPO_E_INVALID

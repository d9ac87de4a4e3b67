"""ctypes binding of ``libsipo.so`` -- argument marshalling only.

Every operation runs in the library's HIP kernels; PyTorch supplies device
memory and the current stream.  If the library is not built, importing works
but every call raises ``SipoError`` (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsipo.so")

SIPO_OK, SIPO_E_INVALID, SIPO_E_DEVICE, SIPO_E_WORKSPACE, SIPO_E_UNSUPPORTED = 0, -1, -2, -3, -4
SIPO_F32, SIPO_F64 = 0, 1
PLAIN, RESTARTED = 0, 1
OPTIMAL, PRIMAL_INFEASIBLE, ITER_LIMIT, NUMERICAL = 0, 1, 2, 3
STATUS_NAMES = {OPTIMAL: "optimal", PRIMAL_INFEASIBLE: "infeasible", ITER_LIMIT: "iter_limit", NUMERICAL: "numerical"}


class SipoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sipo error {code}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("n", C.c_int32), ("nz", C.c_int32), ("n_angles", C.c_int32), ("n_bins", C.c_int32),
                ("angles", C.POINTER(C.c_double)), ("atten", C.c_double)]


class Psf(C.Structure):
    _fields_ = [("rx", C.c_int32), ("ry", C.c_int32), ("rz", C.c_int32),
                ("kx", C.POINTER(C.c_double)), ("ky", C.POINTER(C.c_double)), ("kz", C.POINTER(C.c_double))]


class Problem(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("labels", C.c_void_p), ("act", C.c_void_p),
                ("lo", C.c_void_p), ("hi", C.c_void_p), ("lo_scalar", C.c_double), ("hi_scalar", C.c_double),
                ("u_free", C.c_int32), ("v_free", C.c_int32), ("w1", C.c_double), ("w2", C.c_double),
                ("band_cap", C.c_double), ("y", C.c_void_p), ("lam_up", C.c_void_p), ("lam_lo", C.c_void_p),
                ("u0", C.c_double), ("v0", C.c_double), ("dose_out", C.c_void_p)]


class PdhgOptions(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_iters", C.c_int32), ("check_every", C.c_int32), ("tol", C.c_double),
                ("tau", C.c_double), ("sigma", C.c_double), ("power_iters", C.c_int32), ("eta", C.c_double),
                ("infeas_tol", C.c_double), ("use_graph", C.c_int32), ("profile", C.c_int32),
                ("scalar_weight", C.c_double), ("progress_every", C.c_int32), ("tune_operators", C.c_int32),
                ("op_config", C.c_int32 * 8), ("tiles_2d", C.c_int32 * 3)]

NUM_PHASES = 7
OP_KEYS = ("p_zc", "bp_zc", "bp_splits", "blur_zc", "p_queue", "p_fuse", "p_skip", "p_chunk")
TILE2D_KEYS = ("bp_tile_x", "bp_views", "fp_bins")
PHASES = ("project", "backproject", "blur", "transpose", "primal", "dual", "scalars")


class PdhgResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("restarts", C.c_int32),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("rel_primal", C.c_double), ("rel_dual", C.c_double), ("rel_gap", C.c_double),
                ("u", C.c_double), ("v", C.c_double), ("tau", C.c_double), ("sigma", C.c_double),
                ("omega", C.c_double), ("time_ms", C.c_double), ("loop_ms", C.c_double),
                ("phase_ms", C.c_double * NUM_PHASES), ("phase_launches", C.c_int32 * NUM_PHASES),
                ("op_config", C.c_int32 * 8), ("tiles_2d", C.c_int32 * 3)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if not k.startswith("phase_") and k not in ("op_config", "tiles_2d")}
        d["phase_ms"] = dict(zip(PHASES, list(self.phase_ms)))
        d["phase_launches"] = dict(zip(PHASES, list(self.phase_launches)))
        d["op_config"] = dict(zip(OP_KEYS, list(self.op_config)))
        d["tiles_2d"] = dict(zip(TILE2D_KEYS, list(self.tiles_2d)))
        return d


class Tuning(C.Structure):
    _fields_ = [("p3d_zc", C.c_int32), ("p3d_dma", C.c_int32), ("p3d_skip", C.c_int32), ("p3d_cm", C.c_int32),
                ("blur_zc", C.c_int32), ("bp3d_zc", C.c_int32)]


class Resin(C.Structure):
    _fields_ = [("alpha", C.c_double), ("k", C.c_double), ("beta", C.c_double), ("gamma", C.c_double),
                ("f0", C.c_double)]


class Metrics(C.Structure):
    _fields_ = [("dtvr", C.c_double), ("dsr", C.c_double), ("psr_f", C.c_double),
                ("gel_ratio_min", C.c_double), ("gel_ratio_max", C.c_double), ("band_max", C.c_double),
                ("gel_min", C.c_double), ("alpha_f", C.c_double), ("alpha_m", C.c_double), ("psr_m", C.c_double),
                ("dtvr_m", C.c_double), ("n_gel", C.c_int64), ("n_band", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes): every symbol declared in include/sipo.h
SIGNATURES = {
    "sipo_plan_create": (C.c_int, [C.POINTER(Geometry), C.POINTER(Psf), C.c_int, C.POINTER(C.c_void_p)]),
    "sipo_plan_destroy": (C.c_int, [C.c_void_p]),
    "sipo_plan_device_bytes": (C.c_size_t, [C.c_void_p]),
    "sipo_plan_workspace_size": (C.c_size_t, [C.c_void_p]),
    "sipo_plan_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "sipo_plan_autotune": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sipo_plan_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "sipo_plan_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "sipo_backproject": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "sipo_project": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "sipo_blur": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sipo_regions": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sipo_active_rays": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sipo_pdhg_workspace_size": (C.c_size_t, [C.POINTER(Problem), C.c_int32, C.POINTER(PdhgOptions)]),
    "sipo_pdhg_solve": (C.c_int, [C.POINTER(Problem), C.c_int32, C.POINTER(PdhgOptions), C.c_void_p, C.c_size_t,
                                  C.POINTER(PdhgResult), C.c_void_p]),
    "sipo_response": (C.c_int, [C.c_void_p, C.POINTER(Resin), C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "sipo_evaluate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                C.POINTER(Resin), C.c_void_p, C.c_double, C.POINTER(Metrics), C.c_void_p]),
    "sipo_evaluate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                        C.c_void_p, C.POINTER(Resin), C.c_void_p, C.c_double, C.POINTER(Metrics),
                                        C.c_void_p]),
    "sipo_last_error": (C.c_char_p, []),
    "sipo_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libsipo.so (once); raises SipoError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SipoError(SIPO_E_UNSUPPORTED, f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != SIPO_OK:
        raise SipoError(rc, lib().sipo_last_error().decode(errors="replace"))


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def gaussian_taps(sigma):
    """Normalised Gaussian taps with radius ceil(2 sigma) (identity for sigma <= 0)."""
    if sigma is None or sigma <= 0:
        return [1.0]
    r = int(math.ceil(2.0 * sigma))
    w = [math.exp(-(k * k) / (2.0 * sigma * sigma)) for k in range(-r, r + 1)]
    s = sum(w)
    return [v / s for v in w]


def _require(t: torch.Tensor, name, shape, dtype, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """Geometry + optional separable PSF + element type, bound to the current GPU."""

    def __init__(self, n, n_angles_or_angles, n_bins=None, nz=1, atten=1.0, sigma=None,
                 dtype=torch.float32, device=None):
        if isinstance(n_angles_or_angles, int):
            k = n_angles_or_angles
            angles = [2.0 * math.pi * i / k for i in range(k)]
        else:
            angles = [float(a) for a in n_angles_or_angles]
        self.n, self.nz = int(n), int(nz)
        self.n_bins = int(n if n_bins is None else n_bins)
        self.angles = angles
        self.n_angles = len(angles)
        self.atten = float(atten)
        self.dtype = dtype
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.sigma = sigma
        self._angles_c = (C.c_double * self.n_angles)(*angles)
        geom = Geometry(self.n, self.nz, self.n_angles, self.n_bins, self._angles_c, self.atten)
        psf_p = None
        if sigma is not None:
            sx, sy, sz = sigma
            tx, ty, tz = gaussian_taps(sx), gaussian_taps(sy), gaussian_taps(sz)
            self.taps = (tx, ty, tz)
            self._taps_c = [(C.c_double * len(t))(*t) for t in (tx, ty, tz)]
            psf = Psf((len(tx) - 1) // 2, (len(ty) - 1) // 2, (len(tz) - 1) // 2, *self._taps_c)
            psf_p = C.byref(psf)
        else:
            self.taps = None
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().sipo_plan_create(C.byref(geom), psf_p, SIPO_F64 if dtype == torch.float64 else SIPO_F32,
                                          C.byref(h)))
        self.handle = h
        # the operator workspace is caller memory: one torch buffer per plan, attached once
        need = int(lib().sipo_plan_workspace_size(h))
        self.workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().sipo_plan_set_workspace(h, _ptr(self.workspace), C.c_size_t(need)))

    @property
    def device_bytes(self):
        """Device bytes of the plan's own tables (the workspace is the separate ``workspace`` tensor)."""
        return int(lib().sipo_plan_device_bytes(self.handle))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            try:
                with torch.cuda.device(self.device):
                    _lib.sipo_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def vol_shape(self):
        return (self.nz, self.n, self.n)

    @property
    def sino_shape(self):
        return (self.n_angles, self.nz, self.n_bins)

    def empty_vol(self, dtype=None):
        return torch.empty(self.vol_shape, dtype=dtype or self.dtype, device=self.device)

    def empty_sino(self, dtype=None):
        return torch.empty(self.sino_shape, dtype=dtype or self.dtype, device=self.device)

    def autotune(self):
        """Time the plan's equivalent kernel variants and keep the fastest (synchronous)."""
        with torch.cuda.device(self.device):
            _check(lib().sipo_plan_autotune(self.handle, _stream()))
        return self

    def tuning(self):
        """The plan's work-split settings (dict of the sipo_tuning fields)."""
        t = Tuning()
        _check(lib().sipo_plan_get_tuning(self.handle, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def set_tuning(self, **fields):
        """Apply work-split settings; fields not given keep their current values."""
        cur = self.tuning()
        unknown = set(fields) - set(cur)
        if unknown:
            raise ValueError(f"unknown tuning fields {sorted(unknown)}")
        cur.update({k: int(v) for k, v in fields.items()})
        _check(lib().sipo_plan_set_tuning(self.handle, C.byref(Tuning(**cur))))
        return self

    # ------------------------------------------------------------ operators
    def backproject(self, sino, out=None, accumulate=False):
        _require(sino, "sino", self.sino_shape, self.dtype, self.device)
        out = self.empty_vol() if out is None else out
        _require(out, "out", self.vol_shape, self.dtype, self.device)
        _check(lib().sipo_backproject(self.handle, _ptr(sino), _ptr(out), int(bool(accumulate)), _stream()))
        return out

    def project(self, vol, out=None, accumulate=False):
        _require(vol, "vol", self.vol_shape, self.dtype, self.device)
        out = self.empty_sino() if out is None else out
        _require(out, "out", self.sino_shape, self.dtype, self.device)
        _check(lib().sipo_project(self.handle, _ptr(vol), _ptr(out), int(bool(accumulate)), _stream()))
        return out

    def blur(self, vol, out=None):
        _require(vol, "vol", self.vol_shape, self.dtype, self.device)
        out = self.empty_vol() if out is None else out
        _require(out, "out", self.vol_shape, self.dtype, self.device)
        _check(lib().sipo_blur(self.handle, _ptr(vol), _ptr(out), _stream()))
        return out

    def regions(self, f_target, band_width=10.0):
        _require(f_target, "f_target", self.vol_shape, self.dtype, self.device)
        lab = torch.empty(self.vol_shape, dtype=torch.uint8, device=self.device)
        scratch = torch.empty(self.vol_shape, dtype=torch.uint8, device=self.device)
        bw = -1.0 if band_width is None or math.isinf(band_width) else float(band_width)
        _check(lib().sipo_regions(self.handle, _ptr(f_target), bw, _ptr(lab), _ptr(scratch), _stream()))
        return lab

    def response(self, vol, resin, inverse=False, out=None):
        """M(vol) (Eq. 4) or M^-1(vol) (Eq. 5) with resin = (alpha, k, beta, gamma, f0)."""
        _require(vol, "vol", self.vol_shape, self.dtype, self.device)
        out = self.empty_vol() if out is None else out
        _require(out, "out", self.vol_shape, self.dtype, self.device)
        r = Resin(*[float(v) for v in resin])
        _check(lib().sipo_response(self.handle, C.byref(r), _ptr(vol), _ptr(out), int(bool(inverse)), _stream()))
        return out

    def evaluate(self, dose, labels, f_target_norm=None, f_t_scalar=1.0, f_crit=1.0, weights=None, resin=None,
                 m_target=None, m_t_scalar=float("nan"), noalloc=False):
        """Scale-invariant metrics and post-scaling factors of a normalised dose (Eq. 6-8, 25-28, 46).

        noalloc=True calls sipo_evaluate_noalloc (library-held scratch, no plan workspace)."""
        _require(dose, "dose", self.vol_shape, self.dtype, self.device)
        _require(labels, "labels", self.vol_shape, torch.uint8, self.device)
        for name, t in (("f_target_norm", f_target_norm), ("weights", weights), ("m_target", m_target)):
            if t is not None:
                _require(t, name, self.vol_shape, self.dtype, self.device)
        r = Resin(*[float(v) for v in resin]) if resin is not None else None
        m = Metrics()
        fn = lib().sipo_evaluate_noalloc if noalloc else lib().sipo_evaluate
        _check(fn(self.handle, _ptr(dose), _ptr(labels), _ptr(f_target_norm), float(f_t_scalar),
                                   float(f_crit), _ptr(weights), C.byref(r) if r is not None else None,
                                   _ptr(m_target), float(m_t_scalar), C.byref(m), _stream()))
        return m.as_dict()

    def active_rays(self, f_target, scratch=None):
        _require(f_target, "f_target", self.vol_shape, self.dtype, self.device)
        scratch = self.empty_sino() if scratch is None else scratch
        act = torch.empty(self.sino_shape, dtype=torch.uint8, device=self.device)
        _check(lib().sipo_active_rays(self.handle, _ptr(f_target), _ptr(scratch), _ptr(act), _stream()))
        return act


def version():
    return lib().sipo_version().decode()


# ------------------------------------------------------------------ LP solve
GENERAL, CASE1, CASE2 = 0, 1, 2


def target_levels(plan, f_target, labels):
    """Problem set-up (Sec. 2.5, 3.3) on the host: the smallest gel value of f_T, and a function
    c -> device array c f_T (the per-voxel bounds of a graded target) or None when f_T takes a
    single value on the gel (then scalar bounds are exact)."""
    import numpy as np
    f = f_target.detach().cpu().numpy()
    gel = labels.cpu().numpy() == 2
    if not gel.any():
        return 1.0, lambda c: None
    vals = f[gel].astype(np.float64)
    fmin = float(vals.min())
    if float(vals.max()) == fmin:
        return fmin, lambda c: None
    return fmin, lambda c: torch.as_tensor(c * f.astype(np.float64), dtype=plan.dtype, device=plan.device)


class LP:
    """One LP instance (Eq. 19-24 / 32-37 / 40-45) with its device state.

    Built by ``LP.build``: region labels and active rays come from the HIP
    kernels; normalisation follows Sec. 2.5-2.7 for a binary (or scalar-level)
    target: general f_crit = min gel f_T; Case 1 bounds [tol_lo, tol_hi] f_T
    with f_crit = tol_lo min f_T; Case 2 f_crit = cap min f_T and band cap 1.
    """

    def __init__(self, plan, labels, act, case, u_free, v_free, w1, w2, band_cap, lo, hi,
                 lo_arr=None, hi_arr=None, f_crit=1.0):
        self.plan, self.labels, self.act, self.case = plan, labels, act, case
        self.u_free, self.v_free, self.w1, self.w2, self.band_cap = u_free, v_free, w1, w2, band_cap
        self.lo, self.hi, self.lo_arr, self.hi_arr, self.f_crit = lo, hi, lo_arr, hi_arr, f_crit
        self.y = torch.zeros(plan.sino_shape, dtype=plan.dtype, device=plan.device)
        self.lam_up = torch.zeros(plan.vol_shape, dtype=plan.dtype, device=plan.device)
        self.lam_lo = torch.zeros(plan.vol_shape, dtype=plan.dtype, device=plan.device)
        self.u0 = 0.0
        self.v0 = 0.0
        self.dose = None

    @classmethod
    def build(cls, plan, f_target, case, band_width=10.0, w1=1.0, w2=1.0, tol_lo=0.9, tol_hi=1.0, cap=0.7,
              f_min=None):
        labels = plan.regions(f_target, band_width)
        act = plan.active_rays(f_target)
        fmin, level = target_levels(plan, f_target, labels)
        if f_min is not None:
            fmin = float(f_min)
        # graded targets carry per-voxel bounds (f_T / f_crit on the gel); single-level ones scalars
        if case == GENERAL:
            fc = fmin
            lo = hi = level(1.0 / fc)
            return cls(plan, labels, act, case, 1, 1, w1, w2, 1.0, fmin / fc, fmin / fc, lo_arr=lo, hi_arr=hi,
                       f_crit=fc)
        if case == CASE1:
            fc = tol_lo * fmin
            lo, hi = level(tol_lo / fc), level(tol_hi / fc)
            return cls(plan, labels, act, case, 1, 0, 1.0, 0.0, 1.0, tol_lo * fmin / fc, tol_hi * fmin / fc,
                       lo_arr=lo, hi_arr=hi, f_crit=fc)
        if case == CASE2:
            fc = cap * fmin
            lo = hi = level(1.0 / fc)
            return cls(plan, labels, act, case, 0, 1, 0.0, 1.0, 1.0, fmin / fc, fmin / fc, lo_arr=lo, hi_arr=hi,
                       f_crit=fc)
        raise ValueError(f"unknown case {case}")

    def c_struct(self, want_dose=False):
        if want_dose and self.dose is None:
            self.dose = self.plan.empty_vol()
        return Problem(self.plan.handle.value, self.labels.data_ptr(), self.act.data_ptr(),
                       self.lo_arr.data_ptr() if self.lo_arr is not None else None,
                       self.hi_arr.data_ptr() if self.hi_arr is not None else None,
                       float(self.lo), float(self.hi), int(self.u_free), int(self.v_free), float(self.w1),
                       float(self.w2), float(self.band_cap), self.y.data_ptr(), self.lam_up.data_ptr(),
                       self.lam_lo.data_ptr(), float(self.u0), float(self.v0),
                       self.dose.data_ptr() if (want_dose and self.dose is not None) else None)


def pdhg_options(mode=RESTARTED, max_iters=20000, check_every=64, tol=1e-4, tau=0.0, sigma=0.0, power_iters=100,
                 eta=0.95, infeas_tol=1e-6, use_graph=0, profile=0, scalar_weight=0.0, progress_every=0,
                 tune_operators=0, op_config=None, tiles_2d=None):
    """Solver options.  op_config fixes the masked 3D operators' work splits: a dict with any of the
    keys p_zc, bp_zc, bp_splits, blur_zc, p_queue, p_fuse, p_skip, p_chunk (as in a result's
    op_config) or an 8-sequence; 0 = free."""
    if op_config is None:
        oc = (0,) * len(OP_KEYS)
    elif isinstance(op_config, dict):
        unknown = set(op_config) - set(OP_KEYS)
        if unknown:
            raise ValueError(f"unknown op_config keys {sorted(unknown)}")
        oc = tuple(int(op_config.get(k, 0)) for k in OP_KEYS)
    else:
        oc = tuple(int(v) for v in op_config)
        if len(oc) != len(OP_KEYS):
            raise ValueError(f"op_config needs {len(OP_KEYS)} entries")
    if tiles_2d is None:
        t2 = (0, 0, 0)
    elif isinstance(tiles_2d, dict):
        unknown = set(tiles_2d) - set(TILE2D_KEYS)
        if unknown:
            raise ValueError(f"unknown tiles_2d keys {sorted(unknown)}")
        t2 = tuple(int(tiles_2d.get(k, 0)) for k in TILE2D_KEYS)
    else:
        t2 = tuple(int(v) for v in tiles_2d)
        if len(t2) != len(TILE2D_KEYS):
            raise ValueError(f"tiles_2d needs {len(TILE2D_KEYS)} entries")
    return PdhgOptions(int(mode), int(max_iters), int(check_every), float(tol), float(tau), float(sigma),
                       int(power_iters), float(eta), float(infeas_tol), int(use_graph), int(profile),
                       float(scalar_weight), int(progress_every), int(tune_operators), (C.c_int32 * 8)(*oc),
                       (C.c_int32 * 3)(*t2))


def solve(lps, opts=None, want_dose=True, workspace=None):
    """Solve one LP or a list of LPs on the current stream; returns result dicts."""
    single = isinstance(lps, LP)
    lps = [lps] if single else list(lps)
    opts = pdhg_options() if opts is None else opts
    arr = (Problem * len(lps))(*[lp.c_struct(want_dose) for lp in lps])
    need = lib().sipo_pdhg_workspace_size(arr, len(lps), C.byref(opts))
    dev = lps[0].plan.device
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(int(need), 1), dtype=torch.uint8, device=dev)
    res = (PdhgResult * len(lps))()
    _check(lib().sipo_pdhg_solve(arr, len(lps), C.byref(opts), C.c_void_p(workspace.data_ptr()),
                                 C.c_size_t(workspace.numel()), res, _stream()))
    out = [r.as_dict() for r in res]
    for d in out:
        d["status_name"] = STATUS_NAMES.get(d["status"], "?")
    return out[0] if single else out

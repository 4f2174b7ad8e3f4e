"""Python binding of ``libgsht.so`` (ctypes).  Argument marshalling only.

Every function takes torch tensors that live on the current HIP device and
passes their device pointers and torch's current stream to the C ABI declared
in ``include/gsht.h``; all arithmetic runs in the library's HIP kernels.  If the
library is missing or cannot be loaded, importing this module raises.

Layouts (see the header): a_lm [ncomp][nalm] complex (m-major triangular),
maps [ncomp][npts] real, theta/phi float64.  Precision "f64" -> complex128 /
float64, "f32" -> complex64 / float32.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsht.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libgsht.so not found at %s; build it with "
                      "`python -m paper_2304_10431_amd.build`" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

GSHT_OK, GSHT_EINVAL, GSHT_ENOMEM, GSHT_EHIP, GSHT_EUNSUPPORTED = 0, -1, -2, -3, -4
F64, F32 = 0, 1
_PREC = {"f64": F64, "f32": F32, F64: F64, F32: F32}
_CDT = {F64: torch.complex128, F32: torch.complex64}
_RDT = {F64: torch.float64, F32: torch.float32}


class GshtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("gsht status %d: %s" % (code, msg))
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int), ("mmax", ctypes.c_int), ("spin", ctypes.c_int),
                ("ncomp", ctypes.c_int), ("npts", ctypes.c_int64), ("epsilon", ctypes.c_double),
                ("precision", ctypes.c_int), ("ntheta", ctypes.c_int), ("ndouble", ctypes.c_int),
                ("n1", ctypes.c_int), ("n2", ctypes.c_int), ("w", ctypes.c_int),
                ("beta", ctypes.c_double), ("nrows", ctypes.c_int), ("a_min", ctypes.c_int),
                ("tile1", ctypes.c_int), ("tile2", ctypes.c_int), ("ntile1", ctypes.c_int),
                ("ntile2", ctypes.c_int), ("nchunks", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("column_mode", ctypes.c_int),
                ("spread_colors", ctypes.c_int), ("syn_r", ctypes.c_int), ("adj_r", ctypes.c_int),
                ("adj_b", ctypes.c_int), ("sigma", ctypes.c_double), ("cell_sort", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp, _i, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "gsht_synth_general": [_vp, _i, _i, _i, _vp, _vp, _i64, _d, _i, _vp, _vp],
    "gsht_adjoint_synth_general": [_vp, _i, _i, _i, _vp, _vp, _i64, _d, _i, _vp, _vp],
    "gsht_plan_create": [ctypes.POINTER(_vp), _i, _i, _i, _vp, _vp, _i64, _d, _i, _vp],
    "gsht_plan_create_sigma": [ctypes.POINTER(_vp), _i, _i, _i, _vp, _vp, _i64, _d, _i, _d, _vp],
    "gsht_plan_create_tuned": [ctypes.POINTER(_vp), _i, _i, _i, _vp, _vp, _i64, _d, _i, _vp],
    "gsht_plan_set_points": [_vp, _vp, _vp, _i64, _vp],
    "gsht_plan_synth": [_vp, _vp, _vp, _vp],
    "gsht_plan_adjoint": [_vp, _vp, _vp, _vp],
    "gsht_plan_synth_grad": [_vp, _vp, _vp, _vp],
    "gsht_plan_synth_many": [_vp, _i, _vp, _vp, _vp],
    "gsht_plan_adjoint_many": [_vp, _i, _vp, _vp, _vp],
    "gsht_plan_autotune": [_vp, _vp],
    "gsht_plan_adjoint_grad": [_vp, _vp, _vp, _vp],
    "gsht_plan_synth_deriv": [_vp, _vp, _vp, _vp, _vp, _vp],
    "gsht_plan_synth_vjp": [_vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "gsht_plan_adjoint_vjp": [_vp, _vp, _vp, _vp],
    "gsht_plan_get_info": [_vp, ctypes.POINTER(PlanInfo)],
    "gsht_plan_get_sort": [_vp, _vp, _vp, _vp],
    "gsht_plan_set_profiling": [_vp, _i],
    "gsht_plan_get_stage_times": [_vp, ctypes.POINTER(_d), ctypes.POINTER(_i64), _i],
    "gsht_legendre_rings": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "gsht_legendre_rings_adjoint": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "gsht_legendre_rings_adjoint_noalloc": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "gsht_deflect": [_vp, _vp, _vp, _i, _i64, _vp, _vp, _vp, _vp],
    "gsht_deflect_vjp": [_vp, _vp, _i, _i64, _vp, _vp, _vp, _vp, _vp],
    "gsht_spin_phase": [_vp, _vp, _i, _i, _i, _i64, _vp],
    "gsht_spin_phase_vjp": [_vp, _vp, _vp, _i, _i, _i64, _vp, _vp, _vp],
    "gsht_alm_lscale": [_vp, _vp, _i, _i, _i, _i, _vp],
    "gsht_map_weight": [_vp, _vp, _i, _i64, _i, _vp, _vp],
    "gsht_alm_lfactor": [_vp, _vp, _i, _i, _i, _i, _i, _vp],
    "gsht_magnification": [_vp, _vp, _vp, _vp, _i, _i64, _vp, _vp],
    "gsht_analysis_minimal": [_vp, _i, _i, _i, _i, _i, _vp, _vp],
    "gsht_batch_create": [ctypes.POINTER(_vp), _i],
    "gsht_batch_synth": [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp],
    "gsht_batch_adjoint": [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp],
    "gsht_num_stages": [],
    "gsht_stage_name": [_i],
    "gsht_last_error": [],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.gsht_last_error.restype = ctypes.c_char_p
_lib.gsht_stage_name.restype = ctypes.c_char_p
_lib.gsht_plan_destroy.argtypes = [_vp]
_lib.gsht_plan_destroy.restype = None
_lib.gsht_batch_destroy.argtypes = [_vp]
_lib.gsht_batch_destroy.restype = None

EXPORTED = list(_SIGS) + ["gsht_plan_destroy", "gsht_batch_destroy"]


def _check(rc: int):
    if rc != GSHT_OK:
        raise GshtError(rc, _lib.gsht_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on a HIP device" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def _coords(theta, phi):
    _need(theta, torch.float64, None, "theta")
    _need(phi, torch.float64, tuple(theta.shape), "phi")
    return theta.numel()


def synth_general(alm, theta, phi, lmax: int, mmax: int, spin: int, epsilon: float,
                  precision="f64", out=None):
    """One-shot gsht_synth_general; returns the map [ncomp][npts]."""
    prec = _PREC[precision]
    ncomp = 1 if spin == 0 else 2
    npts = _coords(theta, phi)
    _need(alm, _CDT[prec], (ncomp, nalm(lmax, mmax)), "alm")
    if out is None:
        out = torch.empty((ncomp, npts), dtype=_RDT[prec], device=alm.device)
    _need(out, _RDT[prec], (ncomp, npts), "out")
    _check(_lib.gsht_synth_general(_ptr(alm), lmax, mmax, spin, _ptr(theta), _ptr(phi), npts,
                                   float(epsilon), prec, _ptr(out), _stream()))
    return out


def adjoint_synth_general(maps, theta, phi, lmax: int, mmax: int, spin: int, epsilon: float,
                          precision="f64", out=None):
    """One-shot gsht_adjoint_synth_general; returns a_lm [ncomp][nalm]."""
    prec = _PREC[precision]
    ncomp = 1 if spin == 0 else 2
    npts = _coords(theta, phi)
    _need(maps, _RDT[prec], (ncomp, npts), "map")
    if out is None:
        out = torch.empty((ncomp, nalm(lmax, mmax)), dtype=_CDT[prec], device=maps.device)
    _need(out, _CDT[prec], (ncomp, nalm(lmax, mmax)), "out")
    _check(_lib.gsht_adjoint_synth_general(_ptr(maps), lmax, mmax, spin, _ptr(theta), _ptr(phi),
                                           npts, float(epsilon), prec, _ptr(out), _stream()))
    return out


class Plan:
    """gsht_plan wrapper: geometry, FFT plans and workspace reused across calls."""

    def __init__(self, theta, phi, lmax: int, mmax: int, spin: int, epsilon: float,
                 precision="f64", sigma=None):
        """sigma: None for the default oversampling (2), a number (2, 1.5 or 1.25) for
        gsht_plan_create_sigma, or "tuned" for gsht_plan_create_tuned."""
        self.prec = _PREC[precision]
        self.lmax, self.mmax, self.spin = lmax, mmax, spin
        self.ncomp = 1 if spin == 0 else 2
        self.npts = _coords(theta, phi)
        self.device = theta.device
        h = ctypes.c_void_p(0)
        args = (ctypes.byref(h), lmax, mmax, spin, _ptr(theta), _ptr(phi), self.npts,
                float(epsilon), self.prec)
        if sigma is None:
            _check(_lib.gsht_plan_create(*args, _stream()))
        elif sigma == "tuned":
            _check(_lib.gsht_plan_create_tuned(*args, _stream()))
        else:
            _check(_lib.gsht_plan_create_sigma(*args, float(sigma), _stream()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gsht_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_points(self, theta, phi):
        """Move the plan to new points (at most as many as it was created with); only
        the bin sort is redone."""
        npts = _coords(theta, phi)
        _check(_lib.gsht_plan_set_points(self._h, _ptr(theta), _ptr(phi), npts, _stream()))
        self.npts = npts

    def info(self) -> dict:
        inf = PlanInfo()
        _check(_lib.gsht_plan_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def synth(self, alm, out=None):
        _need(alm, _CDT[self.prec], (self.ncomp, nalm(self.lmax, self.mmax)), "alm")
        if out is None:
            out = torch.empty((self.ncomp, self.npts), dtype=_RDT[self.prec], device=self.device)
        _need(out, _RDT[self.prec], (self.ncomp, self.npts), "out")
        _check(_lib.gsht_plan_synth(self._h, _ptr(alm), _ptr(out), _stream()))
        return out

    def adjoint(self, maps, out=None):
        _need(maps, _RDT[self.prec], (self.ncomp, self.npts), "map")
        if out is None:
            out = torch.empty((self.ncomp, nalm(self.lmax, self.mmax)), dtype=_CDT[self.prec],
                              device=self.device)
        _need(out, _CDT[self.prec], (self.ncomp, nalm(self.lmax, self.mmax)), "out")
        _check(_lib.gsht_plan_adjoint(self._h, _ptr(maps), _ptr(out), _stream()))
        return out

    def autotune(self):
        """Time the Legendre launch shapes on this plan and keep the fastest; returns
        (syn_r, adj_r, adj_b)."""
        _check(_lib.gsht_plan_autotune(self._h, _stream()))
        inf = self.info()
        return inf["syn_r"], inf["adj_r"], inf["adj_b"]

    def synth_many(self, alm, out=None):
        """Several maps on the plan's points: alm [nmaps][ncomp][nalm] -> [nmaps][ncomp][npts]."""
        nm = alm.shape[0]
        _need(alm, _CDT[self.prec], (nm, self.ncomp, nalm(self.lmax, self.mmax)), "alm")
        if out is None:
            out = torch.empty((nm, self.ncomp, self.npts), dtype=_RDT[self.prec], device=self.device)
        _need(out, _RDT[self.prec], (nm, self.ncomp, self.npts), "out")
        _check(_lib.gsht_plan_synth_many(self._h, nm, _ptr(alm), _ptr(out), _stream()))
        return out

    def adjoint_many(self, maps, out=None):
        """Adjoint of several maps on the plan's points: [nmaps][ncomp][npts] -> [nmaps][ncomp][nalm]."""
        nm = maps.shape[0]
        _need(maps, _RDT[self.prec], (nm, self.ncomp, self.npts), "maps")
        if out is None:
            out = torch.empty((nm, self.ncomp, nalm(self.lmax, self.mmax)), dtype=_CDT[self.prec],
                              device=self.device)
        _need(out, _CDT[self.prec], (nm, self.ncomp, nalm(self.lmax, self.mmax)), "out")
        _check(_lib.gsht_plan_adjoint_many(self._h, nm, _ptr(maps), _ptr(out), _stream()))
        return out

    def synth_grad(self, glm, out=None):
        """Gradient-only synthesis (C = 0): glm [1][nalm] -> map [2][npts]."""
        _need(glm, _CDT[self.prec], (1, nalm(self.lmax, self.mmax)), "glm")
        if out is None:
            out = torch.empty((self.ncomp, self.npts), dtype=_RDT[self.prec], device=self.device)
        _need(out, _RDT[self.prec], (self.ncomp, self.npts), "out")
        _check(_lib.gsht_plan_synth_grad(self._h, _ptr(glm), _ptr(out), _stream()))
        return out

    def adjoint_grad(self, maps, out=None):
        """Gradient part of the adjoint: map [2][npts] -> G [1][nalm]."""
        _need(maps, _RDT[self.prec], (self.ncomp, self.npts), "map")
        if out is None:
            out = torch.empty((1, nalm(self.lmax, self.mmax)), dtype=_CDT[self.prec],
                              device=self.device)
        _need(out, _CDT[self.prec], (1, nalm(self.lmax, self.mmax)), "out")
        _check(_lib.gsht_plan_adjoint_grad(self._h, _ptr(maps), _ptr(out), _stream()))
        return out

    def synth_deriv(self, alm, want_map=True):
        """(map or None, d map/d theta, d map/d phi), each [ncomp][npts]."""
        _need(alm, _CDT[self.prec], (self.ncomp, nalm(self.lmax, self.mmax)), "alm")
        shape = (self.ncomp, self.npts)
        mk = lambda: torch.empty(shape, dtype=_RDT[self.prec], device=self.device)
        m = mk() if want_map else None
        dth, dph = mk(), mk()
        _check(_lib.gsht_plan_synth_deriv(self._h, _ptr(alm), _ptr(m), _ptr(dth), _ptr(dph),
                                          _stream()))
        return m, dth, dph

    def synth_vjp(self, alm, gmap, want_alm=True, want_theta=True, want_phi=True):
        """Gradients (galm, gtheta, gphi) of a real loss with dL/dmap = gmap; entries not
        asked for are None."""
        _need(gmap, _RDT[self.prec], (self.ncomp, self.npts), "gmap")
        if want_theta or want_phi:
            _need(alm, _CDT[self.prec], (self.ncomp, nalm(self.lmax, self.mmax)), "alm")
        galm = (torch.empty((self.ncomp, nalm(self.lmax, self.mmax)), dtype=_CDT[self.prec],
                            device=self.device) if want_alm else None)
        gth = torch.empty(self.npts, dtype=torch.float64, device=self.device) if want_theta else None
        gph = torch.empty(self.npts, dtype=torch.float64, device=self.device) if want_phi else None
        if want_alm or want_theta or want_phi:
            _check(_lib.gsht_plan_synth_vjp(self._h, _ptr(alm), _ptr(gmap), _ptr(galm), _ptr(gth),
                                            _ptr(gph), _stream()))
        return galm, gth, gph

    def adjoint_vjp(self, galm):
        """dL/dmap of a real loss of the adjoint's output, given galm = dL/dalm."""
        _need(galm, _CDT[self.prec], (self.ncomp, nalm(self.lmax, self.mmax)), "galm")
        out = torch.empty((self.ncomp, self.npts), dtype=_RDT[self.prec], device=self.device)
        _check(_lib.gsht_plan_adjoint_vjp(self._h, _ptr(galm), _ptr(out), _stream()))
        return out

    def sort(self):
        inf = self.info()
        perm = torch.empty(max(self.npts, 1), dtype=torch.int32, device=self.device)
        start = torch.empty(inf["ntile1"] * inf["ntile2"] + 1, dtype=torch.int32, device=self.device)
        _check(_lib.gsht_plan_get_sort(self._h, _ptr(perm), _ptr(start), _stream()))
        return perm[:self.npts], start

    def set_profiling(self, on: bool):
        _check(_lib.gsht_plan_set_profiling(self._h, 1 if on else 0))

    def stage_times(self) -> dict:
        n = _lib.gsht_num_stages()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(_lib.gsht_plan_get_stage_times(self._h, ms, cnt, n))
        return {_lib.gsht_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}


class Batch:
    """Independent instances (plans of any lmax, spin, point count and precision) run
    over ``nstreams`` worker streams of the library (gsht_batch_*): instance i on
    worker i mod nstreams, after the work queued on torch's current stream, which then
    waits for all of them.  A batch call can be captured in a graph."""

    def __init__(self, nstreams: int = 4):
        h = _vp()
        _check(_lib.gsht_batch_create(ctypes.byref(h), nstreams))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.gsht_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _arr(xs):
        return (_vp * max(len(xs), 1))(*[x if isinstance(x, _vp) else _vp(x) for x in xs])

    def synth(self, plans, alms, outs=None):
        """alms[i] -> maps[i] with plans[i]; returns the list of maps."""
        if outs is None:
            outs = [torch.empty((p.ncomp, p.npts), dtype=_RDT[p.prec], device=p.device) for p in plans]
        for p, a, o in zip(plans, alms, outs):
            _need(a, _CDT[p.prec], (p.ncomp, nalm(p.lmax, p.mmax)), "alm")
            _need(o, _RDT[p.prec], (p.ncomp, p.npts), "out")
        _check(_lib.gsht_batch_synth(self._h, len(plans), self._arr([p._h.value for p in plans]),
                                     self._arr([_ptr(a) for a in alms]),
                                     self._arr([_ptr(o) for o in outs]), _stream()))
        return outs

    def adjoint(self, plans, maps, outs=None):
        """maps[i] -> alms[i] with plans[i]; returns the list of coefficient arrays."""
        if outs is None:
            outs = [torch.empty((p.ncomp, nalm(p.lmax, p.mmax)), dtype=_CDT[p.prec], device=p.device)
                    for p in plans]
        for p, m, o in zip(plans, maps, outs):
            _need(m, _RDT[p.prec], (p.ncomp, p.npts), "map")
            _need(o, _CDT[p.prec], (p.ncomp, nalm(p.lmax, p.mmax)), "out")
        _check(_lib.gsht_batch_adjoint(self._h, len(plans), self._arr([p._h.value for p in plans]),
                                       self._arr([_ptr(m) for m in maps]),
                                       self._arr([_ptr(o) for o in outs]), _stream()))
        return outs


def legendre_rings(alm, lmax: int, mmax: int, spin: int, ntheta: int, precision="f64", out=None):
    """Stage entry point gsht_legendre_rings; returns F [ncol][2 ntheta - 2] complex."""
    prec = _PREC[precision]
    ncomp = 1 if spin == 0 else 2
    ncol = mmax + 1 if spin == 0 else 2 * mmax + 1
    _need(alm, _CDT[prec], (ncomp, nalm(lmax, mmax)), "alm")
    if out is None:
        out = torch.empty((ncol, 2 * ntheta - 2), dtype=_CDT[prec], device=alm.device)
    _need(out, _CDT[prec], (ncol, 2 * ntheta - 2), "F")
    _check(_lib.gsht_legendre_rings(_ptr(alm), lmax, mmax, spin, ntheta, prec, _ptr(out), _stream()))
    return out


def legendre_rings_adjoint(F, lmax: int, mmax: int, spin: int, ntheta: int, precision="f64",
                           out=None):
    """Stage entry point gsht_legendre_rings_adjoint; returns a_lm [ncomp][nalm]."""
    prec = _PREC[precision]
    ncomp = 1 if spin == 0 else 2
    ncol = mmax + 1 if spin == 0 else 2 * mmax + 1
    _need(F, _CDT[prec], (ncol, 2 * ntheta - 2), "F")
    if out is None:
        out = torch.empty((ncomp, nalm(lmax, mmax)), dtype=_CDT[prec], device=F.device)
    _need(out, _CDT[prec], (ncomp, nalm(lmax, mmax)), "alm")
    _check(_lib.gsht_legendre_rings_adjoint(_ptr(F), lmax, mmax, spin, ntheta, prec, _ptr(out),
                                            _stream()))
    return out


def legendre_rings_adjoint_noalloc(F, lmax: int, mmax: int, spin: int, ntheta: int, out,
                                   precision="f64"):
    """Allocation-free stage entry point gsht_legendre_rings_adjoint_noalloc: the same
    result as legendre_rings_adjoint, written into the caller's ``out``
    [ncomp][nalm]; the library allocates nothing (its tables live in a fixed device
    scratch array shared by all calls on the device)."""
    prec = _PREC[precision]
    ncomp = 1 if spin == 0 else 2
    ncol = mmax + 1 if spin == 0 else 2 * mmax + 1
    _need(F, _CDT[prec], (ncol, 2 * ntheta - 2), "F")
    _need(out, _CDT[prec], (ncomp, nalm(lmax, mmax)), "alm")
    _check(_lib.gsht_legendre_rings_adjoint_noalloc(_ptr(F), lmax, mmax, spin, ntheta, prec,
                                                    _ptr(out), _stream()))
    return out


def _prec_of(t):
    if t.dtype in (torch.float64, torch.complex128):
        return F64
    if t.dtype in (torch.float32, torch.complex64):
        return F32
    raise TypeError("unsupported dtype %s" % t.dtype)


def deflect(theta, phi, alpha, want_chi=True):
    """gsht_deflect: deflected positions (theta', phi') and the spin phase chi (or None)
    for a deflection field alpha [2][npts] (alpha_theta, alpha_phi)."""
    npts = _coords(theta, phi)
    prec = _prec_of(alpha)
    _need(alpha, _RDT[prec], (2, npts), "alpha")
    tho = torch.empty_like(theta)
    pho = torch.empty_like(phi)
    chi = torch.empty_like(theta) if want_chi else None
    _check(_lib.gsht_deflect(_ptr(theta), _ptr(phi), _ptr(alpha), prec, npts, _ptr(tho), _ptr(pho),
                             _ptr(chi), _stream()))
    return tho, pho, chi


def deflect_vjp(theta, alpha, g_theta=None, g_phi=None, g_chi=None):
    """gsht_deflect_vjp: gradient with respect to alpha [2][npts] from the gradients with
    respect to theta', phi' and chi (each [npts] FP64 or None)."""
    _need(theta, torch.float64, None, "theta")
    npts = theta.numel()
    prec = _prec_of(alpha)
    _need(alpha, _RDT[prec], (2, npts), "alpha")
    for name, g in (("g_theta", g_theta), ("g_phi", g_phi), ("g_chi", g_chi)):
        if g is not None:
            _need(g, torch.float64, (npts,), name)
    out = torch.empty_like(alpha)
    _check(_lib.gsht_deflect_vjp(_ptr(theta), _ptr(alpha), prec, npts, _ptr(g_theta), _ptr(g_phi),
                                 _ptr(g_chi), _ptr(out), _stream()))
    return out


def spin_phase(maps, chi, spin: int, sign: int):
    """In place: (Q + iU) <- e^{i sign spin chi} (Q + iU); returns maps."""
    prec = _prec_of(maps)
    _need(chi, torch.float64, None, "chi")
    npts = chi.numel()
    _need(maps, _RDT[prec], (2, npts), "map")
    _check(_lib.gsht_spin_phase(_ptr(maps), _ptr(chi), spin, sign, prec, npts, _stream()))
    return maps


def spin_phase_vjp(gmap, lensed, chi, spin: int, want_chi=True):
    """(dL/dP, dL/dchi) for M = e^{i spin chi} P, given gmap = dL/dM and M."""
    prec = _prec_of(gmap)
    _need(chi, torch.float64, None, "chi")
    npts = chi.numel()
    _need(gmap, _RDT[prec], (2, npts), "gmap")
    if want_chi:
        _need(lensed, _RDT[prec], (2, npts), "lensed")
    g_unrot = torch.empty_like(gmap)
    g_chi = torch.empty_like(chi) if want_chi else None
    _check(_lib.gsht_spin_phase_vjp(_ptr(gmap), _ptr(lensed if want_chi else None), _ptr(chi), spin,
                                    prec, npts, _ptr(g_unrot), _ptr(g_chi), _stream()))
    return g_unrot, g_chi


def map_weight(maps, weights, out=None):
    """weights[i] * maps[c][i] (quadrature weights)."""
    prec = _prec_of(maps)
    ncomp, npts = maps.shape
    _need(maps, _RDT[prec], (ncomp, npts), "map")
    _need(weights, torch.float64, (npts,), "weights")
    if out is None:
        out = torch.empty_like(maps)
    _need(out, _RDT[prec], (ncomp, npts), "out")
    _check(_lib.gsht_map_weight(_ptr(maps), _ptr(weights), ncomp, npts, prec, _ptr(out), _stream()))
    return out


def alm_lscale(alm, lmax: int, mmax: int, out=None):
    """sqrt(l (l + 1)) times every coefficient of alm [ncomp][nalm]."""
    prec = _prec_of(alm)
    ncomp = alm.shape[0]
    _need(alm, _CDT[prec], (ncomp, nalm(lmax, mmax)), "alm")
    if out is None:
        out = torch.empty_like(alm)
    _need(out, _CDT[prec], (ncomp, nalm(lmax, mmax)), "out")
    _check(_lib.gsht_alm_lscale(_ptr(alm), _ptr(out), lmax, mmax, ncomp, prec, _stream()))
    return out


def analysis_minimal(maps, lmax: int, mmax: int, spin: int, out=None):
    """gsht_analysis_minimal: maps [ncomp][lmax + 2][nphi] on the minimal equiangular grid
    -> a_lm [ncomp][nalm]."""
    prec = _prec_of(maps)
    ncomp = 1 if spin == 0 else 2
    if maps.dim() != 3 or maps.shape[0] != ncomp or maps.shape[1] != lmax + 2:
        raise ValueError("map must have shape (%d, %d, nphi)" % (ncomp, lmax + 2))
    _need(maps, _RDT[prec], None, "map")
    if out is None:
        out = torch.empty((ncomp, nalm(lmax, mmax)), dtype=_CDT[prec], device=maps.device)
    _need(out, _CDT[prec], (ncomp, nalm(lmax, mmax)), "out")
    _check(_lib.gsht_analysis_minimal(_ptr(maps), lmax, mmax, spin, maps.shape[2], prec, _ptr(out),
                                      _stream()))
    return out


def alm_lfactor(alm, lmax: int, mmax: int, kind: int, out=None):
    """f_l times every coefficient (kind 0: sqrt(l(l+1)), 1: l(l+1)/2,
    2: sqrt((l-1)l(l+1)(l+2))/2)."""
    prec = _prec_of(alm)
    ncomp = alm.shape[0]
    _need(alm, _CDT[prec], (ncomp, nalm(lmax, mmax)), "alm")
    if out is None:
        out = torch.empty_like(alm)
    _need(out, _CDT[prec], (ncomp, nalm(lmax, mmax)), "out")
    _check(_lib.gsht_alm_lfactor(_ptr(alm), _ptr(out), lmax, mmax, ncomp, kind, prec, _stream()))
    return out


def magnification(alpha, kappa, gamma, omega=None):
    """|A| [npts] FP64 from alpha [2][npts], kappa [npts], gamma [2][npts] (omega [npts])."""
    prec = _prec_of(alpha)
    npts = alpha.shape[1]
    _need(alpha, _RDT[prec], (2, npts), "alpha")
    _need(kappa, _RDT[prec], None, "kappa")
    _need(gamma, _RDT[prec], (2, npts), "gamma")
    if kappa.numel() != npts or (omega is not None and omega.numel() != npts):
        raise ValueError("kappa/omega must have npts entries")
    if omega is not None:
        _need(omega, _RDT[prec], None, "omega")
    det = torch.empty(npts, dtype=torch.float64, device=alpha.device)
    _check(_lib.gsht_magnification(_ptr(alpha), _ptr(kappa), _ptr(omega), _ptr(gamma), prec, npts,
                                   _ptr(det), _stream()))
    return det


def last_error() -> str:
    return _lib.gsht_last_error().decode()

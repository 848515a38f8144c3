"""MI355X (gfx950) hot path of the one-step photo-switching optoacoustic
reconstruction (arXiv 2510.23739): A = H S, its adjoint, the regulariser's
proximal maps and the FISTA solver, as HIP kernels behind the C ABI of
include/psoam.h.  This module only marshals torch tensors into that ABI;
every step of the path runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import PREC, PsoamError, check, load

__all__ = ["Plan", "prox_l1", "A", "PREC", "PsoamError", "load"]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _check_f32(t, shape, name):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """A reconstruction geometry bound to the GPU: owns the packed impulse
    response and the padded operand buffers (see psoam_plan_create)."""

    def __init__(self, nx: int, ny: int, nz: int, n_pulses: int, nt: int, f: int,
                 phi: np.ndarray, species, t0: np.ndarray, taps: np.ndarray,
                 prec: str = "fp32", stream=None, separable: bool = False, tune: bool = False):
        """tune: choose the band kernels' launch shape by measurement
        (psoam_plan_create_tuned); what was chosen is in self.tune_report."""
        lib = load()
        species_a, species_b, species_tau = list(species.a), list(species.b), list(species.tau)
        ns = len(species_a)
        phi = np.ascontiguousarray(phi, dtype=np.float32)
        per_voxel = 1 if phi.ndim == 3 else 0
        self.geom = _lib.Geom(nx, ny, nz, ns, n_pulses, nt, f, per_voxel, 1 if separable else 0)
        sp = _lib.Species()
        for s in range(ns):
            sp.a[s], sp.b[s], sp.tau[s] = species_a[s], species_b[s], species_tau[s]
        sp.gamma = float(species.gamma)
        self._t0 = np.ascontiguousarray(t0, dtype=np.int32)
        self._taps = np.ascontiguousarray(taps, dtype=np.float32)
        if self._t0.shape != (nz, f, f) or self._taps.shape[:3] != (nz, f, f):
            raise ValueError("impulse-response table shape does not match (nz, f, f)")
        handle = C.c_void_p()
        self._h = None
        args = (C.byref(self.geom), C.byref(sp), phi.ctypes.data_as(C.c_void_p),
                self._t0.ctypes.data_as(C.c_void_p), self._taps.ctypes.data_as(C.c_void_p),
                int(self._taps.shape[3]), PREC[prec], _stream(stream), C.byref(handle))
        self.tune_report = None
        if tune:
            rep = _lib.TuneReport()
            check(lib.psoam_plan_create_tuned(*args, C.byref(rep)))
            self.tune_report = {name: (list(v) if isinstance(v, C.Array) else v)
                                for name, v in ((n, getattr(rep, n))
                                                for n, _ in _lib.TuneReport._fields_)}
        else:
            check(lib.psoam_plan_create(*args))
        self._h = handle
        self.prec = prec
        self.c_shape = (ns, ny, nx, nz)
        self.y_shape = (n_pulses, ny, nx, nt)
        self.b_shape = (n_pulses, ny, nx, nz)

    @classmethod
    def acoustic(cls, nx: int, ny: int, nz: int, n_pulses: int, nt: int, f: int,
                 t0: np.ndarray, taps: np.ndarray, prec: str = "fp32", stream=None):
        """Plan of H alone on n_pulses volumes (first step of the two-step
        method): its "concentrations" are the pulse volumes b [K][Ny][Nx][Nz]."""
        self = cls.__new__(cls)
        self._h = None
        self.tune_report = None
        self.geom = _lib.Geom(nx, ny, nz, n_pulses, n_pulses, nt, f, 0, 0)
        self._t0 = np.ascontiguousarray(t0, dtype=np.int32)
        self._taps = np.ascontiguousarray(taps, dtype=np.float32)
        if self._t0.shape != (nz, f, f) or self._taps.shape[:3] != (nz, f, f):
            raise ValueError("impulse-response table shape does not match (nz, f, f)")
        handle = C.c_void_p()
        check(load().psoam_plan_create_acoustic(C.byref(self.geom),
                                                self._t0.ctypes.data_as(C.c_void_p),
                                                self._taps.ctypes.data_as(C.c_void_p),
                                                int(self._taps.shape[3]), PREC[prec],
                                                _stream(stream), C.byref(handle)))
        self._h = handle
        self.prec = prec
        self.c_shape = (n_pulses, ny, nx, nz)
        self.y_shape = (n_pulses, ny, nx, nt)
        self.b_shape = self.c_shape
        return self

    @classmethod
    def factorised(cls, nx: int, ny: int, nz: int, n_pulses: int, nt: int, f: int,
                   phi: np.ndarray, species, spr: np.ndarray, eir: np.ndarray, eir_origin: int,
                   dr: float, z_focus: float, t_focus: int, prec: str = "fp32", stream=None):
        """Plan of A = V Lambda S with the paper's factorised acoustic operator
        (unit-weight discrete shells weighted by the spatial response image
        spr [Nz][F][F], then the temporal convolution with eir; see
        psoam_plan_create_factorised)."""
        self = cls.__new__(cls)
        self._h = None
        self.tune_report = None
        species_a, species_b, species_tau = list(species.a), list(species.b), list(species.tau)
        ns = len(species_a)
        phi = np.ascontiguousarray(phi, dtype=np.float32)
        self.geom = _lib.Geom(nx, ny, nz, ns, n_pulses, nt, f, 1 if phi.ndim == 3 else 0, 0)
        sp = _lib.Species()
        for s in range(ns):
            sp.a[s], sp.b[s], sp.tau[s] = species_a[s], species_b[s], species_tau[s]
        sp.gamma = float(species.gamma)
        self._spr = np.ascontiguousarray(spr, dtype=np.float32)
        self._eir = np.ascontiguousarray(eir, dtype=np.float32).ravel()
        if self._spr.shape != (nz, f, f):
            raise ValueError("spatial response image shape does not match (nz, f, f)")
        sh = _lib.Shell(float(dr), float(z_focus), int(t_focus), int(self._eir.size), int(eir_origin))
        handle = C.c_void_p()
        check(load().psoam_plan_create_factorised(C.byref(self.geom), C.byref(sp),
                                                  phi.ctypes.data_as(C.c_void_p),
                                                  self._spr.ctypes.data_as(C.c_void_p),
                                                  self._eir.ctypes.data_as(C.c_void_p),
                                                  C.byref(sh), PREC[prec], _stream(stream),
                                                  C.byref(handle)))
        self._h = handle
        self.prec = prec
        self.c_shape = (ns, ny, nx, nz)
        self.y_shape = (n_pulses, ny, nx, nt)
        self.b_shape = (n_pulses, ny, nx, nz)
        return self

    @classmethod
    def from_config(cls, cfg, phi, species, t0, taps, prec="fp32", stream=None, separable=False,
                    tune=False):
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.n_pulses, cfg.nt, cfg.f, phi, species, t0, taps,
                   prec=prec, stream=stream, separable=separable, tune=tune)

    def close(self):
        if getattr(self, "_h", None):
            load().psoam_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> C.c_void_p:
        if not self._h:
            raise RuntimeError("plan is closed")
        return self._h

    def stats(self) -> dict:
        info = _lib.PlanInfo()
        check(load().psoam_plan_stats(self.handle, C.byref(info)))
        return {k: [int(getattr(info, k)[0]), int(getattr(info, k)[1])]
                for k in ("useful_macs", "chunks", "executed_macs", "operand_bytes", "lds_bytes",
                          "lds_rows")}

    def band_only(self, direction: int, out, stream=None):
        """Launch only the band kernel (0: H -> y, 1: S^T H^T -> c) on the
        operand left by the last apply (for timing)."""
        check(load().psoam_band_only(self.handle, int(direction), _ptr(out), _stream(stream)))
        return out

    # ------------------------------------------------------------- operators
    def apply_A(self, c, y=None, stream=None):
        torch = _torch()
        _check_f32(c, self.c_shape, "c")
        if y is None:
            y = torch.empty(self.y_shape, dtype=torch.float32, device=c.device)
        _check_f32(y, self.y_shape, "y")
        check(load().psoam_apply_A(self.handle, _ptr(c), _ptr(y), _stream(stream)))
        return y

    def apply_AT(self, y, c=None, stream=None):
        torch = _torch()
        _check_f32(y, self.y_shape, "y")
        if c is None:
            c = torch.empty(self.c_shape, dtype=torch.float32, device=y.device)
        _check_f32(c, self.c_shape, "c")
        check(load().psoam_apply_AT(self.handle, _ptr(y), _ptr(c), _stream(stream)))
        return c

    def prox_tv(self, z, theta: float, n_inner: int, nonneg: bool = False, x=None, ws=None,
                stream=None):
        torch = _torch()
        _check_f32(z, self.c_shape, "z")
        if x is None:
            x = torch.empty_like(z)
        nbytes = int(load().psoam_prox_tv_ws_bytes(self.handle))
        if ws is None:
            ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=z.device)
        check(load().psoam_prox_tv(self.handle, _ptr(x), _ptr(z), float(theta), int(n_inner),
                                   1 if nonneg else 0, _ptr(ws), _stream(stream)))
        return x

    def prox_tv_noalloc(self, z, theta: float, n_inner: int, nonneg: bool = False, x=None,
                        stream=None):
        """prox_tv without a workspace (psoam_prox_tv_noalloc: the duals live in
        the library's static device array).  Pass x to allocate nothing here."""
        torch = _torch()
        _check_f32(z, self.c_shape, "z")
        if x is None:
            x = torch.empty_like(z)
        _check_f32(x, self.c_shape, "x")
        check(load().psoam_prox_tv_noalloc(self.handle, _ptr(x), _ptr(z), float(theta),
                                           int(n_inner), 1 if nonneg else 0, _stream(stream)))
        return x

    def prox_r3(self, z, theta_tv: float, theta_tvs: float, theta_l1: float, n_inner: int,
                x=None, ws=None, stream=None):
        """Prox of the full regulariser (TV of c, TV of S c, l1, x >= 0)."""
        torch = _torch()
        _check_f32(z, self.c_shape, "z")
        if x is None:
            x = torch.empty_like(z)
        nbytes = int(load().psoam_prox_r3_ws_bytes(self.handle))
        if ws is None:
            ws = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=z.device)
        check(load().psoam_prox_r3(self.handle, _ptr(x), _ptr(z), float(theta_tv),
                                   float(theta_tvs), float(theta_l1), int(n_inner), _ptr(ws),
                                   _stream(stream)))
        return x

    def solve(self, p, c=None, lambda_tv=0.0, lambda_l1=0.0, k1=100, k2=20, eps1=0.0, eps2=0.0,
              alpha1=0.0, n_power=30, literal_momentum=False, warm_inner=False, v0=None,
              trace: bool = False, stream=None, lambda_tvs=0.0, device_stop: bool = False):
        """Returns (c, stats dict[, trace list]).  device_stop: the stopping
        tests run on the device (no host read per iteration)."""
        _check_f32(p, self.y_shape, "p")
        return self._iterate("psoam_solve", p, c, lambda_tv, lambda_l1, k1, k2, eps1, eps2,
                             alpha1, n_power, literal_momentum, warm_inner, v0, trace, stream,
                             lambda_tvs, device_stop)

    def unmix(self, b, c=None, lambda_tv=0.0, lambda_l1=0.0, k1=100, k2=20, eps1=0.0, eps2=0.0,
              alpha1=0.0, n_power=30, literal_momentum=False, v0=None, trace: bool = False,
              stream=None, device_stop: bool = False):
        """Unmixing step of the two-step method (psoam_unmix): c from pulse
        volumes b [K][Ny][Nx][Nz].  Returns (c, stats dict[, trace list])."""
        _check_f32(b, self.b_shape, "b")
        return self._iterate("psoam_unmix", b, c, lambda_tv, lambda_l1, k1, k2, eps1, eps2,
                             alpha1, n_power, literal_momentum, False, v0, trace, stream, 0.0,
                             device_stop)

    def _iterate(self, fn, p, c, lambda_tv, lambda_l1, k1, k2, eps1, eps2, alpha1, n_power,
                 literal_momentum, warm_inner, v0, trace, stream, lambda_tvs, device_stop):
        torch = _torch()
        if c is None:
            c = torch.zeros(self.c_shape, dtype=torch.float32, device=p.device)
        _check_f32(c, self.c_shape, "c")
        if v0 is not None:
            _check_f32(v0, self.c_shape, "v0")
        tr = (C.c_double * max(k1, 1))() if trace else None
        o = _lib.SolveOpts(float(lambda_tv), float(lambda_l1), int(k1), int(k2), float(eps1),
                           float(eps2), float(alpha1), int(n_power), int(bool(literal_momentum)),
                           int(bool(warm_inner)), C.c_void_p(v0.data_ptr()) if v0 is not None else None,
                           C.cast(tr, C.POINTER(C.c_double)) if tr is not None else None,
                           float(lambda_tvs), int(bool(device_stop)))
        st = _lib.SolveStats()
        check(getattr(load(), fn)(self.handle, _ptr(p), _ptr(c), C.byref(o), C.byref(st),
                                  _stream(stream)))
        stats = dict(iterations=st.iterations, status=st.status, alpha1=st.alpha1,
                     lambda_max=st.lambda_max, objective=st.objective)
        if trace:
            return c, stats, [tr[i] for i in range(st.iterations)]
        return c, stats


def two_step(acoustic: Plan, species: Plan, p, nu1: float, nu2: float, nu3: float,
             k1_acoustic: int = 100, k1_unmix: int = 100, k2: int = 20, alpha_acoustic=0.0,
             alpha_unmix=0.0, n_power: int = 30, stream=None):
    """The paper's two-step method: b = psoam_solve on the acoustic plan with
    TV weight nu1 (nonnegative pulse images), then c = psoam_unmix on the
    species plan with l1 weight nu2 and TV weight nu3.  Returns (b, c, stats)."""
    b, st1 = acoustic.solve(p, lambda_tv=nu1, k1=k1_acoustic, k2=k2, alpha1=alpha_acoustic,
                            n_power=n_power, stream=stream)
    c, st2 = species.unmix(b, lambda_tv=nu3, lambda_l1=nu2, k1=k1_unmix, k2=k2,
                           alpha1=alpha_unmix, n_power=n_power, stream=stream)
    return b, c, (st1, st2)


def solve_batch(plans: Sequence[Plan], ps, cs, opts: Sequence[dict], stream=None):
    """Run psoam_solve_batch over several plans; returns a list of stats dicts.
    ps[i] and cs[i] must be contiguous float32 device tensors of plans[i]'s
    measurement and concentration shapes (checked here, before any call)."""
    n = len(plans)
    if not (len(ps) == n and len(cs) == n and len(opts) == n):
        raise ValueError(f"solve_batch: {n} plans but {len(ps)} measurements, {len(cs)} "
                         f"concentration tensors and {len(opts)} option sets")
    for i in range(n):
        _check_f32(ps[i], plans[i].y_shape, f"p[{i}]")
        _check_f32(cs[i], plans[i].c_shape, f"c[{i}]")
    hs = (C.c_void_p * n)(*[pl.handle.value for pl in plans])
    pp = (C.c_void_p * n)(*[p.data_ptr() for p in ps])
    cc = (C.c_void_p * n)(*[c.data_ptr() for c in cs])
    oo = (_lib.SolveOpts * n)()
    for i, d in enumerate(opts):
        oo[i] = _lib.SolveOpts(float(d.get("lambda_tv", 0.0)), float(d.get("lambda_l1", 0.0)),
                               int(d.get("k1", 100)), int(d.get("k2", 20)),
                               float(d.get("eps1", 0.0)), float(d.get("eps2", 0.0)),
                               float(d.get("alpha1", 0.0)), int(d.get("n_power", 30)), 0, 0,
                               None, None, float(d.get("lambda_tvs", 0.0)),
                               int(bool(d.get("device_stop", False))))
    st = (_lib.SolveStats * n)()
    check(load().psoam_solve_batch(n, hs, pp, cc, oo, st, _stream(stream)))
    return [dict(iterations=s.iterations, status=s.status, alpha1=s.alpha1,
                 lambda_max=s.lambda_max, objective=s.objective) for s in st]


def prox_l1(z, thresh: float, nonneg: bool = True, x=None, stream=None):
    """x = soft threshold of z (max(z - thresh, 0) when nonneg); z and x are
    contiguous float32 device tensors of one shape (x may be z)."""
    torch = _torch()
    _check_f32(z, tuple(z.shape), "z")
    if x is None:
        x = torch.empty_like(z)
    _check_f32(x, tuple(z.shape), "x")
    check(load().psoam_prox_l1(_ptr(x), _ptr(z), int(z.numel()), float(thresh),
                               1 if nonneg else 0, _stream(stream)))
    return x


class _AFunction:
    """torch.autograd.Function whose forward is psoam_apply_A and whose
    backward is the hand-written adjoint psoam_apply_AT."""
    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            torch = _torch()

            class AFn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, c, plan):
                    ctx.plan = plan
                    return plan.apply_A(c.contiguous())

                @staticmethod
                def backward(ctx, gy):
                    return ctx.plan.apply_AT(gy.contiguous()), None

            cls._cls = AFn
        return cls._cls


def A(c, plan: Plan):
    """y = A c, differentiable: the gradient is A^T applied by the library."""
    return _AFunction.get().apply(c, plan)

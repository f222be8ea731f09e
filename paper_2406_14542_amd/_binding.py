"""ctypes binding of libnusht.so (include/nusht.h), plus a torch-facing ``Plan`` wrapper.

The C functions keep their names (``lib().nusht_synthesis`` ...).  ``Plan`` only checks
shapes/dtypes/devices of torch tensors and forwards their data pointers and the current
HIP stream; it does no arithmetic of its own.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(HERE, "libnusht.so")

NUSHT_F64, NUSHT_MIXED = 0, 1
NUSHT_OK, NUSHT_EINVAL, NUSHT_ENOMEM, NUSHT_EDEVICE, NUSHT_ENOCONV, NUSHT_EPRECISION = \
    0, -1, -2, -3, -4, -5
NUSHT_DFS_FUSED, NUSHT_DFS_PAPER = 0, 1
NUSHT_MAX_SPIN = 64  # largest spin of nusht_synthesis_spin / nusht_adjoint_spin


class PlanOpts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("width", ctypes.c_int),
                ("beta_per_w", ctypes.c_double), ("dfs_mode", ctypes.c_int),
                ("timing", ctypes.c_int), ("deterministic", ctypes.c_int),
                ("kernel_eval", ctypes.c_int), ("reserved", ctypes.c_int * 4)]


class Geometry(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int), ("mmax", ctypes.c_int), ("nrings", ctypes.c_int),
                ("ntorus", ctypes.c_int), ("nphi", ctypes.c_int), ("n1", ctypes.c_int),
                ("n2", ctypes.c_int), ("width", ctypes.c_int), ("beta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("tile", ctypes.c_int), ("dtype", ctypes.c_int),
                ("dfs_mode", ctypes.c_int), ("npts", ctypes.c_int64), ("nalm", ctypes.c_int64),
                ("ntiles_used", ctypes.c_int64), ("kernel_eval", ctypes.c_int),
                ("kernel_poly_dev", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NushtError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        msg = f"{where}: {lib().nusht_strerror(status).decode()} ({status})"
        if detail:
            msg += f" [{detail}]"
        super().__init__(msg)


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


def library_path() -> str:
    return _SO


def lib():
    """Load libnusht.so once.  torch is imported first so that the library binds to the HIP
    runtime and rocFFT that torch already loaded (same sonames) instead of a second copy."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401

        if not os.path.exists(_SO):
            raise ImportError(f"{_SO} is missing: build it with `python -m "
                              "paper_2406_14542_amd.build` (the HIP path has no fallback)")
        L = ctypes.CDLL(_SO)
        sig = {
            "nusht_nalm": (_i64, [ctypes.c_int, ctypes.c_int]),
            "nusht_geometry_for": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                  ctypes.c_int, ctypes.POINTER(PlanOpts),
                                                  ctypes.POINTER(Geometry)]),
            "nusht_plan": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64, _vp, _vp,
                                          ctypes.c_double, ctypes.c_int, ctypes.POINTER(_vp)]),
            "nusht_plan_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64, _vp, _vp,
                                             ctypes.c_double, ctypes.c_int,
                                             ctypes.POINTER(PlanOpts), _vp, ctypes.POINTER(_vp)]),
            "nusht_plan_info": (ctypes.c_int, [_vp, ctypes.POINTER(Geometry)]),
            "nusht_plan_status": (ctypes.c_int, [_vp]),
            "nusht_synthesis": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
            "nusht_adjoint": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
            "nusht_synthesis_spin": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int,
                                                    _vp]),
            "nusht_adjoint_spin": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int,
                                                  _vp]),
            "nusht_synthesis_deriv": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                                     _vp]),
            "nusht_pointing": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
            "nusht_deflect": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
            "nusht_vjp_alm": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
            "nusht_vjp_alm_spin": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int,
                                                  _vp]),
            "nusht_synthesis_spin_deriv": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                                                          ctypes.c_int, _vp]),
            "nusht_vjp_points": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _i64,
                                                _vp]),
            "nusht_ring_synthesis": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
            "nusht_ring_adjoint": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp]),
            "nusht_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_double), _vp]),
            "nusht_mlp_param_count": (_i64, []),
            "nusht_density_map": (ctypes.c_int, [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int,
                                                 _vp, _vp]),
            "nusht_density_map_noalloc": (ctypes.c_int, [_vp, _vp, _i64, ctypes.c_int,
                                                         ctypes.c_int, _vp, _vp]),
            "nusht_point_features": (ctypes.c_int, [_vp, _vp, _i64, _vp, ctypes.c_int,
                                                    ctypes.c_int, _vp, _vp]),
            "nusht_mlp_forward": (ctypes.c_int, [_vp, _vp, _i64, ctypes.c_float, _vp, _vp]),
            "nusht_mlp_backward": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.c_float, _vp,
                                                  _vp]),
            "nusht_adam_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, ctypes.c_float,
                                               ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                               ctypes.c_int, _vp]),
            "nusht_weighted_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
            "nusht_weight_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp,
                                                      ctypes.POINTER(ctypes.c_double), _vp]),
            "nusht_solve_ex": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), _vp]),
            "nusht_solve_spin": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp,
                                                ctypes.c_double, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double), _vp]),
            "nusht_stage_times": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                                 ctypes.POINTER(ctypes.c_char_p), ctypes.c_int]),
            "nusht_stage_stats": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                                 ctypes.POINTER(ctypes.c_int),
                                                 ctypes.POINTER(ctypes.c_char_p), ctypes.c_int]),
            "nusht_stage_reset": (None, [_vp]),
            "nusht_destroy": (None, [_vp]),
            "nusht_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "nusht_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status != NUSHT_OK:
        raise NushtError(status, where, lib().nusht_last_error().decode())


def nalm(lmax: int, mmax: int) -> int:
    return int(lib().nusht_nalm(lmax, mmax))


def _opts(sigma=0.0, width=0, beta_per_w=0.0, dfs_mode="fused", timing=False,
          deterministic=False, kernel_eval="poly"):
    o = PlanOpts()
    o.deterministic = 1 if deterministic else 0
    o.kernel_eval = {"poly": 0, "exact": 1}[kernel_eval]
    o.sigma = float(sigma)
    o.width = int(width)
    o.beta_per_w = float(beta_per_w)
    o.dfs_mode = {"fused": NUSHT_DFS_FUSED, "paper": NUSHT_DFS_PAPER}[dfs_mode]
    o.timing = 1 if timing else 0
    return o


def _coord_signature(x):
    """Sums of x, x^2 and (i mod 1021) x_i over a device coordinate tensor (FP64)."""
    import torch
    w = torch.arange(x.numel(), dtype=torch.float64, device=x.device).remainder_(1021.0)
    return torch.stack([x.sum(), (x * x).sum(), (w * x).sum()])


def _dtype_code(dtype):
    return {"f64": NUSHT_F64, "mixed": NUSHT_MIXED}[dtype]


def geometry(lmax, mmax, eps, dtype="f64", **opts) -> dict:
    """Sizes a plan would use (host-only query)."""
    g = Geometry()
    o = _opts(**opts)
    _check(lib().nusht_geometry_for(lmax, mmax, eps, _dtype_code(dtype), ctypes.byref(o),
                                    ctypes.byref(g)), "nusht_geometry_for")
    return g.as_dict()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A nusht plan for fixed points (theta, phi) -- torch float64 tensors on the GPU."""

    def __init__(self, lmax, mmax, theta, phi, eps, dtype="f64", sigma=0.0, width=0,
                 beta_per_w=0.0, dfs_mode="fused", timing=False, deterministic=False,
                 kernel_eval="poly"):
        import torch
        if theta.dtype != torch.float64 or phi.dtype != torch.float64:
            raise TypeError("theta and phi must be float64")
        if not (theta.is_cuda and phi.is_cuda) or theta.shape != phi.shape or theta.dim() != 1:
            raise ValueError("theta and phi must be 1-D device tensors of equal length")
        theta = theta.contiguous()
        phi = phi.contiguous()
        self.lmax, self.mmax, self.eps = int(lmax), int(mmax), float(eps)
        self.dtype = dtype
        self.npts = int(theta.numel())
        self.device = theta.device
        o = _opts(sigma, width, beta_per_w, dfs_mode, timing, deterministic, kernel_eval)
        h = _vp()
        _check(lib().nusht_plan_ex(self.lmax, self.mmax, self.npts, theta.data_ptr(),
                                   phi.data_ptr(), self.eps, _dtype_code(dtype), ctypes.byref(o),
                                   _stream(), ctypes.byref(h)), "nusht_plan_ex")
        self._h = h
        g = Geometry()
        _check(lib().nusht_plan_info(h, ctypes.byref(g)), "nusht_plan_info")
        self.geometry = g.as_dict()
        self.nalm = int(self.geometry["nalm"])
        self._sig_theta = _coord_signature(theta)
        self._sig_phi = _coord_signature(phi)

    def check_points(self, theta=None, phi=None):
        """Raise ValueError unless the given coordinate tensors hold the plan's points in the
        caller's order (compared through sums of the values, their squares and an
        index-weighted sum, so a moved or reordered point is caught)."""
        import torch
        for name, x, sig in (("theta", theta, self._sig_theta), ("phi", phi, self._sig_phi)):
            if x is None:
                continue
            if x.dim() != 1 or x.numel() != self.npts or x.device != self.device:
                raise ValueError(f"{name} must be a 1-D tensor of the plan's {self.npts} points "
                                 f"on {self.device}")
            got = _coord_signature(x.detach().to(torch.float64))
            if not torch.allclose(got, sig, rtol=1e-13, atol=0.0):
                raise ValueError(f"{name} differs from the coordinates the plan was built on; "
                                 "gradients are taken at the plan's points: build a plan on "
                                 "the new coordinates")

    def status(self):
        """Raise NushtError if a kernel of this plan flagged a device-side failure (waits for
        the device)."""
        _check(lib().nusht_plan_status(self._h), "nusht_plan_status")

    # ---- helpers ----
    def _alm_in(self, alm):
        import torch
        if alm.dtype != torch.complex128 or not alm.is_cuda:
            raise TypeError("alm must be a complex128 device tensor")
        if alm.device != self.device:
            raise TypeError(f"alm must live on {self.device}")
        a = alm.reshape(-1, self.nalm) if alm.dim() == 1 else alm
        if a.dim() != 2 or a.shape[1] != self.nalm:
            raise ValueError(f"alm must have shape [B, {self.nalm}]")
        return a.contiguous()

    def _map_in(self, m):
        import torch
        if m.dtype != torch.float64 or not m.is_cuda:
            raise TypeError("maps must be float64 device tensors")
        if m.device != self.device:
            raise TypeError(f"maps must live on {self.device}")
        x = m.reshape(1, -1) if m.dim() == 1 else m
        if x.dim() != 2 or x.shape[1] != self.npts:
            raise ValueError(f"map must have shape [B, {self.npts}]")
        return x.contiguous()

    @staticmethod
    def _out(out, shape, dtype, like):
        """A fresh output tensor, or the caller's `out` checked to be exactly what the
        library will write: dtype, device, shape and a contiguous layout."""
        import torch
        if out is None:
            return torch.empty(shape, dtype=dtype, device=like.device)
        if not isinstance(out, torch.Tensor) or out.dtype != dtype:
            raise TypeError(f"out must be a {dtype} tensor")
        if not out.is_cuda or out.device != like.device:
            raise TypeError(f"out must live on {like.device}")
        if tuple(out.shape) != tuple(shape):
            raise ValueError(f"out must have shape {list(shape)}, got {list(out.shape)}")
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
        return out

    # ---- transforms ----
    def synthesis(self, alm, out=None):
        import torch
        a = self._alm_in(alm)
        B = a.shape[0]
        out = self._out(out, (B, self.npts), torch.float64, a)
        _check(lib().nusht_synthesis(self._h, a.data_ptr(), out.data_ptr(), B, _stream()),
               "nusht_synthesis")
        return out

    def adjoint(self, m, out=None):
        import torch
        x = self._map_in(m)
        B = x.shape[0]
        out = self._out(out, (B, self.nalm), torch.complex128, x)
        _check(lib().nusht_adjoint(self._h, x.data_ptr(), out.data_ptr(), B, _stream()),
               "nusht_adjoint")
        return out

    def synthesis_spin(self, spin, alm, out=None):
        """Spin-`spin` synthesis: alm [F, 2, nalm] complex128 (gradient G, curl C per field)
        -> [F, 2, npts] float64 (Q, U)."""
        import torch
        if alm.dtype != torch.complex128 or not alm.is_cuda or alm.device != self.device:
            raise TypeError(f"alm must be a complex128 tensor on {self.device}")
        a = alm.unsqueeze(0) if alm.dim() == 2 else alm
        if a.dim() != 3 or a.shape[1] != 2 or a.shape[2] != self.nalm:
            raise ValueError(f"alm must have shape [F, 2, {self.nalm}]")
        a = a.contiguous()
        F = a.shape[0]
        out = self._out(out, (F, 2, self.npts), torch.float64, a)
        _check(lib().nusht_synthesis_spin(self._h, int(spin), a.data_ptr(), out.data_ptr(), F,
                                          _stream()), "nusht_synthesis_spin")
        return out

    def adjoint_spin(self, spin, maps, out=None):
        """Adjoint of synthesis_spin: maps [F, 2, npts] float64 -> [F, 2, nalm] complex128."""
        import torch
        if maps.dtype != torch.float64 or not maps.is_cuda or maps.device != self.device:
            raise TypeError(f"maps must be a float64 tensor on {self.device}")
        x = maps.unsqueeze(0) if maps.dim() == 2 else maps
        if x.dim() != 3 or x.shape[1] != 2 or x.shape[2] != self.npts:
            raise ValueError(f"maps must have shape [F, 2, {self.npts}]")
        x = x.contiguous()
        F = x.shape[0]
        out = self._out(out, (F, 2, self.nalm), torch.complex128, x)
        _check(lib().nusht_adjoint_spin(self._h, int(spin), x.data_ptr(), out.data_ptr(), F,
                                        _stream()), "nusht_adjoint_spin")
        return out

    def synthesis_spin_deriv(self, spin, alm):
        """(Q, U) maps and their theta / phi derivatives at the points, each [F, 2, npts]
        (FP64 plans)."""
        import torch
        if alm.dtype != torch.complex128 or not alm.is_cuda or alm.device != self.device:
            raise TypeError(f"alm must be a complex128 tensor on {self.device}")
        a = alm.unsqueeze(0) if alm.dim() == 2 else alm
        if a.dim() != 3 or a.shape[1] != 2 or a.shape[2] != self.nalm:
            raise ValueError(f"alm must have shape [F, 2, {self.nalm}]")
        a = a.contiguous()
        F = a.shape[0]
        f = torch.empty((F, 2, self.npts), dtype=torch.float64, device=a.device)
        dt = torch.empty_like(f)
        dp = torch.empty_like(f)
        _check(lib().nusht_synthesis_spin_deriv(self._h, int(spin), a.data_ptr(), f.data_ptr(),
                                                dt.data_ptr(), dp.data_ptr(), F, _stream()),
               "nusht_synthesis_spin_deriv")
        return f, dt, dp

    def vjp_alm_spin(self, spin, grad_maps):
        """dL/dRe + i dL/dIm of the gradient/curl coefficients for dL/d(Q, U) = grad_maps
        [F, 2, npts] (the spin adjoint with the complex-gradient convention)."""
        import torch
        if grad_maps.dtype != torch.float64 or not grad_maps.is_cuda:
            raise TypeError("grad_maps must be a float64 device tensor")
        x = grad_maps.unsqueeze(0) if grad_maps.dim() == 2 else grad_maps
        if x.dim() != 3 or x.shape[1] != 2 or x.shape[2] != self.npts:
            raise ValueError(f"grad_maps must have shape [F, 2, {self.npts}]")
        x = x.contiguous()
        out = torch.empty((x.shape[0], 2, self.nalm), dtype=torch.complex128, device=x.device)
        _check(lib().nusht_vjp_alm_spin(self._h, int(spin), x.data_ptr(), out.data_ptr(),
                                        x.shape[0], _stream()), "nusht_vjp_alm_spin")
        return out

    def synthesis_deriv(self, alm):
        import torch
        a = self._alm_in(alm)
        B = a.shape[0]
        f = torch.empty((B, self.npts), dtype=torch.float64, device=a.device)
        dt = torch.empty_like(f)
        dp = torch.empty_like(f)
        _check(lib().nusht_synthesis_deriv(self._h, a.data_ptr(), f.data_ptr(), dt.data_ptr(),
                                           dp.data_ptr(), B, _stream()), "nusht_synthesis_deriv")
        return f, dt, dp

    def pointing(self, dlm):
        """nusht_pointing: deflected (theta', phi') of the plan's points under the lensing
        potential with coefficients dlm (complex128 [nalm])."""
        import torch
        a = self._alm_in(dlm)
        if a.shape[0] != 1:
            raise ValueError("pointing takes one potential")
        th = torch.empty(self.npts, dtype=torch.float64, device=a.device)
        ph = torch.empty_like(th)
        _check(lib().nusht_pointing(self._h, a.data_ptr(), th.data_ptr(), ph.data_ptr(),
                                    _stream()), "nusht_pointing")
        return th, ph

    def vjp_alm(self, grad_map):
        """dL/dRe a + i dL/dIm a for g = dL/dmap (nusht_vjp_alm)."""
        import torch
        g = self._map_in(grad_map)
        B = g.shape[0]
        out = torch.empty((B, self.nalm), dtype=torch.complex128, device=g.device)
        _check(lib().nusht_vjp_alm(self._h, g.data_ptr(), out.data_ptr(), B, _stream()),
               "nusht_vjp_alm")
        return out

    def vjp_points(self, grad_map, dtheta, dphi, want_theta=True, want_phi=True):
        """(sum_b g dmap/dtheta, sum_b g dmap/dphi) per point (nusht_vjp_points)."""
        import torch
        g = self._map_in(grad_map)
        B = g.shape[0]
        gt = torch.empty(self.npts, dtype=torch.float64, device=g.device) if want_theta else None
        gp = torch.empty(self.npts, dtype=torch.float64, device=g.device) if want_phi else None
        _check(lib().nusht_vjp_points(g.data_ptr(), dtheta.contiguous().data_ptr(),
                                      dphi.contiguous().data_ptr(),
                                      gt.data_ptr() if gt is not None else None,
                                      gp.data_ptr() if gp is not None else None, B, self.npts,
                                      _stream()), "nusht_vjp_points")
        return gt, gp

    def ring_synthesis(self, alm):
        import torch
        a = self._alm_in(alm)
        B = a.shape[0]
        g = self.geometry
        out = torch.empty((B, g["nrings"], g["nphi"]), dtype=torch.float64, device=a.device)
        _check(lib().nusht_ring_synthesis(self._h, a.data_ptr(), out.data_ptr(), B, _stream()),
               "nusht_ring_synthesis")
        return out

    def ring_adjoint(self, ring):
        import torch
        g = self.geometry
        r = ring.reshape(-1, g["nrings"], g["nphi"]).contiguous()
        if r.dtype != torch.float64 or not r.is_cuda:
            raise TypeError("ring maps must be float64 device tensors")
        B = r.shape[0]
        out = torch.empty((B, self.nalm), dtype=torch.complex128, device=r.device)
        _check(lib().nusht_ring_adjoint(self._h, r.data_ptr(), out.data_ptr(), B, _stream()),
               "nusht_ring_adjoint")
        return out

    def solve(self, d, x0=None, weights=None, tol=1e-8, maxiter=1000, check=True,
              history=False):
        """CGLS inverse (nusht_solve_ex).  Returns (alm, iterations, true relative residual,
        status), plus the per-iteration recurred relative residuals (numpy) if history."""
        import torch
        x = self._map_in(d)
        if x.shape[0] != 1:
            raise ValueError("solve takes one map")
        alm = torch.zeros(self.nalm, dtype=torch.complex128, device=x.device) if x0 is None \
            else self._alm_in(x0).reshape(-1).clone()
        wptr = None
        if weights is not None:
            if weights.dtype != torch.float32 or weights.numel() != self.npts:
                raise ValueError("weights must be float32 [npts]")
            weights = weights.contiguous()
            wptr = weights.data_ptr()
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        hist = (ctypes.c_double * (int(maxiter) + 1))() if history else None
        st = lib().nusht_solve_ex(self._h, x.data_ptr(), alm.data_ptr(), wptr, float(tol),
                                  int(maxiter), ctypes.byref(it), ctypes.byref(rr), hist,
                                  _stream())
        if st not in (NUSHT_OK, NUSHT_ENOCONV) or (check and st != NUSHT_OK):
            _check(st, "nusht_solve")
        if history:
            import numpy as np
            return alm, it.value, rr.value, st, np.array(hist[:it.value + 1])
        return alm, it.value, rr.value, st

    def solve_spin(self, spin, d, x0=None, weights=None, tol=1e-8, maxiter=1000, check=True,
                   history=False):
        """Spin-`spin` CGLS inverse of one field (nusht_solve_spin): d [2, npts] (Q, U) float64
        -> (alm [2, nalm] complex128 (G, C), iterations, true relative residual, status),
        plus the recurred relative residuals (numpy) if history."""
        import torch
        if d.dtype != torch.float64 or not d.is_cuda or d.device != self.device:
            raise TypeError(f"d must be a float64 tensor on {self.device}")
        x = d.reshape(-1)
        if x.numel() != 2 * self.npts:
            raise ValueError(f"d must hold one field's (Q, U): [2, {self.npts}]")
        x = x.contiguous()
        if x0 is None:
            alm = torch.zeros((2, self.nalm), dtype=torch.complex128, device=x.device)
        else:
            if x0.dtype != torch.complex128 or x0.numel() != 2 * self.nalm:
                raise ValueError(f"x0 must be complex128 [2, {self.nalm}]")
            alm = x0.reshape(2, self.nalm).to(x.device).clone()
        wptr = None
        if weights is not None:
            if weights.dtype != torch.float32 or weights.numel() != self.npts:
                raise ValueError("weights must be float32 [npts]")
            weights = weights.contiguous()
            wptr = weights.data_ptr()
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        hist = (ctypes.c_double * (int(maxiter) + 1))() if history else None
        st = lib().nusht_solve_spin(self._h, int(spin), x.data_ptr(), alm.data_ptr(), wptr,
                                    float(tol), int(maxiter), ctypes.byref(it), ctypes.byref(rr),
                                    hist, _stream())
        if st not in (NUSHT_OK, NUSHT_ENOCONV) or (check and st != NUSHT_OK):
            _check(st, "nusht_solve_spin")
        if history:
            import numpy as np
            return alm, it.value, rr.value, st, np.array(hist[:it.value + 1])
        return alm, it.value, rr.value, st

    def weighted_adjoint(self, d, weights):
        """S^H (W d) for one map (nusht_weighted_adjoint): complex128 [1, nalm]."""
        import torch
        x = self._map_in(d)
        if x.shape[0] != 1:
            raise ValueError("weighted_adjoint takes one map")
        w = _f32_dev(weights, self.npts, "weights")
        out = torch.empty((1, self.nalm), dtype=torch.complex128, device=x.device)
        _check(lib().nusht_weighted_adjoint(self._h, x.data_ptr(), w.data_ptr(), out.data_ptr(),
                                            _stream()), "nusht_weighted_adjoint")
        return out

    def weight_loss_grad(self, d, astar, weights, want_grad=True):
        """Loss <r, r>_m / <a*, a*>_m with r = S^H (W d) - a*, and d loss / d w (float32 [npts])
        when want_grad (nusht_weight_loss_grad).  Returns (loss, grad or None)."""
        import torch
        x = self._map_in(d)
        a = self._alm_in(astar)
        if x.shape[0] != 1 or a.shape[0] != 1:
            raise ValueError("weight_loss_grad takes one map and one coefficient set")
        w = _f32_dev(weights, self.npts, "weights")
        g = torch.empty(self.npts, dtype=torch.float32, device=x.device) if want_grad else None
        loss = ctypes.c_double(0.0)
        _check(lib().nusht_weight_loss_grad(self._h, x.data_ptr(), a.data_ptr(), w.data_ptr(),
                                            None if g is None else g.data_ptr(),
                                            ctypes.byref(loss), _stream()),
               "nusht_weight_loss_grad")
        return loss.value, g

    def stage_times(self) -> dict:
        ms = (ctypes.c_double * 16)()
        names = (ctypes.c_char_p * 16)()
        n = lib().nusht_stage_times(self._h, ms, names, 16)
        if n < 0:
            _check(n, "nusht_stage_times")
        return {names[i].decode(): ms[i] for i in range(n)}

    CALL_KINDS = {"synthesis": 0, "adjoint": 1, "synthesis_deriv": 2, "ring": 3,
                  "synthesis_spin": 4, "adjoint_spin": 5}

    def stage_stats(self, kind: str) -> dict:
        """Mean per-stage device ms over the recorded calls of one kind (timing plans):
        {stage: (mean_ms, ncalls)}."""
        ms = (ctypes.c_double * 16)()
        cnt = (ctypes.c_int * 16)()
        names = (ctypes.c_char_p * 16)()
        n = lib().nusht_stage_stats(self._h, self.CALL_KINDS[kind], ms, cnt, names, 16)
        if n < 0:
            _check(n, "nusht_stage_stats")
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(n) if cnt[i] > 0}

    def stage_reset(self):
        lib().nusht_stage_reset(self._h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().nusht_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned-weight kernels (FP32 network; see include/nusht.h) ----

def _f32_dev(x, n, what):
    import torch
    if x.dtype != torch.float32 or not x.is_cuda or x.numel() != n:
        raise ValueError(f"{what} must be a float32 device tensor with {n} elements")
    return x.contiguous()


def _f64_pts(theta, phi):
    import torch
    if theta.dtype != torch.float64 or phi.dtype != torch.float64 or not theta.is_cuda \
            or theta.shape != phi.shape or theta.dim() != 1:
        raise ValueError("theta and phi must be 1-D float64 device tensors of equal length")
    return theta.contiguous(), phi.contiguous()


def mlp_param_count() -> int:
    return int(lib().nusht_mlp_param_count())


def deflect(theta, phi, alpha_theta, alpha_phi):
    """nusht_deflect: Eq. (C1) for given deflection components (float64 device tensors)."""
    import torch
    theta, phi = _f64_pts(theta, phi)
    at, ap = _f64_pts(alpha_theta, alpha_phi)
    if at.numel() != theta.numel() or at.device != theta.device:
        raise ValueError("deflection components must match the points")
    th = torch.empty_like(theta)
    ph = torch.empty_like(theta)
    _check(lib().nusht_deflect(theta.data_ptr(), phi.data_ptr(), at.data_ptr(), ap.data_ptr(),
                               theta.numel(), th.data_ptr(), ph.data_ptr(), _stream()),
           "nusht_deflect")
    return th, ph


def density_map(theta, phi, ntheta, nphi):
    import torch
    theta, phi = _f64_pts(theta, phi)
    out = torch.empty((ntheta, nphi), dtype=torch.float32, device=theta.device)
    _check(lib().nusht_density_map(theta.data_ptr(), phi.data_ptr(), theta.numel(), ntheta,
                                   nphi, out.data_ptr(), _stream()), "nusht_density_map")
    return out


def density_map_noalloc(theta, phi, ntheta, nphi, out):
    """nusht_density_map_noalloc: the density map into the caller's float32 [ntheta, nphi]
    device tensor `out`, with no device allocation by the library."""
    import torch
    theta, phi = _f64_pts(theta, phi)
    if (out.dtype != torch.float32 or not out.is_cuda or out.device != theta.device
            or tuple(out.shape) != (ntheta, nphi) or not out.is_contiguous()):
        raise ValueError(f"out must be a contiguous float32 [{ntheta}, {nphi}] tensor on "
                         f"{theta.device}")
    _check(lib().nusht_density_map_noalloc(theta.data_ptr(), phi.data_ptr(), theta.numel(),
                                           ntheta, nphi, out.data_ptr(), _stream()),
           "nusht_density_map_noalloc")
    return out


def point_features(theta, phi, density):
    import torch
    theta, phi = _f64_pts(theta, phi)
    if density.dtype != torch.float32 or density.dim() != 2 or not density.is_cuda:
        raise ValueError("density must be a float32 [ntheta, nphi] device tensor")
    density = density.contiguous()
    out = torch.empty((theta.numel(), 12), dtype=torch.float32, device=theta.device)
    _check(lib().nusht_point_features(theta.data_ptr(), phi.data_ptr(), theta.numel(),
                                      density.data_ptr(), density.shape[0], density.shape[1],
                                      out.data_ptr(), _stream()), "nusht_point_features")
    return out


def _feat_in(features):
    import torch
    if features.dtype != torch.float32 or features.dim() != 2 or features.shape[1] != 12 \
            or not features.is_cuda:
        raise ValueError("features must be a float32 [npts, 12] device tensor")
    return features.contiguous()


def mlp_forward(params, features, scale):
    import torch
    f = _feat_in(features)
    p = _f32_dev(params, mlp_param_count(), "params")
    out = torch.empty(f.shape[0], dtype=torch.float32, device=f.device)
    _check(lib().nusht_mlp_forward(p.data_ptr(), f.data_ptr(), f.shape[0], float(scale),
                                   out.data_ptr(), _stream()), "nusht_mlp_forward")
    return out


def mlp_backward(params, features, grad_weights, scale):
    import torch
    f = _feat_in(features)
    p = _f32_dev(params, mlp_param_count(), "params")
    g = _f32_dev(grad_weights, f.shape[0], "grad_weights")
    out = torch.empty_like(p)
    _check(lib().nusht_mlp_backward(p.data_ptr(), f.data_ptr(), g.data_ptr(), f.shape[0],
                                    float(scale), out.data_ptr(), _stream()),
           "nusht_mlp_backward")
    return out


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of params (and its moments m, v)."""
    n = params.numel()
    for t, what in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        _f32_dev(t, n, what)
    _check(lib().nusht_adam_step(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                 n, float(lr), float(beta1), float(beta2), float(eps), int(step),
                                 _stream()), "nusht_adam_step")

"""CPU oracle for the nonuniform spherical harmonic transform (spin 0 and spin s).

TEST INFRASTRUCTURE, NOT THE PRODUCT.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with the
GPU library and never imports it.

Three parts live here:

* ``liboracle.so`` (``nusht_oracle.c``): plain C direct sums in FP64 -- synthesis (type 2,
  Eq. 3), adjoint (type 1, Eq. 2) and the synthesis gradient with respect to the point
  coordinates -- with an explicit power-of-two exponent on the Legendre recurrence.
* ``liboracle.so`` (``nusht_spin_oracle.c``): the same direct sums for spin-weighted fields
  (gradient/curl coefficients, Q/U maps) through Wigner's d recurrence.
* a numpy twin (``twin.py``) for tiny sizes: the dense matrix Y of Eq. (4), CGLS on it,
  and an FP64 multilayer perceptron with its hand-derived backward pass.
* the lensing pointing of Appendix C (``pointing.py``): Eq. (C2) through the direct-sum
  synthesis gradient, then Eq. (C1) written out in numpy.

Coefficient layout everywhere: complex128 ``[nmaps, nalm]``, m-major triangle with
``index(l, m) = m (2 lmax + 1 - m) / 2 + l``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "nusht_oracle.c"), os.path.join(_HERE, "nusht_spin_oracle.c")]
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               *_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_nalm.restype = ctypes.c_int64
        lib.oracle_nalm.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.oracle_synthesis.restype = None
        lib.oracle_synthesis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                         ctypes.c_int, dp, ctypes.c_int]
        lib.oracle_adjoint.restype = None
        lib.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                       ctypes.c_int, dp, ctypes.c_int]
        lib.oracle_adjoint_columns.restype = None
        lib.oracle_adjoint_columns.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp,
                                               ctypes.c_int, ctypes.c_int, ip, dp, ctypes.c_int]
        lib.oracle_synthesis_grad.restype = None
        lib.oracle_synthesis_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, dp, dp,
                                              dp, ctypes.c_int, dp, dp, dp, ctypes.c_int]
        lib.oracle_lambda_column.restype = None
        lib.oracle_lambda_column.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, ip]
        lib.oracle_lambda_column_ld.restype = None
        lib.oracle_lambda_column_ld.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                                ip]
        lib.oracle_spin_lambda_column.restype = None
        lib.oracle_spin_lambda_column.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_double, dp, dp, ip]
        lib.oracle_spin_synthesis.restype = None
        lib.oracle_spin_synthesis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int64, dp, dp, dp, ctypes.c_int, dp,
                                              ctypes.c_int]
        lib.oracle_spin_adjoint.restype = None
        lib.oracle_spin_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int64, dp, dp, dp, ctypes.c_int, dp,
                                            ctypes.c_int]
        lib.oracle_spin_adjoint_columns.restype = None
        lib.oracle_spin_adjoint_columns.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                                    dp, dp, dp, ctypes.c_int, ctypes.c_int, ip,
                                                    dp, ctypes.c_int]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def alm_index(lmax: int, l, m):
    return m * (2 * lmax + 1 - m) // 2 + l


def _pts(theta, phi):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    assert th.shape == ph.shape and th.ndim == 1
    return th, ph


def _alm2(alm, lmax, mmax):
    a = np.ascontiguousarray(np.atleast_2d(alm), dtype=np.complex128)
    assert a.shape[1] == nalm(lmax, mmax), (a.shape, nalm(lmax, mmax))
    return a


def synthesis(lmax, mmax, theta, phi, alm, nthreads=0):
    """Type 2 (Eq. 3) by direct summation.  alm: [B, nalm] complex -> [B, N] real."""
    lib = _load()
    th, ph = _pts(theta, phi)
    a = _alm2(alm, lmax, mmax)
    out = np.zeros((a.shape[0], th.size), dtype=np.float64)
    lib.oracle_synthesis(lmax, mmax, th.size, _dp(th), _dp(ph), _dp(a.view(np.float64)),
                         a.shape[0], _dp(out), int(nthreads))
    return out


def adjoint(lmax, mmax, theta, phi, f, nthreads=0):
    """Type 1 (Eq. 2) by direct summation.  f: [B, N] real -> [B, nalm] complex."""
    lib = _load()
    th, ph = _pts(theta, phi)
    fv = np.ascontiguousarray(np.atleast_2d(f), dtype=np.float64)
    assert fv.shape[1] == th.size
    out = np.zeros((fv.shape[0], nalm(lmax, mmax)), dtype=np.complex128)
    lib.oracle_adjoint(lmax, mmax, th.size, _dp(th), _dp(ph), _dp(fv), fv.shape[0],
                       _dp(out.view(np.float64)), int(nthreads))
    return out


def adjoint_columns(lmax, theta, phi, f, mlist, nthreads=0):
    """Type 1 restricted to the given (distinct) m-columns: -> [B, len(mlist), lmax+1]."""
    lib = _load()
    th, ph = _pts(theta, phi)
    fv = np.ascontiguousarray(np.atleast_2d(f), dtype=np.float64)
    ml = np.ascontiguousarray(mlist, dtype=np.int32)
    assert len(set(ml.tolist())) == ml.size
    out = np.zeros((fv.shape[0], ml.size, lmax + 1), dtype=np.complex128)
    lib.oracle_adjoint_columns(lmax, th.size, _dp(th), _dp(ph), _dp(fv), fv.shape[0], ml.size,
                               _ip(ml), _dp(out.view(np.float64)), int(nthreads))
    return out


def synthesis_grad(lmax, mmax, theta, phi, alm, nthreads=0):
    """(f, df/dtheta, df/dphi), each [B, N]."""
    lib = _load()
    th, ph = _pts(theta, phi)
    a = _alm2(alm, lmax, mmax)
    B = a.shape[0]
    f = np.zeros((B, th.size))
    dt = np.zeros((B, th.size))
    dp = np.zeros((B, th.size))
    lib.oracle_synthesis_grad(lmax, mmax, th.size, _dp(th), _dp(ph), _dp(a.view(np.float64)), B,
                              _dp(f), _dp(dt), _dp(dp), int(nthreads))
    return f, dt, dp


def lambda_column(lmax, m, theta, long_double=False):
    """lam_lm(cos theta) for l = m..lmax as (mantissa, exponent): value = mant * 2**exp."""
    lib = _load()
    n = lmax - m + 1
    mant = np.zeros(n)
    ex = np.zeros(n, dtype=np.int32)
    fn = lib.oracle_lambda_column_ld if long_double else lib.oracle_lambda_column
    fn(lmax, m, float(theta), _dp(mant), _ip(ex))
    return mant, ex


def spin_lambda_column(lmax, m, s, theta):
    """(slam_lm, (-s)lam_lm) at theta for l = 0..lmax (zero below max(m, s)), each as
    (mantissa, exponent) arrays sharing the exponent: value = mant * 2**exp."""
    lib = _load()
    pu = np.zeros(lmax + 1)
    pv = np.zeros(lmax + 1)
    ex = np.zeros(lmax + 1, dtype=np.int32)
    lib.oracle_spin_lambda_column(lmax, m, s, float(theta), _dp(pu), _dp(pv), _ip(ex))
    return pu, pv, ex


def _spin_alm(alm, lmax, mmax):
    a = np.ascontiguousarray(alm, dtype=np.complex128)
    if a.ndim == 2:
        a = a[None]
    assert a.ndim == 3 and a.shape[1] == 2 and a.shape[2] == nalm(lmax, mmax), a.shape
    return a


def spin_synthesis(lmax, mmax, s, theta, phi, alm, nthreads=0):
    """Spin-s synthesis by direct summation.  alm: [F, 2, nalm] complex (gradient G, curl C)
    -> [F, 2, N] real (Q, U)."""
    lib = _load()
    th, ph = _pts(theta, phi)
    a = _spin_alm(alm, lmax, mmax)
    out = np.zeros((a.shape[0], 2, th.size))
    lib.oracle_spin_synthesis(lmax, mmax, int(s), th.size, _dp(th), _dp(ph),
                              _dp(a.view(np.float64)), a.shape[0], _dp(out), int(nthreads))
    return out


def _spin_maps(maps, n):
    q = np.ascontiguousarray(maps, dtype=np.float64)
    if q.ndim == 2:
        q = q[None]
    assert q.ndim == 3 and q.shape[1] == 2 and q.shape[2] == n, q.shape
    return q


def spin_adjoint(lmax, mmax, s, theta, phi, maps, nthreads=0):
    """Adjoint of spin_synthesis.  maps: [F, 2, N] (Q, U) -> [F, 2, nalm] complex (G, C)."""
    lib = _load()
    th, ph = _pts(theta, phi)
    q = _spin_maps(maps, th.size)
    out = np.zeros((q.shape[0], 2, nalm(lmax, mmax)), dtype=np.complex128)
    lib.oracle_spin_adjoint(lmax, mmax, int(s), th.size, _dp(th), _dp(ph), _dp(q), q.shape[0],
                            _dp(out.view(np.float64)), int(nthreads))
    return out


def spin_adjoint_columns(lmax, s, theta, phi, maps, mlist, nthreads=0):
    """spin_adjoint restricted to the given distinct m-columns: -> [F, 2, len(mlist), lmax+1]."""
    lib = _load()
    th, ph = _pts(theta, phi)
    q = _spin_maps(maps, th.size)
    ml = np.ascontiguousarray(mlist, dtype=np.int32)
    assert len(set(ml.tolist())) == ml.size
    out = np.zeros((q.shape[0], 2, ml.size, lmax + 1), dtype=np.complex128)
    lib.oracle_spin_adjoint_columns(lmax, int(s), th.size, _dp(th), _dp(ph), _dp(q), q.shape[0],
                                    ml.size, _ip(ml), _dp(out.view(np.float64)), int(nthreads))
    return out


from .pointing import alpha_from_potential, deflect_by_alpha, pointing  # noqa: E402
from .twin import (cgls_dense, cgls_spin, density_map, mdot, mlp_backward,  # noqa: E402
                   mlp_forward, mlp_init, mlp_pack, mlp_unpack, point_features, synthesis_matrix,
                   weight_loss_dense, ylm_dense)

__all__ = [
    "build", "nalm", "alm_index", "synthesis", "adjoint", "adjoint_columns", "synthesis_grad",
    "lambda_column", "spin_lambda_column", "spin_synthesis", "spin_adjoint",
    "spin_adjoint_columns", "ylm_dense", "synthesis_matrix", "mdot", "cgls_dense", "cgls_spin",
    "mlp_init", "mlp_forward", "mlp_backward", "mlp_pack", "mlp_unpack", "density_map",
    "point_features", "weight_loss_dense", "pointing", "deflect_by_alpha", "alpha_from_potential",
]

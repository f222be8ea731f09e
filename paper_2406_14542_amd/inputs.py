"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module holds no transform arithmetic: it only draws coefficients and point sets with
numpy's PCG64 generator.  The tests, the smoke check and the benchmark feed the same
arrays to the GPU library and to the CPU oracle.

Workloads (arXiv:2406.14542, Sec. IV uses a CMB-lensing remap of a Gauss-Legendre grid of
about (lmax+1)(2 lmax+1) points deflected by a few arcminutes; the CMB spectra and lensing
simulations are not available, so these stand in for them with the same shapes):

* ``uniform_points``: cos(theta) ~ U[-1, 1], phi ~ U[0, 2 pi).
* ``deflected_grid``: an equi-angular grid of R rings x P pixels, theta_j = (j + 1/2) pi / R,
  phi_k = 2 pi k / P, each point moved by an isotropic Gaussian deflection (alpha_theta,
  alpha_phi) with the pointing formula of Appendix C, Eq. (C1).
* ``holey_points``: density proportional to (1 + 0.8 cos^2 theta) times 20 Gaussian holes
  of 5 degree radius, drawn by rejection sampling.
* ``red_alm``: a_l0 = sqrt(C_l) N(0,1), a_lm = sqrt(C_l / 2) (N(0,1) + i N(0,1)) for m > 0,
  with C_l = 1 / (l + 10)^2, drawn in m-major coefficient order.
"""
from __future__ import annotations

import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def ell_of_index(lmax: int, mmax: int) -> tuple[np.ndarray, np.ndarray]:
    """(l, m) of every coefficient in m-major order."""
    ls = np.concatenate([np.arange(m, lmax + 1) for m in range(mmax + 1)])
    ms = np.concatenate([np.full(lmax + 1 - m, m) for m in range(mmax + 1)])
    return ls, ms


def red_alm(rng: np.random.Generator, lmax: int, mmax: int, nmaps: int = 1) -> np.ndarray:
    """[nmaps, nalm] complex128 with the C_l = 1/(l+10)^2 law (real-field convention)."""
    ls, ms = ell_of_index(lmax, mmax)
    cl = 1.0 / (ls + 10.0) ** 2
    out = np.empty((nmaps, ls.size), dtype=np.complex128)
    for b in range(nmaps):
        re = rng.standard_normal(ls.size)
        im = rng.standard_normal(ls.size)
        a = np.sqrt(cl / 2.0) * (re + 1j * im)
        a[ms == 0] = np.sqrt(cl[ms == 0]) * re[ms == 0]
        out[b] = a
    return out


def spin_alm(rng: np.random.Generator, lmax: int, mmax: int, spin: int,
             nfields: int = 1) -> np.ndarray:
    """[nfields, 2, nalm] complex128 gradient/curl coefficients of spin-`spin` fields: the
    red_alm law for each of the 2 nfields rows, and 0 where l < spin (no such harmonic)."""
    ls, _ = ell_of_index(lmax, mmax)
    a = red_alm(rng, lmax, mmax, 2 * nfields).reshape(nfields, 2, ls.size)
    a[:, :, ls < spin] = 0.0
    return a


def potential_alm(rng: np.random.Generator, lmax: int, mmax: int, rms_arcmin: float) -> np.ndarray:
    """A lensing-potential-like field Phi_lm [1, nalm]: C_l proportional to l^-4 for l >= 2
    (0 below), scaled so that the rms of the gradient (the deflection) over the sphere is
    rms_arcmin: sum_l (2l+1)/(4 pi) l (l+1) C_l = rms^2.  Real-field convention as red_alm."""
    ls, ms = ell_of_index(lmax, mmax)
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    cl[2:] = ell[2:] ** -4.0
    # mean over the sphere of |grad Phi|^2 for a statistically isotropic field
    power = np.sum((2 * ell + 1) / (4 * np.pi) * ell * (ell + 1) * cl)
    cl *= (rms_arcmin * ARCMIN) ** 2 / power
    out = np.empty((1, ls.size), dtype=np.complex128)
    c = cl[ls]
    re = rng.standard_normal(ls.size)
    im = rng.standard_normal(ls.size)
    out[0] = np.where(ms == 0, np.sqrt(c) * re, np.sqrt(c / 2) * (re + 1j * im))
    return out


def uniform_points(rng: np.random.Generator, n: int) -> tuple[np.ndarray, np.ndarray]:
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.arccos(z), phi


def deflect(theta, phi, a_th, a_ph):
    """Appendix C, Eq. (C1): n' = cos(a) n + sin(a)/a (a_th e_theta + a_ph e_phi)."""
    a = np.hypot(a_th, a_ph)
    sinc = np.where(a > 0, np.sin(a) / np.where(a > 0, a, 1.0), 1.0)
    ct, st = np.cos(theta), np.sin(theta)
    cp, sp = np.cos(phi), np.sin(phi)
    ca = np.cos(a)
    nx = ca * st * cp + sinc * (a_th * ct * cp - a_ph * sp)
    ny = ca * st * sp + sinc * (a_th * ct * sp + a_ph * cp)
    nz = ca * ct + sinc * (-a_th * st)
    th2 = np.arctan2(np.hypot(nx, ny), nz)
    ph2 = np.mod(np.arctan2(ny, nx), 2.0 * np.pi)
    return th2, ph2


def deflected_grid(rng: np.random.Generator, rings: int, pix: int, rms_arcmin: float):
    th = (np.arange(rings) + 0.5) * np.pi / rings
    ph = 2.0 * np.pi * np.arange(pix) / pix
    T, P = np.meshgrid(th, ph, indexing="ij")
    T = T.ravel()
    P = P.ravel()
    sd = rms_arcmin * ARCMIN
    a_th = rng.normal(0.0, sd, T.size)
    a_ph = rng.normal(0.0, sd, T.size)
    return deflect(T, P, a_th, a_ph)


def hole_centres(rng: np.random.Generator, nholes: int = 20):
    z = rng.uniform(-1.0, 1.0, nholes)
    p = rng.uniform(0.0, 2.0 * np.pi, nholes)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(p), s * np.sin(p), z], axis=1)


def holey_density(theta, phi, centres, radius_deg: float = 5.0):
    """Unnormalised density (1 + 0.8 cos^2 theta) prod_h (1 - exp(-d_h^2 / (2 r^2)))."""
    r = np.deg2rad(radius_deg)
    st = np.sin(theta)
    n = np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=1)
    rho = 1.0 + 0.8 * np.cos(theta) ** 2
    for c in centres:
        d = np.arccos(np.clip(n @ c, -1.0, 1.0))
        rho = rho * (1.0 - np.exp(-d * d / (2.0 * r * r)))
    return rho


def holey_points(rng: np.random.Generator, n: int, nholes: int = 20, radius_deg: float = 5.0):
    centres = hole_centres(rng, nholes)
    th_out = np.empty(0)
    ph_out = np.empty(0)
    while th_out.size < n:
        k = int((n - th_out.size) * 1.8) + 1024
        th, ph = uniform_points(rng, k)
        keep = rng.uniform(0.0, 1.8, k) < holey_density(th, ph, centres, radius_deg)
        th_out = np.concatenate([th_out, th[keep]])
        ph_out = np.concatenate([ph_out, ph[keep]])
    return th_out[:n], ph_out[:n], centres


# --------------------------------------------------------------------------------------
# The five workloads.  Each returns a dict of host arrays; every draw comes from one
# default_rng(seed) in a fixed order: coefficients first, then points, then extras.
# --------------------------------------------------------------------------------------

def config_c1(seed: int = 101):
    rng = np.random.default_rng(seed)
    lmax = mmax = 127
    alm = red_alm(rng, lmax, mmax, 1)
    th, ph = uniform_points(rng, 32768)
    d = rng.standard_normal((1, th.size))
    return dict(name="c1", lmax=lmax, mmax=mmax, eps=1e-12, alm=alm, theta=th, phi=ph, d=d)


def config_c2(seed: int = 102):
    rng = np.random.default_rng(seed)
    lmax = mmax = 2047
    alm = red_alm(rng, lmax, mmax, 1)
    th, ph = deflected_grid(rng, 2048, 4095, 3.0)
    d = rng.standard_normal((1, th.size))
    return dict(name="c2", lmax=lmax, mmax=mmax, eps=1e-10, alm=alm, theta=th, phi=ph, d=d)


def config_c3(seed: int = 103, nmaps: int = 4):
    rng = np.random.default_rng(seed)
    lmax = mmax = 4095
    alm = red_alm(rng, lmax, mmax, nmaps)
    th, ph = uniform_points(rng, (lmax + 1) * (2 * lmax + 1))
    d = rng.standard_normal((nmaps, th.size))
    return dict(name="c3", lmax=lmax, mmax=mmax, eps=1e-5, eps_ref=1e-12, alm=alm, theta=th,
                phi=ph, d=d)


def config_c4(seed: int = 104, nmaps: int = 8):
    rng = np.random.default_rng(seed)
    lmax = mmax = 1023
    alm = red_alm(rng, lmax, mmax, nmaps)
    th, ph = deflected_grid(rng, 1024, 2047, 2.0)
    w = rng.uniform(0.0, 1.0, (nmaps, th.size))
    return dict(name="c4", lmax=lmax, mmax=mmax, eps=1e-12, alm=alm, theta=th, phi=ph, w=w)


def config_c5(seed: int, lmax: int = 2047, npts: int | None = None):
    rng = np.random.default_rng(seed)
    mmax = lmax
    alm = red_alm(rng, lmax, mmax, 1)
    n = int(1.5 * (lmax + 1) ** 2) if npts is None else npts
    th, ph, centres = holey_points(rng, n)
    return dict(name="c5", lmax=lmax, mmax=mmax, eps=1e-12, alm=alm, theta=th, phi=ph,
                centres=centres)

"""The C-ABI library loads and exports every function include/nusht.h declares; host-only
queries (sizes, argument validation) behave as documented.  No GPU work is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2406_14542_amd as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "nusht.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(nusht_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "nusht_plan" in names and "nusht_solve" in names and len(names) >= 14
    lib = ctypes.CDLL(P.library_path())
    for n in names:
        assert hasattr(lib, n), n


def test_nalm_and_strerror():
    assert P.nalm(127, 127) == 128 * 129 // 2
    assert P.nalm(4095, 4095) == 8390656
    assert P.nalm(10, 3) == 4 * 11 - 3 * 4 // 2
    assert P.lib().nusht_nalm(3, 4) == -1
    for code in (0, -1, -2, -3, -4, -5):
        assert P.lib().nusht_strerror(code)


@pytest.mark.parametrize("lmax", [0, 1, 7, 127, 1000, 1023, 2047, 3095, 4095, 8191])
def test_geometry_rules(lmax):
    """CC ring count N_r >= lmax + 2 with N_t = 2 (N_r - 1) smooth (the doubled count of
    Appendix B), N_phi >= 2 mmax + 2 even, fine grid >= sigma (2 lmax + 1), tile-aligned."""
    g = P.geometry(lmax, lmax, 1e-10)

    def lpf(n):
        p, b = 2, 1
        while n > 1:
            while n % p == 0:
                b, n = p, n // p
            p += 1
        return b
    assert g["nrings"] >= lmax + 2 and g["ntorus"] == 2 * (g["nrings"] - 1)
    assert lpf(g["ntorus"]) <= 7
    # minimal: no smaller admissible ring count
    for nr in range(lmax + 2, g["nrings"]):
        assert lpf(2 * (nr - 1)) > 7
    assert g["nphi"] >= 2 * lmax + 2 and g["nphi"] % 2 == 0
    assert g["n1"] >= 2.0 * (2 * lmax + 1) and g["n1"] % g["tile"] == 0
    assert g["n2"] % g["tile"] == 0 and lpf(g["n1"]) <= 7
    assert 2 <= g["width"] <= 16


def test_geometry_validation():
    lib = P.lib()
    g = P._binding.Geometry()
    bad = [(-1, 0, 1e-6, 0), (5, 6, 1e-6, 0), (5, 5, 1e-15, 0), (5, 5, 0.5, 0), (5, 5, 1e-6, 7),
           (5, 5, float("nan"), 0)]
    for a in bad:
        assert lib.nusht_geometry_for(*a, None, ctypes.byref(g)) == P.NUSHT_EINVAL, a
    assert lib.nusht_geometry_for(5, 5, 1e-8, P.NUSHT_MIXED, None, ctypes.byref(g)) == \
        P.NUSHT_EPRECISION
    o = P._binding._opts(sigma=1.25)
    assert lib.nusht_geometry_for(5, 5, 1e-12, 0, ctypes.byref(o), ctypes.byref(g)) == \
        P.NUSHT_EINVAL  # would need w > 16
    # the mixed-precision floor is 1e-6 at sigma = 2 and 1e-5 below
    assert lib.nusht_geometry_for(5, 5, 1e-6, P.NUSHT_MIXED, None, ctypes.byref(g)) == P.NUSHT_OK
    o = P._binding._opts(sigma=1.25)
    assert lib.nusht_geometry_for(5, 5, 1e-6, P.NUSHT_MIXED, ctypes.byref(o), ctypes.byref(g)) \
        == P.NUSHT_EPRECISION
    assert lib.nusht_geometry_for(5, 5, 1e-5, P.NUSHT_MIXED, ctypes.byref(o), ctypes.byref(g)) \
        == P.NUSHT_OK
    o = P._binding._opts()
    o.reserved[2] = 1
    assert lib.nusht_geometry_for(5, 5, 1e-6, 0, ctypes.byref(o), ctypes.byref(g)) == \
        P.NUSHT_EINVAL
    o = P._binding._opts()
    o.kernel_eval = 5
    assert lib.nusht_geometry_for(5, 5, 1e-6, 0, ctypes.byref(o), ctypes.byref(g)) == \
        P.NUSHT_EINVAL
    # null plan handles are rejected before any device work
    assert lib.nusht_synthesis(None, 1, 1, 1, None) == P.NUSHT_EINVAL
    assert lib.nusht_adjoint(None, 1, 1, 1, None) == P.NUSHT_EINVAL
    assert lib.nusht_synthesis_spin(None, 2, 1, 1, 1, None) == P.NUSHT_EINVAL
    assert lib.nusht_adjoint_spin(None, 2, 1, 1, 1, None) == P.NUSHT_EINVAL
    assert lib.nusht_solve_spin(None, 2, 1, 1, None, 1e-6, 5, None, None, None, None) == \
        P.NUSHT_EINVAL
    lib.nusht_destroy(None)


def _es_1d_error(w, beta, sigma=2.0, nmodes=256, npts=3000, seed=0):
    """Relative L2 error of a 1D type-2 ES nuFFT with the plan's (w, beta) -- a numpy model
    of the interpolation step (deconvolve, zero-pad, inverse FFT, w-tap ES interpolation)."""
    rng = np.random.default_rng(seed)
    K = nmodes // 2
    k = np.arange(-K, K)
    c = rng.standard_normal(k.size) + 1j * rng.standard_normal(k.size)
    x = rng.uniform(0, 2 * np.pi, npts)
    n = int(2 * np.ceil(sigma * nmodes / 2))
    h = 2 * np.pi / n
    zq, wq = np.polynomial.legendre.leggauss(400)
    t = 0.5 * np.pi * zq
    base = wq * 0.5 * np.pi * np.exp(beta * (np.cos(t) - 1)) * np.cos(t)
    I = np.array([np.sum(base * np.cos(w * np.pi / n * kk * np.sin(t))) for kk in k])
    b = c * 2.0 / (w * I)
    spec = np.zeros(n, dtype=complex)
    spec[k % n] = b
    u = np.fft.ifft(spec) * n
    tt = x / h
    ls = np.ceil(tt - w / 2).astype(int)
    f = np.zeros(npts, dtype=complex)
    for a in range(w):
        z = 2 * (tt - ls - a) / w
        q = np.clip(1 - z * z, 0, None)
        psi = np.where(q > 0, np.exp(beta * (np.sqrt(q) - 1)), 0)
        f += psi * u[(ls + a) % n]
    exact = np.exp(1j * np.outer(x, k)) @ c
    return np.linalg.norm(f - exact) / np.linalg.norm(exact)


@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-8, 1e-10, 1e-12])
def test_es_width_meets_eps_1d(eps):
    """The plan's (w, beta) for eps reaches eps/2 on a 1D model of the nuFFT step (the 2D
    error is about twice the 1D one)."""
    g = P.geometry(127, 127, eps)
    err = _es_1d_error(g["width"], g["beta"])
    assert err <= eps / 2, (eps, g["width"], err)

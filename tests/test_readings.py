"""Tests of how the paper's silent or garbled passages are read (CPU only).

* Appendix B: the printed list of good ring counts pins the sample-count relation.
* Sec. II.B / Appendix B: N_r >= lmax + 1 CC rings is not enough for the doubled map to
  carry the band limit; N_r >= lmax + 2 is.
"""
import os

import numpy as np

from paper_2406_14542_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_b_good_ring_counts.txt")


def _largest_prime_factor(n):
    p, best = 2, 1
    while n > 1:
        while n % p == 0:
            best = p
            n //= p
        p += 1
        if p * p > n and n > 1:
            best = max(best, n)
            break
    return best


def _read_golden():
    vals, under = [], []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        vals.append(int(line.rstrip("*")))
        under.append(line.endswith("*"))
    return np.array(vals), np.array(under)


def test_appendix_b_list_is_2nr_minus_2_smooth():
    """The list equals {N_r <= 10000: 4 | N_r, N_r - 1 is 11-smooth} -- equivalently
    2 N_r - 2 (the doubled CC ring count) is 11-smooth -- and the underlined entries are
    exactly those whose largest prime factor is 11.  The text's "2 N_r + 2" does not
    reproduce it."""
    vals, under = _read_golden()
    assert vals.size == 63
    mine = [n for n in range(4, 10001, 4) if _largest_prime_factor(n - 1) <= 11]
    assert mine == vals.tolist()
    doubled = [n for n in range(4, 10001, 4) if _largest_prime_factor(2 * n - 2) <= 11]
    assert doubled == vals.tolist()
    plus2 = [n for n in range(4, 10001, 4) if _largest_prime_factor(2 * n + 2) <= 11]
    assert plus2 != vals.tolist()
    lpf11 = np.array([_largest_prime_factor(n - 1) == 11 for n in vals])
    assert np.array_equal(lpf11, under)


def _dfs_eval(oracle_mod, L, nr, alm, th, ph):
    """Sample the map on nr CC rings x nphi longitudes with the oracle, double it over the
    poles (Fig. 1), take the 2D DFT and sum the Fourier series at (th, ph)."""
    nphi = 2 * L + 2
    tj = np.pi * np.arange(nr) / (nr - 1)
    pk = 2 * np.pi * np.arange(nphi) / nphi
    T, P = np.meshgrid(tj, pk, indexing="ij")
    g = oracle_mod.synthesis(L, L, T.ravel(), P.ravel(), alm)[0].reshape(nr, nphi)
    nt = 2 * (nr - 1)
    torus = np.empty((nt, nphi))
    torus[:nr] = g
    for t in range(nr, nt):
        torus[t] = np.roll(g[nt - t], -nphi // 2)
    C = np.fft.fft2(torus) / (nt * nphi)
    kap = np.fft.fftfreq(nt, 1.0 / nt)
    mu = np.fft.fftfreq(nphi, 1.0 / nphi)
    E = np.exp(1j * (np.outer(th, kap)))
    F = np.exp(1j * (np.outer(ph, mu)))
    return np.real(np.einsum("ik,kl,il->i", E, C, F))


def test_ring_count_lmax_plus_2(oracle_mod):
    """N_r = lmax + 1 rings alias the odd-m modes (sin(lmax theta) vanishes on the nodes);
    N_r = lmax + 2 reproduces the direct sum to rounding."""
    rng = np.random.default_rng(11)
    L = 7
    alm = inputs.red_alm(rng, L, L, 1)
    th, ph = inputs.uniform_points(rng, 200)
    want = oracle_mod.synthesis(L, L, th, ph, alm)[0]
    err = {}
    for nr in (L + 1, L + 2, L + 3):
        got = _dfs_eval(oracle_mod, L, nr, alm, th, ph)
        err[nr] = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err[L + 1] > 1e-3
    assert err[L + 2] < 1e-13 and err[L + 3] < 1e-13


def test_input_generators_are_seeded_and_shaped():
    a = inputs.config_c1()
    b = inputs.config_c1()
    assert np.array_equal(a["alm"], b["alm"]) and np.array_equal(a["theta"], b["theta"])
    assert a["alm"].shape == (1, inputs.nalm(127, 127)) and a["theta"].size == 32768
    _, ms = inputs.ell_of_index(127, 127)
    assert np.all(a["alm"][0, ms == 0].imag == 0)
    assert np.all((a["theta"] >= 0) & (a["theta"] <= np.pi))
    rng = np.random.default_rng(0)
    th, ph = inputs.deflected_grid(rng, 16, 31, 3.0)
    assert th.size == 16 * 31
    base = (np.arange(16) + 0.5) * np.pi / 16
    # arcminute deflections: every point stays within ~20 arcmin of its grid ring
    assert np.max(np.abs(th - np.repeat(base, 31))) < 20 * inputs.ARCMIN
    th, ph, _ = inputs.holey_points(np.random.default_rng(1), 5000)
    assert th.size == 5000 and np.all((ph >= 0) & (ph < 2 * np.pi))


def test_deflection_is_a_rotation_by_alpha():
    """Eq. (C1) moves each point by exactly the geodesic angle alpha = |(a_th, a_ph)|."""
    rng = np.random.default_rng(12)
    th, ph = inputs.uniform_points(rng, 1000)
    at = rng.normal(0, 1e-3, 1000)
    ap = rng.normal(0, 1e-3, 1000)
    t2, p2 = inputs.deflect(th, ph, at, ap)
    n1 = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    n2 = np.stack([np.sin(t2) * np.cos(p2), np.sin(t2) * np.sin(p2), np.cos(t2)])
    ang = np.arctan2(np.linalg.norm(np.cross(n1.T, n2.T), axis=1), np.sum(n1 * n2, axis=0))
    np.testing.assert_allclose(ang, np.hypot(at, ap), rtol=1e-9)

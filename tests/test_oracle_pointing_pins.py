"""Pins of the pointing oracle (arXiv:2406.14542 Appendix C, Eq. C1 and C2) against facts
that do not come from its own formula.

Eq. (C1) moves n by the angle alpha along the great circle whose initial direction is
alpha_theta e_theta + alpha_phi e_phi, so: the angle between n and n' is alpha; the
deflection direction is recovered from n' by the tangent-plane projection; a deflection
along e_theta changes theta by exactly alpha_theta; and a rotation about the z axis commutes
with the pointing.  Eq. (C2) is checked on potentials whose gradient is known in closed
form (Y_10, Y_11) and by finite differences of the direct-sum synthesis.
"""
import math

import numpy as np
import pytest

from paper_2406_14542_amd import inputs


def unit(th, ph):
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def test_geodesic_distance_and_direction(oracle_mod):
    rng = np.random.default_rng(60)
    th, ph = inputs.uniform_points(rng, 2000)
    th = np.clip(th, 1e-3, np.pi - 1e-3)
    a_th = rng.normal(0, 0.01, th.size)
    a_ph = rng.normal(0, 0.01, th.size)
    th2, ph2 = oracle_mod.deflect_by_alpha(th, ph, a_th, a_ph)
    n, n2 = unit(th, ph), unit(th2, ph2)
    # angle between n and n' (atan2 of |n x n'| and n . n', accurate for small angles)
    ang = np.arctan2(np.linalg.norm(np.cross(n.T, n2.T), axis=1), np.sum(n * n2, axis=0))
    np.testing.assert_allclose(ang, np.hypot(a_th, a_ph), rtol=1e-10, atol=1e-15)
    # initial direction: the tangent component of n' is parallel to (a_th e_th + a_ph e_ph)
    e_th = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    e_ph = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)])
    t_th = np.sum(n2 * e_th, axis=0)
    t_ph = np.sum(n2 * e_ph, axis=0)
    scale = np.sin(np.hypot(a_th, a_ph)) / np.hypot(a_th, a_ph)
    np.testing.assert_allclose(t_th, scale * a_th, rtol=0, atol=1e-15)
    np.testing.assert_allclose(t_ph, scale * a_ph, rtol=0, atol=1e-15)


def test_meridian_step_and_zero_deflection(oracle_mod):
    """alpha_phi = 0: the point moves along its meridian, theta' = theta + alpha_theta (while
    that stays inside (0, pi)), phi' = phi; alpha = 0 leaves the point where it is."""
    th = np.array([0.3, 1.0, 2.0, 2.9])
    ph = np.array([0.1, 2.0, 4.0, 6.0])
    a = np.array([0.05, -0.2, 0.3, -0.1])
    th2, ph2 = oracle_mod.deflect_by_alpha(th, ph, a, np.zeros(4))
    np.testing.assert_allclose(th2, th + a, rtol=0, atol=1e-14)
    np.testing.assert_allclose(ph2, ph, rtol=0, atol=1e-14)
    th3, ph3 = oracle_mod.deflect_by_alpha(th, ph, np.zeros(4), np.zeros(4))
    np.testing.assert_allclose(th3, th, rtol=0, atol=1e-15)
    np.testing.assert_allclose(ph3, ph, rtol=0, atol=1e-15)


def test_z_rotation_commutes(oracle_mod):
    rng = np.random.default_rng(61)
    th, ph = inputs.uniform_points(rng, 500)
    a_th, a_ph = rng.normal(0, 0.02, (2, 500))
    th2, ph2 = oracle_mod.deflect_by_alpha(th, ph, a_th, a_ph)
    th3, ph3 = oracle_mod.deflect_by_alpha(th, ph + 0.7, a_th, a_ph)
    np.testing.assert_allclose(th3, th2, rtol=0, atol=1e-14)
    d = np.angle(np.exp(1j * (ph3 - ph2 - 0.7)))
    np.testing.assert_allclose(d, 0.0, atol=1e-13)


def test_alpha_closed_forms(oracle_mod):
    """Phi = Y_10: alpha_theta = -sqrt(3/4pi) sin theta, alpha_phi = 0.  Phi = 2 Re(a Y_11)
    with a = 1: Phi = -2 sqrt(3/8pi) sin theta cos phi, so alpha_theta = -2 sqrt(3/8pi)
    cos theta cos phi and alpha_phi = (1/sin theta) dPhi/dphi = 2 sqrt(3/8pi) sin phi."""
    rng = np.random.default_rng(62)
    th, ph = inputs.uniform_points(rng, 300)
    L = 3
    a10 = np.zeros((1, inputs.nalm(L, L)), dtype=np.complex128)
    a10[0, 1] = 1.0
    at, ap = oracle_mod.alpha_from_potential(L, L, th, ph, a10)
    np.testing.assert_allclose(at, -math.sqrt(3 / (4 * math.pi)) * np.sin(th), atol=1e-15)
    np.testing.assert_allclose(ap, 0.0, atol=1e-15)
    a11 = np.zeros((1, inputs.nalm(L, L)), dtype=np.complex128)
    a11[0, (2 * L + 1 - 1) // 2 + 1] = 1.0
    at, ap = oracle_mod.alpha_from_potential(L, L, th, ph, a11)
    c = 2 * math.sqrt(3 / (8 * math.pi))
    np.testing.assert_allclose(at, -c * np.cos(th) * np.cos(ph), atol=1e-15)
    np.testing.assert_allclose(ap, c * np.sin(ph), atol=1e-14)


def test_alpha_against_finite_differences(oracle_mod):
    """Eq. (C2) on a random potential: alpha_theta and sin(theta) alpha_phi against central
    differences of the direct-sum synthesis (h = 1e-6, truncation ~ (h L)^2)."""
    rng = np.random.default_rng(63)
    L = 40
    dlm = inputs.red_alm(rng, L, L, 1)
    th, ph = inputs.uniform_points(rng, 200)
    at, ap = oracle_mod.alpha_from_potential(L, L, th, ph, dlm)
    h = 1e-6
    f = lambda t, p: oracle_mod.synthesis(L, L, t, p, dlm)[0]  # noqa: E731
    ft = (f(th + h, ph) - f(th - h, ph)) / (2 * h)
    fp = (f(th, ph + h) - f(th, ph - h)) / (2 * h)
    np.testing.assert_allclose(at, ft, rtol=0, atol=1e-7 * np.abs(ft).max())
    np.testing.assert_allclose(ap * np.sin(th), fp, rtol=0, atol=1e-7 * np.abs(fp).max())

"""Oracle of the lensing pointing (arXiv:2406.14542, Appendix C).  TEST INFRASTRUCTURE,
NOT THE PRODUCT: only tests/, the smoke check and the benchmark's CPU-baseline leg use it.

Eq. (C2): the deflection is the gradient of the lensing potential Phi,
    alpha_theta + i alpha_phi = (d/dtheta + (i / sin theta) d/dphi) Phi,
so alpha_theta = dPhi/dtheta and alpha_phi = (dPhi/dphi) / sin(theta); both derivatives of
the synthesis of Phi_lm come from the direct-sum oracle (synthesis_grad).

Eq. (C1): with n = (sin t cos p, sin t sin p, cos t), e_theta = (cos t cos p, cos t sin p,
-sin t) and e_phi = (-sin p, cos p, 0) the right-handed basis at the point, the deflected
direction is
    n' = cos(alpha) n + (sin(alpha) / alpha) (alpha_theta e_theta + alpha_phi e_phi),
alpha = sqrt(alpha_theta^2 + alpha_phi^2): a step of length alpha along the great circle that
leaves n in the direction of the deflection.  theta' = atan2(sqrt(n'_x^2 + n'_y^2), n'_z),
phi' = atan2(n'_y, n'_x) taken into [0, 2 pi).

At an exact pole (sin theta = 0) the division of Eq. (C2) is undefined; there alpha_phi is
taken as 0 (the tangent basis of Eq. C1 is still the one fixed by phi).
"""
from __future__ import annotations

import numpy as np


def deflect_by_alpha(theta, phi, a_th, a_ph):
    """Eq. (C1): deflected angles (theta', phi') of the points (theta, phi) under the
    deflection components (alpha_theta, alpha_phi)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    a_th = np.asarray(a_th, dtype=np.float64)
    a_ph = np.asarray(a_ph, dtype=np.float64)
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    n = np.stack([st * cp, st * sp, ct])
    e_th = np.stack([ct * cp, ct * sp, -st])
    e_ph = np.stack([-sp, cp, np.zeros_like(sp)])
    alpha = np.sqrt(a_th * a_th + a_ph * a_ph)
    safe = np.where(alpha > 0, alpha, 1.0)
    sinc = np.where(alpha > 0, np.sin(alpha) / safe, 1.0)
    n2 = np.cos(alpha) * n + sinc * (a_th * e_th + a_ph * e_ph)
    th2 = np.arctan2(np.sqrt(n2[0] ** 2 + n2[1] ** 2), n2[2])
    ph2 = np.arctan2(n2[1], n2[0])
    ph2 = np.where(ph2 < 0, ph2 + 2 * np.pi, ph2)
    return th2, ph2


def alpha_from_potential(lmax, mmax, theta, phi, dlm, nthreads=0):
    """Eq. (C2) by direct sums: (alpha_theta, alpha_phi) at the points for potential
    coefficients dlm [nalm] (or [1, nalm])."""
    from . import synthesis_grad
    _, dth, dph = synthesis_grad(lmax, mmax, theta, phi, np.atleast_2d(dlm), nthreads=nthreads)
    st = np.sin(np.asarray(theta, dtype=np.float64))
    a_ph = np.where(st > 0, dph[0] / np.where(st > 0, st, 1.0), 0.0)
    return dth[0], a_ph


def pointing(lmax, mmax, theta, phi, dlm, nthreads=0):
    """Deflected angles (theta', phi') of the points for the potential Phi_lm = dlm."""
    a_th, a_ph = alpha_from_potential(lmax, mmax, theta, phi, dlm, nthreads=nthreads)
    return deflect_by_alpha(theta, phi, a_th, a_ph)

"""Pins of the oracle's weighted least-squares and learned-weight pieces (CGLS, density map,
point features, weight loss, multilayer perceptron) against facts from outside the oracle:
library least squares, hand-evaluated cells and closed forms, brute-force finite
differences.  CPU only."""
import math

import numpy as np
import pytest

from paper_2406_14542_amd import inputs


def test_cgls_reaches_library_least_squares(oracle_mod):
    """CGLS after 70 iterations (81 real unknowns, a well-conditioned 300-row system) equals
    numpy's lstsq on the real synthesis matrix, unweighted and with row weights (lstsq on
    W^(1/2) A); the m = 0 imaginary parts are outside the model."""
    rng = np.random.default_rng(50)
    L = M = 8
    th, ph = inputs.uniform_points(rng, 300)
    d = rng.standard_normal(300)
    A = oracle_mod.synthesis_matrix(L, M, th, ph)
    _, ms = inputs.ell_of_index(L, M)
    n = ms.size
    keep = np.concatenate([np.ones(n, bool), ms > 0])
    for w in (None, rng.uniform(0.2, 3.0, 300)):
        sw = np.ones(300) if w is None else np.sqrt(w)
        z = np.linalg.lstsq(A[:, keep] * sw[:, None], d * sw, rcond=None)[0]
        full = np.zeros(2 * n)
        full[keep] = z
        want = full[:n] + 1j * full[n:]
        got, it, hist = oracle_mod.cgls_dense(L, M, th, ph, d, weights=w, tol=0.0, maxiter=70)
        err = math.sqrt(oracle_mod.mdot(got - want, got - want, L, M)
                        / oracle_mod.mdot(want, want, L, M))
        assert err <= 1e-10, err
        assert it == 70


def test_density_map_hand_cells(oracle_mod):
    """Points placed at known cells give rho = count / (N area / 4 pi) with the cell area
    2 pi / nph (cos(pi a / nt) - cos(pi (a + 1) / nt)); phi wraps modulo 2 pi."""
    nt, nph = 4, 8
    th = np.array([0.1, 0.2, 1.0, 3.0, 3.1])
    ph = np.array([0.1, 0.1 + 2 * np.pi, 3.2, -0.1, 6.2])
    rho = oracle_mod.density_map(th, ph, nt, nph)
    want = np.zeros((nt, nph))
    for t, p in zip(th, ph):
        a = int(t // (np.pi / nt))
        b = int((p % (2 * np.pi)) // (2 * np.pi / nph))
        want[a, b] += 1
    for a in range(nt):
        area = (math.cos(math.pi * a / nt) - math.cos(math.pi * (a + 1) / nt)) * 2 * math.pi / nph
        want[a] /= 5 * area / (4 * math.pi)
    np.testing.assert_allclose(rho, want, rtol=1e-14)
    # areas cover the sphere: sum rho * area = 4 pi for any point set
    rng = np.random.default_rng(51)
    t2, p2 = inputs.uniform_points(rng, 5000)
    r2 = oracle_mod.density_map(t2, p2, 16, 32)
    rows = np.arange(16)
    area = (np.cos(np.pi * rows / 16) - np.cos(np.pi * (rows + 1) / 16)) * 2 * np.pi / 32
    assert abs(np.sum(r2 * area[:, None]) - 4 * np.pi) <= 1e-12
    # uniform points: rho ~ 1 (Poisson spread ~ 1/sqrt(count per cell))
    assert abs(np.mean(r2) - 1.0) < 0.05


def test_point_features_special_cases(oracle_mod):
    rng = np.random.default_rng(52)
    nt, nph = 6, 12
    rho = np.exp(rng.standard_normal((nt, nph)) * 0.3)
    lr = np.log(rho)
    # a point at a cell centre: the bilinear feature is that cell's log rho, the 3 x 3 block
    # is read directly (with phi wrapping across 0 and theta clamped at the pole)
    a, b = 0, 0
    th = np.array([np.pi * (a + 0.5) / nt])
    ph = np.array([2 * np.pi * (b + 0.5) / nph])
    f = oracle_mod.point_features(th, ph, rho)[0]
    assert abs(f[0] - lr[a, b]) <= 1e-12
    block = [lr[0, nph - 1], lr[0, 0], lr[0, 1],
             lr[0, nph - 1], lr[0, 0], lr[0, 1],
             lr[1, nph - 1], lr[1, 0], lr[1, 1]]
    np.testing.assert_allclose(f[1:10], block, rtol=0, atol=1e-15)
    assert abs(f[10] - math.cos(th[0])) < 1e-15 and abs(f[11] - math.sin(th[0])) < 1e-15
    # half way between two cell centres in phi: the mean of the two
    th2 = np.array([np.pi * 2.5 / nt])
    ph2 = np.array([2 * np.pi * 4.0 / nph])
    f2 = oracle_mod.point_features(th2, ph2, rho)[0]
    assert abs(f2[0] - 0.5 * (lr[2, 3] + lr[2, 4])) <= 1e-12
    # a constant map gives constant log features
    fc = oracle_mod.point_features(*inputs.uniform_points(rng, 50), np.full((nt, nph), 2.0))
    np.testing.assert_allclose(fc[:, :10], np.log(2.0), rtol=1e-14)


def test_weight_loss_gradient_by_finite_differences(oracle_mod):
    """The loss is quadratic in w: central differences along random directions are exact up
    to rounding.  With Gauss-Legendre x equispaced-phi points and their quadrature weights
    the weighted adjoint inverts the synthesis, so the loss at those weights is ~0."""
    rng = np.random.default_rng(53)
    L = 6
    th, ph = inputs.uniform_points(rng, 200)
    a = inputs.red_alm(rng, L, L, 1)[0]
    _, ms = inputs.ell_of_index(L, L)
    Y = oracle_mod.ylm_dense(L, L, th, ph)
    d = (Y[:, ms == 0] @ a[ms == 0].real).real + 2 * (Y[:, ms > 0] @ a[ms > 0]).real
    w = rng.uniform(0.5, 1.5, 200) * 4 * np.pi / 200
    loss, g = oracle_mod.weight_loss_dense(L, L, th, ph, d, a, w)
    for _ in range(4):
        v = rng.standard_normal(200) * 4 * np.pi / 200
        h = 0.1
        lp, _ = oracle_mod.weight_loss_dense(L, L, th, ph, d, a, w + h * v)
        lm, _ = oracle_mod.weight_loss_dense(L, L, th, ph, d, a, w - h * v)
        assert abs((lp - lm) / (2 * h) - g @ v) <= 1e-10 * (abs(g @ v) + loss)
    x, gw = np.polynomial.legendre.leggauss(L + 1)
    nphi = 2 * L + 2
    tg = np.repeat(np.arccos(x), nphi)
    pg = np.tile(2 * np.pi * np.arange(nphi) / nphi, L + 1)
    wg = np.repeat(gw, nphi) * 2 * np.pi / nphi
    Yg = oracle_mod.ylm_dense(L, L, tg, pg)
    dg = (Yg[:, ms == 0] @ a[ms == 0].real).real + 2 * (Yg[:, ms > 0] @ a[ms > 0]).real
    lg, _ = oracle_mod.weight_loss_dense(L, L, tg, pg, dg, a, wg)
    assert lg <= 1e-26


def test_mlp_closed_form_one_unit(oracle_mod):
    """A 1 -> 1 -> 1 network: y = softplus(w2 tanh(w1 x + b1) + b2) * scale."""
    params = [(np.array([[0.7]]), np.array([-0.2])), (np.array([[1.3]]), np.array([0.4]))]
    x = np.array([[0.5], [-2.0], [30.0]])
    y, _ = oracle_mod.mlp_forward(params, x, scale=3.0)
    for xi, yi in zip(x[:, 0], y):
        z = 1.3 * math.tanh(0.7 * xi - 0.2) + 0.4
        assert abs(yi - 3.0 * math.log1p(math.exp(z))) <= 1e-15 * 3.0 * (1 + abs(z))
    # softplus switches to the identity for large arguments
    big = [(np.array([[1.0]]), np.array([0.0])), (np.array([[1.0]]), np.array([25.0]))]
    yb, _ = oracle_mod.mlp_forward(big, np.array([[0.0]]))
    assert abs(yb[0] - 25.0) <= 1e-12


def test_mlp_backward_by_finite_differences(oracle_mod):
    sizes = [12, 16, 16, 16, 1]
    params = oracle_mod.mlp_init(sizes, seed=3)
    rng = np.random.default_rng(54)
    X = rng.standard_normal((40, 12))
    gy = rng.standard_normal(40)
    scale = 0.7
    _, cache = oracle_mod.mlp_forward(params, X, scale)
    grads = oracle_mod.mlp_backward(params, cache, gy, scale)
    flat = oracle_mod.mlp_pack(params)
    gflat = oracle_mod.mlp_pack(grads)
    for k in rng.choice(flat.size, 40, replace=False):
        h = 1e-6
        fp = flat.copy()
        fp[k] += h
        fm = flat.copy()
        fm[k] -= h
        yp, _ = oracle_mod.mlp_forward(oracle_mod.mlp_unpack(fp, sizes), X, scale)
        ym, _ = oracle_mod.mlp_forward(oracle_mod.mlp_unpack(fm, sizes), X, scale)
        fd = float(gy @ (yp - ym)) / (2 * h)
        assert abs(fd - gflat[k]) <= 1e-7 * (1 + abs(gflat[k])), (k, fd, gflat[k])


def test_mlp_pack_layout(oracle_mod):
    """Flat layout: per layer the transposed weight [in][out], then the bias."""
    sizes = [3, 2, 1]
    params = [(np.arange(6.0).reshape(2, 3), np.array([10.0, 11.0])),
              (np.array([[20.0, 21.0]]), np.array([30.0]))]
    flat = oracle_mod.mlp_pack(params)
    assert list(flat) == [0, 3, 1, 4, 2, 5, 10, 11, 20, 21, 30]
    back = oracle_mod.mlp_unpack(flat, sizes)
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)

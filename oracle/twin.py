"""Numpy twin of the oracle for tiny sizes.  TEST INFRASTRUCTURE, NOT THE PRODUCT.

* ``ylm_dense``: the dense matrix Y of Eq. (4) of arXiv:2406.14542 (rows = points,
  columns = (l, m) with m >= 0), built column by column from the three-term recurrence,
  vectorised over points.  No exponent scaling: use it for lmax <= 64 only.
* ``synthesis_matrix``: the real-field synthesis as a real matrix acting on the stacked
  vector [Re a, Im a] (the real form of Eq. 3 for a real map).
* ``mdot``: the inner product on coefficients under which the real-field synthesis and
  Eq. (2) are exact adjoints: <a, b>_m = sum_l [Re(a_l0* b_l0) + 2 sum_{m>0} Re(a_lm* b_lm)].
* ``cgls_dense``: CGLS for min ||W^(1/2)(S a - d)|| with dense S (least squares on the
  synthesis, the setting in which transforms are called repeatedly, Sec. I).
* ``cgls_spin``: the same CGLS for one spin-s field, with S and S^H the oracle's spin-s
  synthesis and adjoint (direct sums) and <.,.>_m summed over the G and C triangles.
* ``density_map``, ``point_features``, ``weight_loss_dense``: the learned-weight inputs and
  loss for the weighted least-squares inverse, written out plainly.
* ``mlp_*``: an FP64 multilayer perceptron (tanh hidden layers, softplus output) with its
  backward pass derived by hand; it is the reference for the GPU network kernels.
"""
from __future__ import annotations

import numpy as np


def _nalm(lmax, mmax):
    return (mmax + 1) * (lmax + 1) - mmax * (mmax + 1) // 2


def _idx(lmax, l, m):
    return m * (2 * lmax + 1 - m) // 2 + l


def ylm_dense(lmax, mmax, theta, phi):
    """Y[i, index(l, m)] = lam_lm(cos theta_i) exp(i m phi_i) for m >= 0."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    assert lmax <= 64, "no exponent scaling in the twin"
    x = np.cos(theta)
    s = np.sin(theta)
    out = np.zeros((theta.size, _nalm(lmax, mmax)), dtype=np.complex128)
    pmm = np.full(theta.size, 1.0 / np.sqrt(4.0 * np.pi))
    for m in range(mmax + 1):
        if m > 0:
            pmm = pmm * (-np.sqrt((2.0 * m + 1.0) / (2.0 * m))) * s
        e = np.exp(1j * m * phi)
        lam_prev = np.zeros_like(x)
        lam = pmm.copy()
        out[:, _idx(lmax, m, m)] = lam * e
        for l in range(m + 1, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            lam, lam_prev = a * (x * lam - b * lam_prev), lam
            out[:, _idx(lmax, l, m)] = lam * e
    return out


def _mvec(lmax, mmax):
    m = np.concatenate([np.full(lmax + 1 - mm, mm) for mm in range(mmax + 1)])
    return m


def synthesis_matrix(lmax, mmax, theta, phi):
    """Real matrix A with f = A @ [Re a; Im a] for the real-field synthesis."""
    Y = ylm_dense(lmax, mmax, theta, phi)
    w = np.where(_mvec(lmax, mmax) == 0, 1.0, 2.0)
    # Re(a Y) = Re a Re Y - Im a Im Y; the m=0 imaginary part is ignored.
    im = -Y.imag * w
    im[:, _mvec(lmax, mmax) == 0] = 0.0
    return np.concatenate([Y.real * w, im], axis=1)


def mdot(a, b, lmax, mmax):
    """<a, b>_m, summed over everything but the trailing coefficient axis' weights."""
    w = np.where(_mvec(lmax, mmax) == 0, 1.0, 2.0)
    return float(np.sum(w * np.real(np.conj(a) * b)))


def cgls_dense(lmax, mmax, theta, phi, d, weights=None, x0=None, tol=1e-8, maxiter=1000):
    """CGLS on min ||W^(1/2)(S a - d)||_2 in the <.,.>_m geometry with dense matrices.

    Returns (a, iterations, history of ||d - S a|| / ||d||).  S a is the real-field
    synthesis and S^H the adjoint of Eq. (2)."""
    Y = ylm_dense(lmax, mmax, theta, phi)
    mv = _mvec(lmax, mmax)

    def S(a):
        return np.real(Y[:, mv == 0] @ a[mv == 0].real) + 2.0 * np.real(Y[:, mv > 0] @ a[mv > 0])

    def SH(f):
        c = np.conj(Y).T @ f
        c[mv == 0] = c[mv == 0].real
        return c

    w = np.ones_like(d) if weights is None else np.asarray(weights, dtype=np.float64)
    a = np.zeros(Y.shape[1], dtype=np.complex128) if x0 is None else x0.astype(np.complex128)
    u = d - S(a)
    s = SH(w * u)
    p = s.copy()
    gamma = mdot(s, s, lmax, mmax)
    dn = np.linalg.norm(d)
    hist = [np.linalg.norm(u) / dn]
    it = 0
    while hist[-1] > tol and it < maxiter:
        q = S(p)
        alpha = gamma / float(np.sum(w * q * q))
        a = a + alpha * p
        u = u - alpha * q
        s = SH(w * u)
        gnew = mdot(s, s, lmax, mmax)
        p = s + (gnew / gamma) * p
        gamma = gnew
        it += 1
        hist.append(np.linalg.norm(u) / dn)
    return a, it, np.array(hist)


def cgls_spin(lmax, mmax, spin, theta, phi, d, weights=None, x0=None, tol=1e-8, maxiter=1000):
    """cgls_dense for one spin-s field: d [2, N] (Q, U) -> (a [2, nalm] (G, C), iterations,
    history).  S is the oracle's spin synthesis, S^H its adjoint; a point's weight scales its
    Q and its U residual."""
    from . import spin_adjoint, spin_synthesis

    def S(a):
        return spin_synthesis(lmax, mmax, spin, theta, phi, a[None])[0]

    def SH(f):
        return spin_adjoint(lmax, mmax, spin, theta, phi, f[None])[0]

    d = np.asarray(d, dtype=np.float64)
    w = np.ones(d.shape[1]) if weights is None else np.asarray(weights, dtype=np.float64)
    a = np.zeros((2, _nalm(lmax, mmax)), dtype=np.complex128) if x0 is None \
        else np.array(x0, dtype=np.complex128)
    u = d - S(a)
    s = SH(w * u)
    p = s.copy()
    gamma = mdot(s, s, lmax, mmax)
    dn = np.linalg.norm(d)
    hist = [np.linalg.norm(u) / dn]
    it = 0
    while hist[-1] > tol and it < maxiter:
        q = S(p)
        alpha = gamma / float(np.sum(w * q * q))
        a = a + alpha * p
        u = u - alpha * q
        s = SH(w * u)
        gnew = mdot(s, s, lmax, mmax)
        p = s + (gnew / gamma) * p
        gamma = gnew
        it += 1
        hist.append(np.linalg.norm(u) / dn)
    return a, it, np.array(hist)


# ---------------------------------------------------------------------------------------
# FP64 multilayer perceptron: h_{k+1} = tanh(W_k h_k + b_k) for the hidden layers, then
# y = softplus(w_out . h + b_out) * scale.  Weights stored as W_k [out, in].
# ---------------------------------------------------------------------------------------

def mlp_init(sizes, seed=0):
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(sizes) - 1):
        fan_in = sizes[i]
        W = rng.standard_normal((sizes[i + 1], fan_in)) / np.sqrt(fan_in)
        b = np.zeros(sizes[i + 1])
        params.append((W, b))
    return params


def _softplus(z):
    return np.where(z > 20.0, z, np.log1p(np.exp(np.minimum(z, 20.0))))


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def mlp_forward(params, X, scale=1.0):
    """X: [N, in] -> (y [N], cache)."""
    hs = [X]
    h = X
    for W, b in params[:-1]:
        h = np.tanh(h @ W.T + b)
        hs.append(h)
    W, b = params[-1]
    z = (h @ W.T + b)[:, 0]
    return _softplus(z) * scale, (hs, z)


def mlp_backward(params, cache, gy, scale=1.0):
    """Gradients of sum(gy * y) with respect to every (W, b)."""
    hs, z = cache
    grads = [None] * len(params)
    gz = gy * scale * _sigmoid(z)
    W, b = params[-1]
    grads[-1] = (gz[None, :] @ hs[-1], np.array([gz.sum()]))
    gh = gz[:, None] * W  # [N, hidden]
    for k in range(len(params) - 2, -1, -1):
        W, b = params[k]
        h_out = hs[k + 1]
        ga = gh * (1.0 - h_out * h_out)
        grads[k] = (ga.T @ hs[k], ga.sum(axis=0))
        gh = ga @ W
    return grads


# ---------------------------------------------------------------------------------------
# Learned quadrature weights for the least-squares inverse (not in the paper; the
# definitions below are the ones the GPU kernels implement, written out plainly).
# ---------------------------------------------------------------------------------------

def density_map(theta, phi, nt, nph):
    """rho[a, b] = count of points in equal-angle cell (a, b) / (N * cell area / 4 pi).

    Cell a holds theta in [pi a / nt, pi (a + 1) / nt), cell b holds phi mod 2 pi in
    [2 pi b / nph, 2 pi (b + 1) / nph); both indices are clamped to the map.  Uniform points
    give rho ~ 1."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    a = np.clip((theta * (nt / np.pi)).astype(np.int64), 0, nt - 1)
    pw = phi - 2.0 * np.pi * np.floor(phi / (2.0 * np.pi))
    b = np.clip((pw * (nph / (2.0 * np.pi))).astype(np.int64), 0, nph - 1)
    cnt = np.zeros((nt, nph))
    np.add.at(cnt, (a, b), 1.0)
    rows = np.arange(nt)
    area = (np.cos(np.pi * rows / nt) - np.cos(np.pi * (rows + 1) / nt)) * (2.0 * np.pi / nph)
    return cnt / (theta.size * area[:, None] / (4.0 * np.pi))


def point_features(theta, phi, rho):
    """[N, 12] features of each point from the density map rho [nt, nph]:
    0: log rho bilinearly interpolated between cell centres at the point,
    1..9: log rho of the 3 x 3 cells around the point's own cell (row-major, theta clamped at
    the poles, phi periodic), 10: cos theta, 11: sin theta.  log rho is floored at log 1e-3."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    nt, nph = rho.shape
    lr = np.log(np.maximum(rho, 1e-3))

    def cell(a, b):
        return lr[np.clip(a, 0, nt - 1), np.mod(b, nph)]

    pw = phi - 2.0 * np.pi * np.floor(phi / (2.0 * np.pi))
    u = theta * (nt / np.pi) - 0.5
    v = pw * (nph / (2.0 * np.pi)) - 0.5
    a0 = np.floor(u).astype(np.int64)
    b0 = np.floor(v).astype(np.int64)
    fu = u - a0
    fv = v - b0
    out = np.empty((theta.size, 12))
    out[:, 0] = ((1 - fu) * ((1 - fv) * cell(a0, b0) + fv * cell(a0, b0 + 1))
                 + fu * ((1 - fv) * cell(a0 + 1, b0) + fv * cell(a0 + 1, b0 + 1)))
    ac = np.clip((theta * (nt / np.pi)).astype(np.int64), 0, nt - 1)
    bc = np.clip((pw * (nph / (2.0 * np.pi))).astype(np.int64), 0, nph - 1)
    q = 1
    for da in (-1, 0, 1):
        for db in (-1, 0, 1):
            out[:, q] = cell(ac + da, bc + db)
            q += 1
    out[:, 10] = np.cos(theta)
    out[:, 11] = np.sin(theta)
    return out


def weight_loss_dense(lmax, mmax, theta, phi, d, astar, w):
    """loss = <r, r>_m / <a*, a*>_m with r = S^H (w d) - a*, and its gradient with respect to
    the per-point weights: d loss / d w_i = 2 d_i (S r)_i / <a*, a*>_m."""
    Y = ylm_dense(lmax, mmax, theta, phi)
    mv = _mvec(lmax, mmax)
    c = np.conj(Y).T @ (np.asarray(w, dtype=np.float64) * d)
    c[mv == 0] = c[mv == 0].real
    r = c - astar
    den = mdot(astar, astar, lmax, mmax)
    sr = np.real(Y[:, mv == 0] @ r[mv == 0].real) + 2.0 * np.real(Y[:, mv > 0] @ r[mv > 0])
    return mdot(r, r, lmax, mmax) / den, 2.0 * d * sr / den


def mlp_pack(params):
    """Flat FP32-ready parameter vector in the layout of the GPU network: for each layer the
    transposed weight [in][out] row-major, then its bias."""
    return np.concatenate([np.concatenate([W.T.ravel(), b]) for W, b in params])


def mlp_unpack(flat, sizes):
    params = []
    o = 0
    for i in range(len(sizes) - 1):
        nin, nout = sizes[i], sizes[i + 1]
        W = np.asarray(flat[o:o + nin * nout], dtype=np.float64).reshape(nin, nout).T.copy()
        o += nin * nout
        b = np.asarray(flat[o:o + nout], dtype=np.float64).copy()
        o += nout
        params.append((W, b))
    assert o == len(flat)
    return params

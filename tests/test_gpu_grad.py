"""Gradients through the synthesis (autograd) against the oracle gradient and finite
differences.

* coefficient gradient: the loss sum(w f^2) is quadratic in a, so central differences along
  a direction are exact up to rounding;
* position gradient: against the oracle's df/dtheta, df/dphi and against central
  differences of the loss with h = 1e-6 (truncation ~ (h lmax)^2, plus eps-level noise).
"""
import numpy as np
import pytest

from paper_2406_14542_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def P():
    import paper_2406_14542_amd as P
    P.lib()
    return P


def test_deriv_kernel_matches_oracle_gradient(P, oracle_mod):
    print("[deriv vs oracle]", flush=True)
    rng = np.random.default_rng(30)
    L = 60
    th, ph = inputs.uniform_points(rng, 3000)
    th[:3] = [0.0, np.pi, 1e-7]
    alm = inputs.red_alm(rng, L, L, 5)
    pl = P.Plan(L, L, dev(th), dev(ph), 1e-12)
    f, dt, dp = (x.cpu().numpy() for x in pl.synthesis_deriv(dev(alm)))
    rf, rt, rp = oracle_mod.synthesis_grad(L, L, th, ph, alm)
    assert rel(f, rf) <= 1e-11
    assert rel(dt, rt) <= 1e-9, rel(dt, rt)
    assert rel(dp, rp) <= 1e-9, rel(dp, rp)


def test_mixed_plan_refuses_deriv(P):
    th = np.array([0.3, 1.0])
    ph = np.array([0.1, 2.0])
    pl = P.Plan(8, 8, dev(th), dev(ph), 1e-5, dtype="mixed")
    with pytest.raises(P.NushtError) as e:
        pl.synthesis_deriv(torch.zeros((1, pl.nalm), dtype=torch.complex128, device="cuda"))
    assert e.value.status == P.NUSHT_EPRECISION


def _loss(pl, a, w):
    from paper_2406_14542_amd.autograd import synthesis
    f = synthesis(pl, a)
    return (w * f * f).sum()


def test_autograd_alm_against_finite_differences(P):
    """dL/dRe a + i dL/dIm a (torch convention) against exact central differences."""
    print("[autograd alm]", flush=True)
    from paper_2406_14542_amd.autograd import synthesis
    rng = np.random.default_rng(31)
    L = 40
    th, ph = inputs.uniform_points(rng, 4000)
    a0 = inputs.red_alm(rng, L, L, 3)
    w = dev(rng.uniform(0, 1, (3, th.size)))
    pl = P.Plan(L, L, dev(th), dev(ph), 1e-12)
    a = dev(a0).requires_grad_(True)
    loss = (w * synthesis(pl, a) ** 2).sum()
    loss.backward()
    g = a.grad.cpu().numpy()
    _, ms = inputs.ell_of_index(L, L)
    assert np.all(g[:, ms == 0].imag == 0)
    for k in range(8):
        v = rng.standard_normal(a0.shape) + 1j * rng.standard_normal(a0.shape)
        v[:, ms == 0] = v[:, ms == 0].real
        h = 1e-3
        with torch.no_grad():
            lp = float((w * synthesis(pl, dev(a0 + h * v)) ** 2).sum())
            lm = float((w * synthesis(pl, dev(a0 - h * v)) ** 2).sum())
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(g.real * v.real + g.imag * v.imag))
        assert abs(fd - an) <= 1e-8 * abs(fd), (k, fd, an)


def test_autograd_positions_against_oracle_and_fd(P, oracle_mod):
    print("[autograd positions]", flush=True)
    from paper_2406_14542_amd.autograd import synthesis
    rng = np.random.default_rng(32)
    L = 48
    th0, ph0 = inputs.uniform_points(rng, 2500)
    th0 = np.clip(th0, 0.05, np.pi - 0.05)
    a0 = inputs.red_alm(rng, L, L, 2)
    wv = rng.uniform(0, 1, (2, th0.size))
    w = dev(wv)
    pl = P.Plan(L, L, dev(th0), dev(ph0), 1e-12)
    th = dev(th0).requires_grad_(True)
    ph = dev(ph0).requires_grad_(True)
    loss = (w * synthesis(pl, dev(a0), th, ph) ** 2).sum()
    loss.backward()
    gt, gp = th.grad.cpu().numpy(), ph.grad.cpu().numpy()
    f, dt, dp = oracle_mod.synthesis_grad(L, L, th0, ph0, a0)
    want_t = np.sum(2 * wv * f * dt, axis=0)
    want_p = np.sum(2 * wv * f * dp, axis=0)
    assert rel(gt, want_t) <= 1e-9 and rel(gp, want_p) <= 1e-9
    # directional central differences of the loss, each side with its own plan
    h = 1e-6
    for which in ("theta", "phi"):
        v = rng.standard_normal(th0.size)
        sign_l = []
        for sgn in (+1, -1):
            t2 = th0 + sgn * h * v if which == "theta" else th0
            p2 = ph0 + sgn * h * v if which == "phi" else ph0
            pl2 = P.Plan(L, L, dev(t2), dev(p2), 1e-12)
            with torch.no_grad():
                sign_l.append(float((w * synthesis(pl2, dev(a0)) ** 2).sum()))
        fd = (sign_l[0] - sign_l[1]) / (2 * h)
        an = float(np.dot(gt if which == "theta" else gp, v))
        assert abs(fd - an) <= 1e-5 * abs(an), (which, fd, an)


def test_autograd_refuses_other_points(P):
    """Position gradients are taken at the plan's points, so coordinates that differ from
    them (moved, or the same points in another order) are refused; the plan's own
    coordinates, as new tensors, are accepted."""
    print("[autograd point check]", flush=True)
    from paper_2406_14542_amd.autograd import synthesis
    rng = np.random.default_rng(34)
    L = 16
    th0, ph0 = inputs.uniform_points(rng, 800)
    a = dev(inputs.red_alm(rng, L, L, 1))
    pl = P.Plan(L, L, dev(th0), dev(ph0), 1e-10)
    ok = synthesis(pl, a, dev(th0.copy()).requires_grad_(True), dev(ph0).requires_grad_(True))
    assert ok.shape == (1, 800)
    perm = rng.permutation(800)
    for t, p in ((th0 + 1e-4 * rng.standard_normal(800), ph0), (th0, ph0[perm]),
                 (th0[perm], ph0[perm]), (th0[:799], ph0[:799])):
        with pytest.raises(ValueError):
            synthesis(pl, a, dev(t).requires_grad_(True), dev(p).requires_grad_(True))
    with pytest.raises(ValueError):
        synthesis(pl, a, None, dev(ph0 + 1e-3).requires_grad_(True))


def test_c4_gradients_full_size(P, oracle_mod):
    """lmax = 1023, 8 maps, the deflected 1024 x 2047 grid (2' rms): loss = sum w f^2.
    Position gradients are summed over the batch; checked against the oracle on sampled
    points, and the coefficient gradient against exact central differences."""
    print("[c4 full size]", flush=True)
    from paper_2406_14542_amd.autograd import synthesis
    cfg = inputs.config_c4()
    L = cfg["lmax"]
    th0, ph0, a0, wv = cfg["theta"], cfg["phi"], cfg["alm"], cfg["w"]
    pl = P.Plan(L, L, dev(th0), dev(ph0), cfg["eps"])
    w = dev(wv)
    a = dev(a0).requires_grad_(True)
    th = dev(th0).requires_grad_(True)
    ph = dev(ph0).requires_grad_(True)
    loss = (w * synthesis(pl, a, th, ph) ** 2).sum()
    loss.backward()
    gt, gp = th.grad.cpu().numpy(), ph.grad.cpu().numpy()
    idx = np.sort(np.random.default_rng(5).choice(th0.size, 256, replace=False))
    f, dt, dp = oracle_mod.synthesis_grad(L, L, th0[idx], ph0[idx], a0)
    want_t = np.sum(2 * wv[:, idx] * f * dt, axis=0)
    want_p = np.sum(2 * wv[:, idx] * f * dp, axis=0)
    et, ep = rel(gt[idx], want_t), rel(gp[idx], want_p)
    print(f"  position gradients vs oracle on 256 points: {et:.2e} {ep:.2e}", flush=True)
    assert et <= 1e-9 and ep <= 1e-9
    g = a.grad.cpu().numpy()
    rng = np.random.default_rng(6)
    _, ms = inputs.ell_of_index(L, L)
    v = rng.standard_normal(a0.shape) + 1j * rng.standard_normal(a0.shape)
    v[:, ms == 0] = v[:, ms == 0].real
    h = 1e-3
    with torch.no_grad():
        lp = float((w * synthesis(pl, dev(a0 + h * v)) ** 2).sum())
        lm = float((w * synthesis(pl, dev(a0 - h * v)) ** 2).sum())
    fd = (lp - lm) / (2 * h)
    an = float(np.sum(g.real * v.real + g.imag * v.imag))
    assert abs(fd - an) <= 1e-8 * abs(fd), (fd, an)

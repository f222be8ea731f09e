"""The lensing pointing of App. C on the GPU (nusht_pointing, nusht_deflect) against the
oracle's: Eq. (C1) written out in numpy, and Eq. (C2) from the direct-sum synthesis gradient.
Angles are compared as great-circle distances between the deflected directions."""
import numpy as np
import pytest

from paper_2406_14542_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def arc(t1, p1, t2, p2):
    """great-circle distance between the directions (t1, p1) and (t2, p2)"""
    def vec(t, p):
        return np.stack([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
    chord = np.linalg.norm(vec(t1, p1) - vec(t2, p2), axis=0)
    return 2.0 * np.arcsin(np.minimum(chord / 2.0, 1.0))


@pytest.fixture(scope="module")
def P():
    import paper_2406_14542_amd as P
    P.lib()
    return P


def test_deflect_matches_eq_c1(P):
    """Eq. (C1) for given deflections, including the poles, zero deflection and large steps."""
    print("[deflect]", flush=True)
    from oracle.pointing import deflect_by_alpha
    rng = np.random.default_rng(90)
    th, ph = inputs.uniform_points(rng, 50_000)
    th[:4] = [0.0, np.pi, 1e-9, np.pi - 1e-9]
    a_th = rng.normal(0, 1e-3, th.size)
    a_ph = rng.normal(0, 1e-3, th.size)
    a_th[4:8] = 0.0
    a_ph[4:8] = 0.0
    a_th[8:12] = [0.5, -1.0, 2.0, 3.0]          # steps of up to ~3 rad
    t_ref, p_ref = deflect_by_alpha(th, ph, a_th, a_ph)
    t, p = P.deflect(dev(th), dev(ph), dev(a_th), dev(a_ph))
    t, p = t.cpu().numpy(), p.cpu().numpy()
    d = arc(t, p, t_ref, p_ref)
    print(f"  max distance {d.max():.2e} rad", flush=True)
    assert d.max() <= 1e-14
    assert np.all((t >= 0) & (t <= np.pi)) and np.all((p >= 0) & (p < 2 * np.pi))
    assert np.max(np.abs(t - t_ref)) <= 1e-14


@pytest.mark.parametrize("lmax,rings", [(63, 64), (255, 256)])
def test_pointing_matches_oracle(P, oracle_mod, lmax, rings):
    """Deflected angles of an equi-angular grid (rings x (2 rings - 1) pixels, no pole rings)
    under a potential with 2.5' rms deflection, against the oracle's direct sums."""
    print(f"[pointing lmax={lmax}]", flush=True)
    from oracle.pointing import pointing as oracle_pointing
    rng = np.random.default_rng(91 + lmax)
    dlm = inputs.potential_alm(rng, lmax, lmax, 2.5)
    th = (np.arange(rings) + 0.5) * np.pi / rings
    ph = 2 * np.pi * np.arange(2 * rings - 1) / (2 * rings - 1)
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    T, Ph = T.ravel(), Ph.ravel()
    t_ref, p_ref = oracle_pointing(lmax, lmax, T, Ph, dlm[0])
    pl = P.Plan(lmax, lmax, dev(T), dev(Ph), 1e-12)
    t, p = pl.pointing(dev(dlm))
    t, p = t.cpu().numpy(), p.cpu().numpy()
    d = arc(t, p, t_ref, p_ref)
    moved = arc(T, Ph, t_ref, p_ref)
    print(f"  max distance to the oracle {d.max():.2e} rad (deflections up to "
          f"{moved.max():.2e} rad)", flush=True)
    # alpha carries the derivative synthesis' relative error (the derivative taps amplify the
    # plan's 1e-12; its gradient test allows 1e-9 at small sizes) times the gradient scale,
    # and alpha_phi = dPhi/dphi / sin(theta) amplifies it by up to 1 / sin(pi / (2 rings)) on
    # the rings next to the poles
    amp = 1.0 / np.sin(0.5 * np.pi / rings)
    assert d.max() <= 1e-10 * moved.max() * amp
    # mixed plans cannot run the derivative synthesis
    plm = P.Plan(lmax, lmax, dev(T), dev(Ph), 1e-5, dtype="mixed")
    with pytest.raises(P.NushtError) as e:
        plm.pointing(dev(dlm))
    assert e.value.status == P.NUSHT_EPRECISION

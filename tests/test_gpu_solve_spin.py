"""Spin-s CGLS inverse (nusht_solve_spin) against the oracle's spin CGLS twin, on consistent
data with and without weights, from a warm start, bit-reproducible on a deterministic plan in
the paper DFS composition, and its argument checks."""
import numpy as np
import pytest

from paper_2406_14542_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def P():
    import paper_2406_14542_amd as P
    P.lib()
    return P


def mnorm(a, L, M):
    """||a||_m over the G and C triangles of one field ([2, nalm])."""
    _, ms = inputs.ell_of_index(L, M)
    w = np.where(ms == 0, 1.0, 2.0)
    return float(np.sqrt(np.sum(w * np.abs(a) ** 2)))


@pytest.mark.parametrize("spin", [1, 2])
def test_spin_cgls_matches_twin(P, oracle_mod, spin):
    """Same iteration count, iterate and residual history as the oracle's spin CGLS (direct
    sums) on noisy data, unweighted and with point weights, at L = 12 before the iteration
    reaches its rounding floor."""
    print(f"[spin cgls vs twin] s={spin}", flush=True)
    rng = np.random.default_rng(60 + spin)
    L = M = 12
    N = 400
    th, ph = inputs.uniform_points(rng, N)
    a_true = inputs.spin_alm(rng, L, M, spin, 1)
    d = oracle_mod.spin_synthesis(L, M, spin, th, ph, a_true)[0]
    d = d + 1e-3 * rng.standard_normal(d.shape)
    pl = P.Plan(L, M, dev(th), dev(ph), 1e-13)
    for weights in (None, rng.uniform(0.5, 2.0, N).astype(np.float32)):
        wref = None if weights is None else weights.astype(np.float64)
        ref, it_ref, hist_ref = oracle_mod.cgls_spin(L, M, spin, th, ph, d, weights=wref,
                                                     tol=1e-6, maxiter=20)
        wt = None if weights is None else dev(weights)
        x, it, rr, st, hist = pl.solve_spin(spin, dev(d), weights=wt, tol=1e-6, maxiter=20,
                                            check=False, history=True)
        assert st == P.NUSHT_ENOCONV
        x = x.cpu().numpy()
        # the residual floor is ~1e-3 (the noise), so both stop at maxiter
        assert it == it_ref == 20
        assert mnorm(x - ref, L, M) <= 1e-8 * mnorm(ref, L, M)
        np.testing.assert_allclose(hist, hist_ref, rtol=1e-9, atol=0)
        ls, _ = inputs.ell_of_index(L, M)
        assert np.all(x[:, ls < spin] == 0)


@pytest.mark.parametrize("spin,dtype,eps,tol", [(2, "f64", 1e-12, 1e-8),
                                                (3, "f64", 1e-12, 1e-8),
                                                (2, "mixed", 1e-6, 1e-5)])
def test_spin_solve_consistent_data(P, spin, dtype, eps, tol):
    """Data synthesised from known coefficients (4 (L + 1)^2 random points, L = 32) are
    inverted to them, unweighted and weighted; a warm start at the solution takes no
    iteration."""
    print(f"[spin cg consistent] s={spin} {dtype}", flush=True)
    rng = np.random.default_rng(70 + spin)
    L = 32
    th, ph = inputs.uniform_points(rng, 4 * (L + 1) ** 2)
    a_true = inputs.spin_alm(rng, L, L, spin, 1)
    pl = P.Plan(L, L, dev(th), dev(ph), eps, dtype=dtype)
    d = pl.synthesis_spin(spin, dev(a_true))[0]
    ref = mnorm(a_true[0], L, L)
    x, it, rr, st = pl.solve_spin(spin, d, tol=tol, maxiter=500)
    assert st == P.NUSHT_OK and rr <= tol and it > 0
    err = mnorm(x.cpu().numpy() - a_true[0], L, L) / ref
    assert err <= 100 * tol, err
    w = dev(rng.uniform(0.5, 2.0, th.size).astype(np.float32))
    x2, it2, rr2, st2 = pl.solve_spin(spin, d, weights=w, tol=tol, maxiter=500)
    assert st2 == P.NUSHT_OK and rr2 <= tol
    assert mnorm(x2.cpu().numpy() - a_true[0], L, L) / ref <= 100 * tol
    x3, it3, rr3, st3 = pl.solve_spin(spin, d, x0=x, tol=10 * tol, maxiter=10)
    assert it3 == 0 and st3 == P.NUSHT_OK


def test_spin_solve_arguments(P):
    rng = np.random.default_rng(79)
    L = 10
    th, ph = inputs.uniform_points(rng, 500)
    pl = P.Plan(L, L, dev(th), dev(ph), 1e-10)
    d = dev(rng.standard_normal((2, 500)))
    for bad in (0, -1, L + 1):
        with pytest.raises(P.NushtError):
            pl.solve_spin(bad, d, tol=1e-6, maxiter=3)
    with pytest.raises(ValueError):
        pl.solve_spin(2, dev(rng.standard_normal((1, 500))))
    with pytest.raises(ValueError):
        pl.solve_spin(2, d, weights=dev(np.ones(499, np.float32)))
    # not converged in 3 iterations: ENOCONV, finite iterate, true residual reported
    x, it, rr, st = pl.solve_spin(2, d, tol=1e-12, maxiter=3, check=False)
    assert st == P.NUSHT_ENOCONV and it == 3 and 0 < rr < 1
    assert np.all(np.isfinite(x.cpu().numpy()))


def test_spin_solve_deterministic_paper_mode(P):
    """On a deterministic plan in the paper DFS composition, two spin solves of the same data
    give identical bits, and they agree with the fused plan's solve."""
    print("[spin cg deterministic, paper mode]", flush=True)
    rng = np.random.default_rng(78)
    L = 24
    th, ph = inputs.uniform_points(rng, 3 * (L + 1) ** 2)
    d = rng.standard_normal((2, th.size))
    pp = P.Plan(L, L, dev(th), dev(ph), 1e-12, dfs_mode="paper", deterministic=True)
    pf = P.Plan(L, L, dev(th), dev(ph), 1e-12)
    x1, it1, rr1, _ = pp.solve_spin(2, dev(d), tol=1e-6, maxiter=30, check=False)
    x2, it2, rr2, _ = pp.solve_spin(2, dev(d), tol=1e-6, maxiter=30, check=False)
    assert it1 == it2 and rr1 == rr2
    assert torch.equal(x1, x2)
    xf, itf, rrf, _ = pf.solve_spin(2, dev(d), tol=1e-6, maxiter=30, check=False)
    assert itf == it1
    x1 = x1.cpu().numpy()
    assert mnorm(xf.cpu().numpy() - x1, L, L) <= 1e-9 * mnorm(x1, L, L)

"""Pins for oracle.projection (paper Sec. 3.1, eq. simplex-tau, simplex-proj,
projF-dualpath) against brute-force KKT enumeration, an independent
threshold bisection, closed forms and the variational inequality."""
import numpy as np
import pytest

from gen import random_vector
from oracle import projection as P
from oracle import qp


@pytest.mark.parametrize("n", [1, 2, 3, 7, 50, 1000])
@pytest.mark.parametrize("kind", ["normal", "uniform", "ties"])
def test_simplex_threshold_sort_vs_bisection(n, kind):
    for seed in range(5):
        v = random_vector(n, 100 * n + seed, kind, scale=0.7)
        t1 = P.simplex_threshold_sort(v)
        t2 = P.simplex_threshold_bisect(v)
        assert abs(t1 - t2) <= 1e-12 * max(1.0, abs(t1))
        x = P.proj_simplex(v)
        assert x.min() >= 0.0
        assert abs(x.sum() - 1.0) <= 1e-13 * n
        np.testing.assert_allclose(x, np.maximum(v - t1, 0.0), rtol=0, atol=0)


def test_simplex_known_values():
    # v already on the simplex -> unchanged; uniform shift invariance
    v = np.array([0.2, 0.3, 0.5])
    np.testing.assert_allclose(P.proj_simplex(v), v, atol=1e-15)
    np.testing.assert_allclose(P.proj_simplex(v + 3.0), v, atol=1e-14)
    # a dominant coordinate takes everything
    assert np.array_equal(P.proj_simplex(np.array([5.0, 0.0, -1.0])), np.array([1.0, 0.0, 0.0]))
    # equal entries -> uniform
    np.testing.assert_allclose(P.proj_simplex(np.zeros(4)), np.full(4, 0.25), atol=1e-15)


def _bf_projection(v, mu, r):
    n = v.size
    sols = qp.brute_force(np.eye(n), -v, mu, r)
    assert sols, "brute force found no KKT point"
    xs = np.array([s[0] for s in sols])
    # all KKT points of a strictly convex problem coincide
    assert np.abs(xs - xs[0]).max() <= 1e-9
    return xs[0]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8])
def test_projF_vs_bruteforce(n):
    rng = np.random.default_rng(n)
    n_active = 0
    for trial in range(25):
        v = rng.standard_normal(n) * rng.choice([0.1, 1.0, 10.0])
        mu = rng.standard_normal(n) * 1e-3 + 5e-4
        # target between min and max of mu so F is nonempty and often binding
        r = mu.min() + rng.random() * (mu.max() - mu.min())
        x, nu, tau = P.proj_F(v, mu, r)
        xb = _bf_projection(v, mu, r)
        assert np.abs(x - xb).max() <= 1e-9, (trial, x, xb)
        n_active += nu > 0
        # KKT structure of eq. projF-dualpath: x = (v + nu mu - tau)_+
        np.testing.assert_allclose(x, np.maximum(v + nu * mu - tau, 0.0), atol=1e-12)
    assert n_active >= 5  # the active branch is exercised


def test_projF_inactive_is_simplex():
    v = random_vector(40, 7)
    mu = np.linspace(-1e-3, 1e-3, 40)
    xd = P.proj_simplex(v)
    r = mu @ xd - 1e-4  # slack -> Pi_F = Pi_Delta (Sec. 3.1)
    x, nu, _ = P.proj_F(v, mu, r)
    assert nu == 0.0
    np.testing.assert_array_equal(x, xd)


def test_projF_two_assets_segment():
    # n = 2: F is the segment x = (a, 1-a) with a in [a_lo, 1]; projection is a clamp.
    rng = np.random.default_rng(3)
    for _ in range(200):
        v = rng.standard_normal(2)
        mu = np.array([2e-3, -1e-3])
        r = rng.uniform(-1e-3, 2e-3)
        a_lo = max(0.0, (r - mu[1]) / (mu[0] - mu[1]))
        a = np.clip((v[0] - v[1] + 1.0) / 2.0, a_lo, 1.0)
        x, _, _ = P.proj_F(v, mu, r)
        np.testing.assert_allclose(x, [a, 1 - a], atol=1e-12)


def test_projF_variational_inequality():
    rng = np.random.default_rng(11)
    n = 60
    for trial in range(20):
        v = rng.standard_normal(n) * 0.05
        mu = rng.normal(4e-4, 3e-4, n)
        r = np.percentile(mu, 90)
        x, nu, _ = P.proj_F(v, mu, r)
        assert x.min() >= 0 and abs(x.sum() - 1) < 1e-12 and mu @ x >= r - 1e-15
        # feasible z: vertices with mu_i >= r and random mixtures of them with x
        verts = np.nonzero(mu >= r)[0]
        Z = [np.eye(n)[i] for i in verts]
        for _ in range(20):
            w = rng.random(len(verts))
            z = np.zeros(n)
            z[verts] = w / w.sum()
            Z.append(0.5 * z + 0.5 * x)
        for z in Z:
            assert (v - x) @ (z - x) <= 1e-12


def test_projF_infeasible_raises():
    with pytest.raises(ValueError):
        P.proj_F(np.zeros(3), np.array([1.0, 2.0, 3.0]), 3.5)


def test_projF_target_equals_max_mu():
    mu = np.array([1e-3, 3e-3, 2e-3, 3e-3])
    x, nu, _ = P.proj_F(np.array([0.5, 0.0, 0.5, 0.1]), mu, 3e-3)
    assert x[0] == 0 and x[2] == 0
    assert abs(x.sum() - 1) < 1e-14 and abs(mu @ x - 3e-3) < 1e-15


@pytest.mark.parametrize("seed", range(8))
def test_dykstra_converges_to_exact_projection(seed):
    """Dykstra's alternating projections (the paper's fallback) reach the
    exact Pi_F computed by the dual search; the half-space step is checked
    against its closed form on its own."""
    from oracle.projection import dykstra, proj_halfspace
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(2, 60))
    mu = rng.normal(5e-4, 3e-4, size=n)
    v = rng.normal(1.0 / n, 0.05, size=n)
    q = [0.2, 0.5, 0.8, 0.95][seed % 4]
    r = float(np.quantile(mu, q)) if seed % 3 else float(mu.min()) - 1e-3  # active / inactive
    x_exact, _, _ = P.proj_F(v, mu, r)
    y, k = dykstra(v, mu, r, tol=1e-14)
    assert np.abs(y - x_exact).max() <= 1e-10, (k, np.abs(y - x_exact).max())
    assert y.min() >= 0 and abs(y.sum() - 1) <= 1e-12
    # the half-space projection: feasible, and the move is along mu
    z = rng.normal(size=n)
    h = proj_halfspace(z, mu, float(mu @ z) + 1e-3)
    assert mu @ h == pytest.approx(float(mu @ z) + 1e-3, rel=1e-12)
    d = h - z
    assert np.allclose(d, (d @ mu) / (mu @ mu) * mu, rtol=0, atol=1e-15)
    assert np.array_equal(proj_halfspace(z, mu, float(mu @ z) - 1.0), z)

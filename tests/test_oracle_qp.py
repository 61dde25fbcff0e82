"""Pins for oracle.qp and oracle.reference: the exact minimiser of eq. mv
against brute-force face enumeration, textbook closed forms, scale
invariance and the KKT certificate."""
import numpy as np
import pytest

from oracle import projection as P
from oracle import qp
from oracle.reference import exact_mv


def _random_pd(rng, n, cond=50.0):
    A = rng.standard_normal((n, n))
    Qo, _ = np.linalg.qr(A)
    ev = np.geomspace(1.0, 1.0 / cond, n) * 1e-3
    return (Qo * ev) @ Qo.T


def _instance(rng, n):
    Q = _random_pd(rng, n, cond=rng.choice([5.0, 100.0, 1e4]))
    mu = rng.normal(4e-4, 3e-4, n)
    r = np.quantile(mu, rng.choice([0.0, 0.5, 0.8, 1.0]))
    return Q, mu, r


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8])
def test_active_set_vs_bruteforce(n):
    rng = np.random.default_rng(1000 + n)
    for trial in range(30):
        Q, mu, r = _instance(rng, n)
        H = 2 * Q
        sols = qp.brute_force(H, np.zeros(n), mu, r)
        assert sols
        xb = sols[0][0]
        for s in sols:
            assert np.abs(s[0] - xb).max() <= 1e-8
        x, lam, nu, _ = qp.active_set(H, np.zeros(n), mu, r, P.proj_F(np.full(n, 1 / n), mu, r)[0])
        assert np.abs(x - xb).max() <= 1e-9, (trial, x, xb)
        rep = qp.kkt_report(H, np.zeros(n), mu, r, x, lam, nu)
        assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=abs(mu).max())


def test_bruteforce_n12():
    rng = np.random.default_rng(12)
    for trial in range(2):
        Q, mu, r = _instance(rng, 12)
        H = 2 * Q
        xb = qp.brute_force(H, np.zeros(12), mu, r)[0][0]
        out = exact_mv(Q, mu, r)
        assert np.abs(out["x"] - xb).max() <= 1e-9


def test_scaled_identity_is_projection_of_zero():
    # Q = c I  =>  x* = Pi_F(0)
    rng = np.random.default_rng(5)
    n = 30
    mu = rng.normal(4e-4, 3e-4, n)
    r = np.percentile(mu, 80)
    out = exact_mv(3.7 * np.eye(n), mu, r)
    x0, _, _ = P.proj_F(np.zeros(n), mu, r)
    assert np.abs(out["x"] - x0).max() <= 1e-12


def test_global_min_variance_closed_form():
    # Q^{-1} 1 / (1^T Q^{-1} 1) when it is nonnegative and the return is slack
    rng = np.random.default_rng(6)
    n = 25
    D = np.diag(rng.uniform(1e-4, 3e-4, n))
    b = rng.uniform(0.5, 1.0, n) * 1e-2
    Q = D + 1e-3 * np.outer(b, b) / n
    w = np.linalg.solve(Q, np.ones(n))
    x_mv = w / w.sum()
    assert x_mv.min() > 0
    mu = rng.normal(4e-4, 3e-4, n)
    r = mu @ x_mv - 1e-4
    out = exact_mv(Q, mu, r)
    assert np.abs(out["x"] - x_mv).max() <= 1e-12
    assert out["nu"] == 0.0


def test_two_fund_closed_form():
    # active return, interior: x = Q^{-1}(lam 1 + nu mu)/2 with the two linear constraints
    rng = np.random.default_rng(7)
    n = 25
    D = np.diag(rng.uniform(1e-4, 3e-4, n))
    Q = D + 1e-6 * np.ones((n, n))
    mu = rng.normal(4e-4, 0.5e-4, n)
    a = np.linalg.solve(Q, np.ones(n))
    b = np.linalg.solve(Q, mu)
    x_mv = a / a.sum()
    M = 0.5 * np.array([[a.sum(), b.sum()], [mu @ a, mu @ b]])
    delta = 2e-5
    while True:  # largest tested return increment keeping the two-fund point interior
        r = mu @ x_mv + delta
        lam, nu = np.linalg.solve(M, [1.0, r])
        x2 = 0.5 * (lam * a + nu * b)
        if x2.min() > 0:
            break
        delta *= 0.5
    assert x2.min() > 0 and nu > 0 and delta > 1e-7
    out = exact_mv(Q, mu, r)
    assert np.abs(out["x"] - x2).max() <= 1e-11
    assert abs(out["nu"] - nu) <= 1e-8 * abs(nu)


def _diag_solution(d, mu, r):
    """Diagonal Q: x_i = ((lam + nu mu_i)/(2 d_i))_+ ; lam, nu by nested bisection."""
    def x_of(lam, nu):
        return np.maximum((lam + nu * mu) / (2 * d), 0.0)

    def lam_for(nu):
        lo, hi = -1.0, 1.0
        while x_of(hi, nu).sum() < 1:
            hi *= 2
        while x_of(lo, nu).sum() > 1:
            lo *= 2
        for _ in range(200):
            m = 0.5 * (lo + hi)
            if x_of(m, nu).sum() < 1:
                lo = m
            else:
                hi = m
        return 0.5 * (lo + hi)
    x0 = x_of(lam_for(0.0), 0.0)
    if mu @ x0 >= r:
        return x0
    lo, hi = 0.0, 1.0
    while mu @ x_of(lam_for(hi), hi) < r:
        hi *= 2
    for _ in range(200):
        m = 0.5 * (lo + hi)
        if mu @ x_of(lam_for(m), m) < r:
            lo = m
        else:
            hi = m
    nu = 0.5 * (lo + hi)
    return x_of(lam_for(nu), nu)


def test_diagonal_covariance():
    rng = np.random.default_rng(8)
    for trial in range(5):
        n = 40
        d = rng.uniform(1e-4, 1e-3, n)
        mu = rng.normal(4e-4, 3e-4, n)
        r = np.percentile(mu, [30, 70, 95][trial % 3])
        xd = _diag_solution(d, mu, r)
        out = exact_mv(np.diag(d), mu, r)
        assert np.abs(out["x"] - xd).max() <= 1e-9


def test_scale_invariance():
    rng = np.random.default_rng(9)
    Q, mu, r = _instance(rng, 20)
    a = exact_mv(Q, mu, r)["x"]
    b = exact_mv(123.0 * Q, mu, r)["x"]
    assert np.abs(a - b).max() <= 1e-10


def test_certificate_rejects_perturbed_point():
    # a planted mistake: the certificate must fail at a non-optimal feasible point
    rng = np.random.default_rng(10)
    Q, mu, r = _instance(rng, 15)
    out = exact_mv(Q, mu, r)
    H = 2 * Q
    rep = qp.kkt_report(H, np.zeros(15), mu, r, out["x"])
    assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=abs(mu).max())
    y = P.proj_F(out["x"] + 1e-3 * rng.standard_normal(15), mu, r)[0]
    rep2 = qp.kkt_report(H, np.zeros(15), mu, r, y)
    assert not qp.certificate_ok(rep2, tol_stat=1e-9, tol_feas=1e-12, r_scale=abs(mu).max())


def test_gap_formula():
    assert qp.gap(1.1, 1.0) == pytest.approx(0.1)
    assert qp.gap(0.9, 1.0) == 0.0
    assert qp.gap(1e-13, 0.0) == pytest.approx(0.1)

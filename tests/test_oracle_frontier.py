"""Pins of the frontier oracle (oracle/frontier.py) by properties the
parametric problem fixes, independent of the oracle's own arithmetic."""
import numpy as np
import pytest

import gen
from oracle import factor as ofactor
from oracle.frontier import frontier, min_variance
from oracle.reference import exact_mv


def _small(n, T, seed):
    spec = gen.SPECS["c1"].scaled(n, T)
    spec = type(spec)(**{**spec.__dict__, "seed": seed})
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    return mu, L


@pytest.mark.parametrize("n,T,seed,gamma", [(12, 60, 11, 0.0), (30, 150, 12, 0.0), (30, 20, 14, 1e-4)])
def test_frontier_monotone_convex_envelope(n, T, seed, gamma):
    mu, L = _small(n, T, seed)
    Q = L @ L.T + gamma * np.eye(n)
    x_mv, r_mv = min_variance(Q, mu)
    rs = np.linspace(r_mv, 0.95 * mu.max(), 9)
    fr = frontier(L, gamma, mu, rs)
    # the ridge enters f as gamma ||x||^2
    assert fr[0]["f"] == pytest.approx(float(fr[0]["x"] @ Q @ fr[0]["x"]), rel=1e-12)
    f = np.array([p["f"] for p in fr])
    scale = f.max()
    # nondecreasing and convex in r
    assert np.all(np.diff(f) >= -1e-12 * scale)
    h = rs[1] - rs[0]
    assert np.all(f[:-2] - 2 * f[1:-1] + f[2:] >= -1e-10 * scale)
    # envelope: nu*(r) lies between the one-sided difference quotients
    for j in range(1, len(rs) - 1):
        back = (f[j] - f[j - 1]) / h
        fwd = (f[j + 1] - f[j]) / h
        nu = fr[j]["nu"]
        assert back - 1e-7 * abs(fwd) <= nu <= fwd + 1e-7 * abs(fwd), (j, back, nu, fwd)
    # a central difference with a small step matches nu closely where the
    # active set does not change
    j = len(rs) // 2
    hh = 1e-4 * (rs[-1] - rs[0])
    fp = frontier(L, gamma, mu, [rs[j] + hh])[0]["f"]
    fm = frontier(L, gamma, mu, [rs[j] - hh])[0]["f"]
    assert abs((fp - fm) / (2 * hh) - fr[j]["nu"]) <= 1e-3 * abs(fr[j]["nu"]) + 1e-12


def test_frontier_start_is_min_variance():
    mu, L = _small(20, 100, 13)
    Q = L @ L.T
    x_mv, r_mv = min_variance(Q, mu)
    f_mv = float(x_mv @ Q @ x_mv)
    for r in [r_mv, r_mv - 1e-3, float(mu.min())]:
        p = frontier(L, 0.0, mu, [r])[0]
        assert p["f"] == pytest.approx(f_mv, rel=1e-9)
        assert p["nu"] <= 1e-9 * abs(p["lam"]) + 1e-15
        np.testing.assert_allclose(p["x"], x_mv, atol=1e-8)


def test_two_asset_frontier_closed_form():
    """n = 2: x = (w, 1 - w) with w = (r - mu_2)/(mu_1 - mu_2) once the return
    constraint binds, f = w^2 q11 + 2 w (1 - w) q12 + (1 - w)^2 q22."""
    L = np.array([[0.03, 0.01, -0.02], [0.01, 0.02, 0.015]])
    Q = L @ L.T
    mu = np.array([0.002, 0.0005])
    x_mv, r_mv = min_variance(Q, mu)
    # unconstrained two-asset minimiser
    w_mv = (Q[1, 1] - Q[0, 1]) / (Q[0, 0] - 2 * Q[0, 1] + Q[1, 1])
    np.testing.assert_allclose(x_mv, [w_mv, 1 - w_mv], atol=1e-10)
    for r in np.linspace(r_mv + 1e-5, 0.0019, 5):
        w = (r - mu[1]) / (mu[0] - mu[1])
        f = w * w * Q[0, 0] + 2 * w * (1 - w) * Q[0, 1] + (1 - w) ** 2 * Q[1, 1]
        s = exact_mv(Q, mu, r)
        np.testing.assert_allclose(s["x"], [w, 1 - w], atol=1e-10)
        assert s["f"] == pytest.approx(f, rel=1e-10)
        # df/dr = (df/dw)(dw/dr)
        dfdw = 2 * w * Q[0, 0] + 2 * (1 - 2 * w) * Q[0, 1] - 2 * (1 - w) * Q[1, 1]
        assert s["nu"] == pytest.approx(dfdw / (mu[0] - mu[1]), rel=1e-7)

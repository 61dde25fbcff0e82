"""Pins of the adjoint oracle (oracle/adjoint.py): central finite
differences of the exact solution map (the face checked unchanged at +-h),
the inactive-return case and the two-asset closed form."""
import numpy as np
import pytest

import gen
from oracle import factor as ofactor
from oracle.adjoint import face_is_stable, kkt_adjoint
from oracle.reference import exact_mv


def _problem(n, T, seed, q=0.6):
    spec = gen.SPECS["c5fd"].scaled(n, T)
    spec = type(spec)(**{**spec.__dict__, "seed": seed})
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu, q))
    return mu, L, r


def _loss(n, seed):
    """l(x) = x^T A x - b^T x with A PSD (an out-of-sample variance minus a
    return, the shape of the held-out loss)."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, 2 * n)) * 0.01
    A = M @ M.T / (2 * n)
    b = rng.normal(5e-4, 3e-4, n)
    return (lambda x: float(x @ A @ x - b @ x)), (lambda x: 2 * A @ x - b)


def _solve(L, gamma, mu, r):
    Q = L @ L.T + gamma * np.eye(L.shape[0])
    s = exact_mv(Q, mu, r, fista_tol=1e-12)
    return s, Q


@pytest.mark.parametrize("n,T,seed,gamma", [(12, 60, 31, 0.0), (20, 80, 32, 1e-5)])
def test_adjoint_matches_central_differences(n, T, seed, gamma):
    mu, L, r = _problem(n, T, seed)
    loss, grad = _loss(n, seed + 100)
    s, Q = _solve(L, gamma, mu, r)
    assert s["nu"] > 0, "want an active return constraint"
    assert face_is_stable(Q, mu, s["x"], s["lam"], s["nu"])
    adj = kkt_adjoint(L, gamma, mu, r, s["x"], s["lam"], s["nu"], grad(s["x"]))
    supp = set(np.flatnonzero(s["x"] > 0).tolist())

    def fd(perturb, h):
        outs = []
        for sign in (+1, -1):
            Lp, mup, rp, gp = perturb(sign * h)
            sp, _ = _solve(Lp, gp, mup, rp)
            assert set(np.flatnonzero(sp["x"] > 0).tolist()) == supp  # same face at +-h
            outs.append(loss(sp["x"]))
        return (outs[0] - outs[1]) / (2 * h)

    hm = 1e-5 * np.abs(mu).max()
    scale_mu = np.abs(adj["dmu"]).max()
    for i in range(n):
        def pm(d, i=i):
            m2 = mu.copy()
            m2[i] += d
            return L, m2, r, gamma
        assert abs(fd(pm, hm) - adj["dmu"][i]) <= 1e-4 * scale_mu + 1e-10, i
    assert fd(lambda d: (L, mu, r + d, gamma), hm) == pytest.approx(adj["dr"], rel=1e-4)
    hL = 1e-5 * np.abs(L).max()
    scale_L = np.abs(adj["dL"]).max()
    rng = np.random.default_rng(seed)
    for _ in range(6):
        i, t = int(rng.integers(n)), int(rng.integers(T))

        def pL(d, i=i, t=t):
            L2 = L.copy()
            L2[i, t] += d
            return L2, mu, r, gamma
        assert abs(fd(pL, hL) - adj["dL"][i, t]) <= 1e-4 * scale_L, (i, t)
    if gamma:
        hg = 1e-3 * gamma
        assert fd(lambda d: (L, mu, r, gamma + d), hg) == pytest.approx(adj["dgamma"], rel=1e-4)
    # dL is the sum of two outer products
    sv = np.linalg.svd(adj["dL"], compute_uv=False)
    assert sv[2] <= 1e-10 * sv[0]


def test_adjoint_inactive_return():
    """r below the minimum-variance return: the constraint is slack, nu = 0,
    and the loss does not depend on mu or r."""
    mu, L, _ = _problem(15, 70, 33)
    loss, grad = _loss(15, 133)
    r = float(mu.min()) - 1e-3
    s, Q = _solve(L, 0.0, mu, r)
    assert s["nu"] == 0.0
    adj = kkt_adjoint(L, 0.0, mu, r, s["x"], s["lam"], s["nu"], grad(s["x"]))
    assert not adj["active"]
    assert np.all(adj["dmu"] == 0.0) and adj["dr"] == 0.0
    # dL still matches finite differences
    h = 1e-5 * np.abs(L).max()
    i, t = 3, 11
    vals = []
    for sign in (+1, -1):
        L2 = L.copy()
        L2[i, t] += sign * h
        vals.append(loss(_solve(L2, 0.0, mu, r)[0]["x"]))
    assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(adj["dL"][i, t], rel=1e-4, abs=1e-9)


def test_adjoint_two_asset_closed_form():
    """n = 2 with the return constraint binding: x = (w, 1 - w),
    w = (r - mu_2)/(mu_1 - mu_2), independent of L, so dl/dL = 0 and
    dl/dmu, dl/dr follow from dw."""
    L = np.array([[0.03, 0.01, -0.02], [0.01, 0.02, 0.015]])
    mu = np.array([0.002, 0.0005])
    r = 0.0015
    s, Q = _solve(L, 0.0, mu, r)
    w = (r - mu[1]) / (mu[0] - mu[1])
    np.testing.assert_allclose(s["x"], [w, 1 - w], atol=1e-12)
    g = np.array([0.3, -0.2])
    adj = kkt_adjoint(L, 0.0, mu, r, s["x"], s["lam"], s["nu"], g)
    d = mu[0] - mu[1]
    assert np.abs(adj["dL"]).max() <= 1e-12
    np.testing.assert_allclose(adj["dmu"], [(g[0] - g[1]) * (-w / d), (g[0] - g[1]) * ((w - 1) / d)], rtol=1e-10)
    assert adj["dr"] == pytest.approx((g[0] - g[1]) / d, rel=1e-10)


@pytest.mark.slow
def test_adjoint_fd_at_config5_shape():
    """The finite-difference check at the adjoint workload's own shape:
    n = 200, T = 2000 (seed 5), r = 60th percentile of mu, loss = held-out
    variance minus held-out mean return (5000 periods, seed 105), central
    differences in float64 with h = 1e-6 on sampled mu entries (support and
    off-support), on r and on sampled entries of L; every perturbed solve
    must keep the face (support and return-row state) of the base solution."""
    spec = gen.SPECS["c5fd"]
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    r = float(np.percentile(np.asarray(Rt, dtype=np.float64).mean(axis=0), 60))
    Rh = gen.heldout_returns_TxN(spec, 5000, gen.factor_model.HELDOUT_SEED_C5)
    mu_h, L_h = ofactor.build_factor(Rh.T)
    A = L_h @ L_h.T

    def loss(x):
        return float(x @ A @ x - mu_h @ x)

    n = spec.n
    s, Q = _solve(L, 0.0, mu, r)
    assert s["nu"] > 0, "want an active return constraint"
    assert face_is_stable(Q, mu, s["x"], s["lam"], s["nu"])
    x0 = s["x"]
    adj = kkt_adjoint(L, 0.0, mu, r, x0, s["lam"], s["nu"], 2.0 * A @ x0 - mu_h)
    supp = set(np.flatnonzero(x0 > 0).tolist())
    h = 1e-6

    def solve_at(Lp, mup, rp):
        Qp = Lp @ Lp.T
        sp = exact_mv(Qp, mup, rp, fista_tol=1e-12, x0=x0)
        assert set(np.flatnonzero(sp["x"] > 0).tolist()) == supp   # same support at +-h
        assert sp["nu"] > 0                                          # return row still in the face
        return loss(sp["x"])

    def fd(perturb):
        lp = solve_at(*perturb(+h))
        lm = solve_at(*perturb(-h))
        return (lp - lm) / (2 * h)

    rng = np.random.default_rng(205)
    on = sorted(supp)
    off = [i for i in range(n) if i not in supp]
    idx = list(rng.choice(on, 6, replace=False)) + list(rng.choice(off, min(2, len(off)), replace=False))
    scale_mu = np.abs(adj["dmu"]).max()
    for i in idx:
        def pm(d, i=int(i)):
            m2 = mu.copy()
            m2[i] += d
            return L, m2, r
        assert abs(fd(pm) - adj["dmu"][i]) <= 1e-6 * scale_mu, i   # observed ~1e-8
    assert fd(lambda d: (L, mu, r + d)) == pytest.approx(adj["dr"], rel=1e-6)
    scale_L = np.abs(adj["dL"]).max()
    for _ in range(4):
        i, t = int(rng.choice(on)), int(rng.integers(spec.T))

        def pL(d, i=i, t=t):
            L2 = L.copy()
            L2[i, t] += d
            return L2, mu, r
        assert abs(fd(pL) - adj["dL"][i, t]) <= 1e-6 * scale_L, (i, t)

"""Pins for oracle.factor (Sec. 2.1), oracle.npga (Alg. 1, power-method
remark) and the seeded generator."""
import numpy as np
import pytest

import gen
from oracle import factor, npga, qp
from oracle.projection import proj_F
from oracle.reference import exact_mv, exact_mv_factor, factor_objective


def _small_panel(n=30, T=200, seed=0):
    spec = gen.SPECS["c1"].scaled(n, T)
    spec = spec.__class__(**{**spec.__dict__, "seed": seed})
    return spec, gen.returns_TxN(spec)


def test_factor_matches_numpy_cov():
    spec, Rt = _small_panel()
    mu, L = factor.build_factor(Rt.T)
    np.testing.assert_allclose(L @ L.T, np.cov(Rt.T.astype(np.float64), ddof=1), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(mu, Rt.astype(np.float64).mean(axis=0), rtol=1e-13)
    # centering: every row of L sums to zero
    assert np.abs(L.sum(axis=1)).max() <= 1e-15 * np.abs(L).sum(axis=1).max()


def test_generator_deterministic_and_chunk_invariant():
    spec = gen.SPECS["c1"]
    a = gen.returns_TxN(spec)
    b = gen.returns_TxN(spec, chunk=17)
    assert a.dtype == np.float32 and a.shape == (spec.T, spec.n)
    assert np.array_equal(a, b)
    c = gen.returns_TxN(spec.__class__(**{**spec.__dict__, "seed": 99}))
    assert not np.array_equal(a, c)


def test_generator_moments_c1():
    spec = gen.SPECS["c1"]
    Rt = gen.returns_TxN(spec).astype(np.float64)
    # idiosyncratic sd of 0.02 * t_4 is 0.02 * sqrt(2); factors add ~0.01 * |B_i|
    sd = Rt.std(axis=0)
    assert 0.02 < np.median(sd) < 0.045
    assert abs(np.mean(Rt) - spec.drift_mean) < 5e-3


def test_power_method_monotone_and_bounded():
    rng = np.random.default_rng(1)
    L = rng.standard_normal((40, 300))
    ray, _ = npga.power_method(L, 30, rng.standard_normal(40))
    s = np.linalg.norm(L, 2)
    assert np.all(np.diff(ray) >= -1e-12 * s)   # rises monotonically (Remark)
    assert ray[-1] <= s * (1 + 1e-12)
    assert ray[-1] >= 0.999 * s


def test_lipschitz_matches_eigs():
    rng = np.random.default_rng(2)
    L = rng.standard_normal((20, 50))
    m = npga.FactorModel(L, gamma=0.3)
    ev = np.linalg.eigvalsh(L @ L.T)
    assert m.lipschitz_exact() == pytest.approx(2 * ev[-1] + 0.6, rel=1e-12)


def test_npga_converges_to_exact_minimiser():
    spec, Rt = _small_panel(40, 400, seed=3)
    mu, L = factor.build_factor(Rt.T)
    r = float(np.percentile(mu, 60))
    model = npga.FactorModel(L)
    alpha = 1.0 / model.lipschitz_exact()
    out = npga.npga(model, mu, r, alpha, np.full(40, 1 / 40), tol=1e-10, max_iter=100000)
    assert out["converged"]
    ref = exact_mv_factor(L, 0.0, mu, r)
    assert np.abs(out["x"] - ref["x"]).max() <= 1e-6
    assert abs(model.value(out["x"]) - ref["f"]) <= 1e-9 * ref["f"]
    # the stopping residual vanishes at the certified minimiser (G_alpha(x*) = 0)
    p, _, _ = proj_F(ref["x"] - alpha * model.grad(ref["x"]), mu, r)
    assert np.linalg.norm(p - ref["x"]) <= 1e-12


def test_npga_residual_envelope_convex_and_ridge():
    """Qualitative regimes of Thm. npga-convergence / Sec. 5.3: the residual
    falls far faster with a ridge (strongly convex) than without."""
    spec, Rt = _small_panel(60, 50, seed=4)   # T < n: singular Sigma
    mu, L = factor.build_factor(Rt.T)
    r = float(np.median(mu))
    res = {}
    for g in (0.0, 5e-2 * np.trace(L @ L.T) / 60):
        model = npga.FactorModel(L, g)
        alpha = 1.0 / model.lipschitz_exact()
        out = npga.npga(model, mu, r, alpha, np.full(60, 1 / 60), tol=1e-8,
                        check_every=1, max_iter=20000, record=True)
        res[g > 0] = out
    assert res[True]["converged"]
    assert res[True]["iters"] < res[False]["iters"]


def test_exact_mv_certificate_c1():
    spec = gen.SPECS["c1"]
    Rt = gen.returns_TxN(spec)
    mu, L = factor.build_factor(Rt.T)
    r = gen.target_return(spec, Rt)
    out = exact_mv_factor(L, 0.0, mu, r)
    H = 2 * (L @ L.T)
    rep = qp.kkt_report(H, np.zeros(spec.n), mu, r, out["x"], out["lam"], out["nu"])
    assert qp.certificate_ok(rep, tol_stat=1e-10, tol_feas=1e-13, r_scale=abs(mu).max())
    assert out["f"] == pytest.approx(factor_objective(L, 0.0, out["x"]))


def test_constant_momentum_linear_rate():
    """Strongly convex specialization (Sec. 3.1, Thm. npga-convergence (b)):
    with m_f = 2 gamma and beta = (1 - sqrt(alpha m_f))/(1 + sqrt(alpha m_f)),
    f(x^k) - f* <= (1 - sqrt(alpha m_f))^k (f(x^0) - f* + m_f/2 ||x^0 - x*||^2)
    (the standard constant-momentum bound), and the iterates reach x*."""
    from oracle.npga import FactorModel, constant_momentum, npga
    from oracle.projection import proj_F
    from oracle.reference import exact_mv
    rng = np.random.default_rng(77)
    n, T = 20, 12                                   # rank-deficient: the ridge gives m_f > 0
    L = rng.standard_normal((n, T)) * 0.02
    mu = rng.normal(5e-4, 3e-4, n)
    r = float(np.quantile(mu, 0.6))
    gamma = 1e-3 * float(np.sum(L * L)) / n
    model = FactorModel(L, gamma)
    alpha = 1.0 / model.lipschitz_exact()
    m_f = 2.0 * gamma
    beta = constant_momentum(alpha, m_f)
    q = 1.0 - np.sqrt(alpha * m_f)
    ref = exact_mv(L @ L.T + gamma * np.eye(n), mu, r, fista_tol=1e-12)
    fstar = model.value(ref["x"])
    x0 = np.full(n, 1.0 / n)
    xp0, _, _ = proj_F(x0, mu, r)
    c0 = model.value(xp0) - fstar + 0.5 * m_f * float(np.sum((xp0 - ref["x"]) ** 2))
    for k in (10, 40, 160):
        out = npga(model, mu, r, alpha, x0, tol=0.0, check_every=10 ** 9, max_iter=k, beta_const=beta)
        gap = model.value(out["x"]) - fstar
        assert gap <= q ** k * c0 * (1 + 1e-9) + 1e-18, (k, gap, q ** k * c0)
    out = npga(model, mu, r, alpha, x0, tol=1e-12, check_every=5, max_iter=20000, beta_const=beta)
    assert out["converged"]
    np.testing.assert_allclose(out["x"], ref["x"], atol=1e-9)


@pytest.mark.parametrize("case", range(6))
def test_npga_trajectory_two_assets(case):
    """Pins the iterate trajectory of Algorithm 1 (not only its limit): with
    two assets F is the segment {(s, 1 - s) : s_min <= s <= s_max}, the
    projection is the clamp of s = (v_1 - v_2 + 1)/2, and the momentum point
    y stays on the same line.  A scalar FISTA written on s must reproduce
    every iterate of the oracle (a wrong momentum index, a gradient taken at
    x instead of y, or a missing projection would not)."""
    rng = np.random.default_rng(40 + case)
    B = rng.standard_normal((2, 2))
    Q = B @ B.T + 0.05 * np.eye(2)
    mu = rng.normal(5e-4, 3e-4, size=2)
    lo_mu, hi_mu = mu.min(), mu.max()
    r = lo_mu + (0.3 + 0.5 * rng.random()) * (hi_mu - lo_mu) if case % 2 else lo_mu - 1e-4  # active / inactive
    # feasible s range for x = (s, 1 - s): mu_2 + s (mu_1 - mu_2) >= r
    d = mu[0] - mu[1]
    if d > 0:
        s_min, s_max = max(0.0, (r - mu[1]) / d), 1.0
    else:
        s_min, s_max = 0.0, min(1.0, (r - mu[1]) / d) if d < 0 else 1.0
    alpha = 1.0 / (2.0 * np.linalg.eigvalsh(Q)[-1]) * (0.5 + 0.5 * rng.random())
    x0 = rng.random(2)
    K = 25
    out = npga.npga(npga.CovarianceModel(Q), mu, r, alpha, x0, tol=0.0, check_every=1, max_iter=0)
    traj = [out["x"]]
    for k in range(1, K + 1):
        traj.append(npga.npga(npga.CovarianceModel(Q), mu, r, alpha, x0, tol=0.0, check_every=1,
                              max_iter=k)["x"])
    # scalar FISTA on s
    clamp = lambda s: min(max(s, s_min), s_max)
    s = clamp((x0[0] - x0[1] + 1.0) / 2.0)
    s_prev, t, beta = s, 1.0, 0.0
    assert abs(traj[0][0] - s) <= 1e-14 and abs(traj[0][1] - (1 - s)) <= 1e-14
    for k in range(1, K + 1):
        ys = s + beta * (s - s_prev)
        y = np.array([ys, 1.0 - ys])
        v = y - alpha * (2.0 * Q @ y)
        s_new = clamp((v[0] - v[1] + 1.0) / 2.0)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        beta = (t - 1.0) / t_new
        t = t_new
        s_prev, s = s, s_new
        assert abs(traj[k][0] - s) <= 1e-13 and abs(traj[k][1] - (1.0 - s)) <= 1e-13, (k, traj[k], s)


def test_backtracking_accepts_admissible_steps_and_converges():
    """The backtracking rule of Sec. 3.1: from a trial step 8/L_f the
    accepted steps shrink geometrically, never below rho/L_f (the condition
    holds for every alpha <= 1/L_f), every accepted point satisfies the
    sufficient-decrease inequality, and the limit is the exact minimiser."""
    rng = np.random.default_rng(77)
    n, T = 30, 120
    L = rng.standard_normal((n, T)) / np.sqrt(T)
    mu = rng.normal(5e-4, 3e-4, size=n)
    r = float(np.quantile(mu, 0.6))
    model = npga.FactorModel(L)
    lf = model.lipschitz_exact()
    rho = 0.5
    out = npga.npga(model, mu, r, 8.0 / lf, np.full(n, 1.0 / n), tol=1e-10, max_iter=20000, backtrack=rho)
    assert out["converged"] and out["rejections"] >= 3
    assert rho / lf <= out["alpha"] <= 8.0 / lf
    # the test's rearranged form is the paper's inequality: for this
    # quadratic f, f(x) - f(y) - <grad f(y), x - y> = curv(x - y)
    for _ in range(5):
        x1, y1 = rng.standard_normal(n), rng.standard_normal(n)
        lhs = model.value(x1) - model.value(y1) - model.grad(y1) @ (x1 - y1)
        assert lhs == pytest.approx(model.curv(x1 - y1), rel=1e-10)
    ref = exact_mv_factor(L, 0.0, mu, r)
    assert np.abs(out["x"] - ref["x"]).max() <= 1e-7
    # an admissible trial step is never shrunk
    out2 = npga.npga(model, mu, r, 1.0 / lf, np.full(n, 1.0 / n), tol=1e-10, max_iter=20000, backtrack=rho)
    assert out2["rejections"] == 0 and out2["alpha"] == 1.0 / lf
    fixed = npga.npga(model, mu, r, 1.0 / lf, np.full(n, 1.0 / n), tol=1e-10, max_iter=20000)
    assert out2["iters"] == fixed["iters"] and np.array_equal(out2["x"], fixed["x"])

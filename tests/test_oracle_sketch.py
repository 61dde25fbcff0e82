"""Pins for oracle.sketch: the STR spectrum and one-sketch identities
(Sec. 2.5, App. D), and the sketch bounds of Sec. 4 measured at small
shapes where the embedding distortion eps < 1 can be computed exactly."""
import numpy as np
import pytest

import gen
from oracle import factor, sketch
from oracle.reference import exact_mv


def _L(n=64, T=4096, seed=21):
    spec = gen.SPECS["c1"].scaled(n, T)
    spec = spec.__class__(**{**spec.__dict__, "seed": seed})
    Rt = gen.returns_TxN(spec)
    mu, L = factor.build_factor(Rt.T)
    return mu, L


def test_str_spectrum_and_condition_number():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((50, 30))
    L_eff, sig, gamma = sketch.str_factor(Y, 8, 1e-2)
    Sh = sketch.str_covariance(L_eff, gamma)
    ev = np.sort(np.linalg.eigvalsh(Sh))[::-1]
    expect = np.sort(np.concatenate([sig[:8] ** 2 + gamma, np.full(42, gamma)]))[::-1]
    np.testing.assert_allclose(ev, expect, rtol=1e-11, atol=1e-12 * ev[0])
    assert ev[0] / ev[-1] == pytest.approx((sig[0] ** 2 + gamma) / gamma, rel=1e-10)
    assert gamma == pytest.approx(1e-2 * np.trace(Y @ Y.T) / 50, rel=1e-13)


def test_str_one_sketch_identity():
    # (Y V_ell)(Y V_ell)^T = U_ell S_ell^2 U_ell^T   (App. D)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((40, 25))
    U, s, V, _ = sketch.truncate(Y, 6)
    A = (Y @ V) @ (Y @ V).T
    B = (U * s ** 2) @ U.T
    np.testing.assert_allclose(A, B, atol=1e-12 * np.abs(B).max())


def test_eckart_young():
    rng = np.random.default_rng(2)
    L = rng.standard_normal((30, 60))
    S = L @ L.T
    w, Q = np.linalg.eigh(S)
    w, Q = w[::-1], Q[:, ::-1]
    for ell in (1, 5, 12):
        S_ell = (Q[:, :ell] * w[:ell]) @ Q[:, :ell].T
        assert np.linalg.norm(S - S_ell, 2) == pytest.approx(w[ell], rel=1e-10)


def test_gaussian_sketch_moments():
    S = gen.gaussian_sketch(2000, 512, seed=5).astype(np.float64)  # (k, T)
    # E[Phi Phi^T] = I_T: diagonal mean ~ 1, off-diagonal mean ~ 0
    G = S.T @ S   # T x T = Phi Phi^T
    assert abs(np.mean(np.diag(G)) - 1.0) < 0.01
    off = G[np.triu_indices(2000, 1)]
    assert abs(off.mean()) < 0.005 and abs(off.std() - 1 / np.sqrt(512)) < 0.01


@pytest.mark.parametrize("k", [512, 1024, 2048])
def test_sketch_bounds_measured_eps(k):
    mu, L = _L(n=32)
    n, T = L.shape
    Phi = gen.gaussian_sketch(T, k, seed=100 + k).astype(np.float64).T  # T x k
    eps = sketch.embedding_epsilon(L, Phi)
    assert 0 < eps < 1
    Y = sketch.sketch(L, Phi)
    Sig, Sig_t = L @ L.T, Y @ Y.T
    nS = np.linalg.norm(Sig, 2)
    # Cor. spectral: ||Sigma_tilde - Sigma|| <= eps ||Sigma||
    assert np.linalg.norm(Sig_t - Sig, 2) <= eps * nS * (1 + 1e-10)
    # App. D sandwich on the eigenvalues
    lam = np.sort(np.linalg.eigvalsh(Sig))[::-1]
    lamt = np.sort(np.linalg.eigvalsh(Sig_t))[::-1]
    assert np.all(lamt <= (1 + eps) * lam * (1 + 1e-10))
    assert np.all(lamt >= (1 - eps) * lam * (1 - 1e-10))
    # truncation bound eq. rank_lbound: lambda_{ell+1} <= lambda~_{ell+1}/(1-eps)
    for ell in (5, 20):
        assert lam[ell] <= lamt[ell] / (1 - eps) * (1 + 1e-10)
    # Thm mv-robust: value within eps ||Sigma||; solution within
    # 2 eps ||Sigma|| / (lam_min + lam~_min) <= eps kappa (2/(2-eps))
    r = float(np.percentile(mu, 60))
    a = exact_mv(Sig, mu, r)
    b = exact_mv(Sig_t, mu, r)
    assert abs(b["f"] - a["f"]) <= eps * nS
    d = np.linalg.norm(b["x"] - a["x"])
    assert d <= 2 * np.linalg.norm(Sig_t - Sig, 2) / (lam[-1] + lamt[-1])
    assert d <= eps * (lam[0] / lam[-1]) * 2 / (2 - eps)


def test_str_stability_deterministic():
    """Thm STR-stability in its deterministic form: |v^ - v*| <= ||Sigma^ - Sigma||
    and ||x^ - x*|| <= 2 ||Sigma^ - Sigma|| / (lam_min(Sigma) + gamma); plus the
    STR spectral bound with the measured eps."""
    mu, L = _L(n=32)
    n, T = L.shape
    Phi = gen.gaussian_sketch(T, 2048, seed=7).astype(np.float64).T
    eps = sketch.embedding_epsilon(L, Phi)
    Y = sketch.sketch(L, Phi)
    L_eff, sig, gamma = sketch.str_factor(Y, 12, 1e-2)
    Sh = sketch.str_covariance(L_eff, gamma)
    Sig = L @ L.T
    D = np.linalg.norm(Sh - Sig, 2)
    lam = np.sort(np.linalg.eigvalsh(Sig))[::-1]
    # eq. STR-stability-bound
    assert D <= 2 * eps * lam[0] + sig[12] ** 2 / (1 - eps) + gamma + 1e-12
    r = float(np.percentile(mu, 60))
    a = exact_mv(Sig, mu, r)
    b = exact_mv(Sh, mu, r)
    assert abs(b["f"] - a["f"]) <= D
    assert np.linalg.norm(b["x"] - a["x"]) <= 2 * D / (lam[-1] + gamma)


def test_knee_rule_and_kappa_target():
    lam = np.array([100.0, 50.0, 10.0, 9.5, 9.0, 8.9, 0.01])
    # knee: the largest i with lam_i/lam_1 >= tau and lam_{i+1}/lam_i <= rho
    assert sketch.ell_knee(lam, 1e-2, 0.9) == 6     # the final drop 8.9 -> 0.01 qualifies
    assert sketch.ell_knee(lam, 1e-1, 0.9) == 2     # tau = 0.1 leaves i <= 3; 10 -> 9.5 is no knee
    g = sketch.gamma_kappa_target(3.0, 101.0)
    assert (9.0 + g) / g == pytest.approx(101.0)


def test_countsketch_apply_matches_dense():
    """L Phi by the bucket scatter equals the product with the dense
    CountSketch matrix Phi(t, h(t)) = s(t), and E[Phi Phi^T] = I."""
    import gen
    from oracle.sketch import countsketch_apply
    rng = np.random.default_rng(8)
    L = rng.standard_normal((7, 50))
    h, s = gen.countsketch(50, 9, 4)
    Phi = np.zeros((50, 9))
    Phi[np.arange(50), h] = s
    np.testing.assert_allclose(countsketch_apply(L, h, s, 9), L @ Phi, rtol=1e-14, atol=1e-14)
    # each row of Phi has one +-1: diag(Phi Phi^T) = 1 exactly
    assert np.all(np.diag(Phi @ Phi.T) == 1.0)

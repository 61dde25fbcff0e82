"""GPU sketch-truncate-ridge build (Sec. 2.5, App. D) and STR solve against
the FP64 oracle run step by step from the identical sketch S."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import sketch as osketch
from oracle.reference import exact_mv_factor, factor_objective
from tests.gpu_util import banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


CASES = [
    (64, 256, 48, 8),
    (130, 700, 100, 20),
    (300, 2000, 256, 32),
    (517, 3001, 410, 60),
]


def _case(n, T, k, ell, seed):
    spec = spec_with("c2", n, T, seed=seed)
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    S = gen.gaussian_sketch(T, k, seed=seed + 1000)   # (k, T) float32
    return Rt, r, S


@pytest.mark.parametrize("n,T,k,ell", CASES)
def test_str_build_and_solve(npga, n, T, k, ell):
    banner(f"STR n={n} T={T} k={k} ell={ell}")
    Rt, r, S = _case(n, T, k, ell, seed=40 + n)
    L, mu = npga.build_factor(to_dev(Rt))
    Leff, sigma, gamma = npga.sketch_str(L, to_dev(S), ell, ridge_coef=1e-4)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    Y = osketch.sketch(L_o, S.astype(np.float64).T)
    Le_o, sig_o, gam_o = osketch.str_factor(Y, ell, 1e-4)
    sig = sigma.cpu().numpy().astype(np.float64)
    Le = Leff.cpu().numpy().astype(np.float64).T      # n x ell
    # singular values of Y (float32 sketch product, float64 eigensolver)
    np.testing.assert_allclose(sig, sig_o[:ell], rtol=2e-5)
    assert abs(gamma - gam_o) <= 1e-5 * gam_o
    # V_ell orthonormal eigenvectors of Y^T Y  =>  L_eff^T L_eff = diag(sigma^2)
    C = Le.T @ Le
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() <= 1e-5 * sig_o[0] ** 2
    # Sigma_hat = L_eff L_eff^T is basis independent: compare with U S^2 U^T
    Sh = Le @ Le.T
    Sh_o = Le_o @ Le_o.T
    assert np.linalg.norm(Sh - Sh_o, 2) <= 1e-5 * np.linalg.norm(Sh_o, 2)
    # STR solve parity (NPGA + refinement on the GPU factor vs the exact oracle model)
    ref = exact_mv_factor(Le_o, gam_o, mu_o, r)
    x, info = npga.solve(Leff, mu, r, gamma=gamma)
    assert info["status"] == 0, info
    xg = x.cpu().numpy().astype(np.float64)
    f_gpu = factor_objective(Le_o, gam_o, xg)
    assert xg.min() >= 0 and abs(xg.sum() - 1) <= 1e-6
    assert mu_o @ xg >= r - 1e-6 * max(1.0, abs(r))
    assert abs(f_gpu - ref["f"]) <= 1e-6 * ref["f"], (f_gpu, ref["f"])
    assert np.abs(xg - ref["x"]).max() <= 1e-5, np.abs(xg - ref["x"]).max()


def test_str_largest_k(npga):
    """k = 8192, the largest sketch size, with n = 700 < T < k: G = Y^T Y has
    rank 700, so most Householder steps see an all-zero column (tau = 0).
    Ten factors put a wide gap after sigma_10, so ell = 10 is well posed;
    the oracle truncates the float64 SVD of Y built from the same S."""
    n, T, k, ell = 700, 1000, 8192, 10
    banner(f"STR largest k: n={n} T={T} k={k} ell={ell}")
    Rt, r, S = _case(n, T, k, ell, seed=77)
    L, mu = npga.build_factor(to_dev(Rt))
    Leff, sigma, gamma = npga.sketch_str(L, to_dev(S), ell, ridge_coef=1e-4)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    Y = osketch.sketch(L_o, S.astype(np.float64).T)
    Le_o, sig_o, gam_o = osketch.str_factor(Y, ell, 1e-4)
    assert sig_o[ell - 1] > 4 * sig_o[ell]  # the gap the test relies on
    sig = sigma.cpu().numpy().astype(np.float64)
    Le = Leff.cpu().numpy().astype(np.float64).T
    np.testing.assert_allclose(sig, sig_o[:ell], rtol=2e-5)
    assert abs(gamma - gam_o) <= 1e-5 * gam_o
    C = Le.T @ Le
    assert np.abs(C - np.diag(np.diag(C))).max() <= 1e-5 * sig_o[0] ** 2
    Sh, Sh_o = Le @ Le.T, Le_o @ Le_o.T
    assert np.linalg.norm(Sh - Sh_o, 2) <= 1e-5 * np.linalg.norm(Sh_o, 2)

"""Trajectory parity of Algorithm 1: with the step fixed by the caller
(options.alpha, the same number on both sides), the GPU iterate x^k after
exactly k steps (max_iter = k, no refinement) matches the oracle's x^k, not
only the limit.  The GPU computes the gradient at y^k from those at x^k and
x^{k-1} by linearity and in float32 products; the trajectories agree to
about 5e-9 over 60 steps (bar 1e-7; 1e-6 for the batched matrix-core
products).  On the covariance path Sigma = L L^T is formed once, to float32
accuracy (entries within ~4e-7 relative): a fixed perturbation of the
quadratic that the momentum iteration carries from step to step, where the
sweep's rounding is fresh each step; there the trajectories agree to about
1e-7 at n = 37, T = 100 (bar 1e-6)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import npga as onpga
from tests.gpu_util import banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


KS = [1, 2, 3, 5, 10, 25, 60]


def _setup(n, T, seed, q):
    spec = spec_with("c2", n, T, seed=seed)
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu, q))
    model = onpga.FactorModel(L)
    alpha = 1.0 / (1.05 * model.lipschitz_exact())
    return Rt, mu, L, r, model, alpha


@pytest.mark.parametrize("path", ["gemv", "syrk"])
@pytest.mark.parametrize("n,T,q", [(64, 256, 0.6), (300, 1000, 0.8), (37, 100, 0.3)])
def test_trajectory_matches_oracle(npga, n, T, q, path):
    Rt, mu, L, r, model, alpha = _setup(n, T, 900 + n, q)
    Ld, mud = npga.build_factor(to_dev(Rt))
    worst = 0.0
    for k in KS:
        ref = onpga.npga(model, mu, r, alpha, np.full(n, 1.0 / n), tol=0.0, check_every=5, max_iter=k)
        assert not ref["converged"] and ref["iters"] == k
        x, info = npga.solve(Ld, mud, r, alpha=alpha, max_iter=k, refine=False, tol=1e-300, path=path)
        assert info["status"] == 3 and info["iters"] == k and info["alpha"] == alpha, info
        xh = x.cpu().numpy().astype(np.float64)
        assert xh.min() >= 0.0 and abs(xh.sum() - 1.0) <= 1e-6
        err = float(np.abs(xh - ref["x"]).max())
        worst = max(worst, err)
        assert err <= (1e-7 if path == "gemv" else 1e-6), (k, err)
    banner(f"trajectory n={n} T={T} {path}: max |x_gpu^k - x_oracle^k| over k in {KS} = {worst:.2e}")


@pytest.mark.parametrize("path", ["gemv", "syrk"])
def test_batched_trajectory_matches_oracle(npga, path):
    """The batched solver shares the step: each target's x^k is the oracle's
    (factor form and covariance form)."""
    n, T = 120, 600
    Rt, mu, L, r, model, alpha = _setup(n, T, 950, 0.5)
    rs = [float(np.quantile(mu, 0.3)), float(np.quantile(mu, 0.7)), float(np.quantile(mu, 0.9))]
    Ld, mud = npga.build_factor(to_dev(Rt))
    k = 20
    X, infos = npga.solve_batched(Ld, mud, rs, alpha=alpha, max_iter=k, refine=False, tol=1e-300, path=path)
    for j, rj in enumerate(rs):
        ref = onpga.npga(model, mu, rj, alpha, np.full(n, 1.0 / n), tol=0.0, check_every=5, max_iter=k)
        assert infos[j]["iters"] == k and infos[j]["alpha"] == alpha
        err = float(np.abs(X[j].cpu().numpy().astype(np.float64) - ref["x"]).max())
        banner(f"batched trajectory ({path}) target {j}: max |x_gpu^k - x_oracle^k| = {err:.2e}")
        assert err <= 1e-6, (j, err)


def test_fixed_step_solve_reaches_the_minimiser(npga):
    """A caller-fixed alpha (no estimate, step_sweeps = 0) still converges to
    the oracle's minimiser."""
    from oracle.reference import exact_mv_factor
    n, T = 64, 256
    Rt, mu, L, r, model, alpha = _setup(n, T, 960, 0.6)
    ref = exact_mv_factor(L, 0.0, mu, r)
    Ld, mud = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(Ld, mud, r, alpha=alpha)
    assert info["status"] == 0 and info["step_sweeps"] == 0 and info["alpha"] == alpha
    assert np.abs(x.cpu().numpy().astype(np.float64) - ref["x"]).max() <= 1e-5


def test_full_model_trajectory(npga):
    """At the full model (n = 5440, T = 48374; the benchmark's launch
    configuration), the first ten iterates against the oracle's.  The step
    1/(2 ||L||_F^2) (||L||_F^2 >= ||L||_2^2, so alpha <= 1/L_f) needs no
    eigen-solve on the host."""
    spec = gen.SPECS["c2"]
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    mu, L = ofactor.build_factor(Rt.T)
    alpha = 1.0 / (2.0 * float(np.sum(L * L)))
    model = onpga.FactorModel(L)
    n = L.shape[0]
    banner("full-model trajectory: device factor")
    Ld, mud = npga.build_factor(to_dev(Rt))
    del Rt
    for k in (1, 4, 10):
        ref = onpga.npga(model, mu, r, alpha, np.full(n, 1.0 / n), tol=0.0, check_every=5, max_iter=k)
        x, info = npga.solve(Ld, mud, r, alpha=alpha, max_iter=k, refine=False, tol=1e-300, path="gemv")
        assert info["status"] == 3 and info["iters"] == k
        err = float(np.abs(x.cpu().numpy().astype(np.float64) - ref["x"]).max())
        banner(f"full-model trajectory k={k}: max |x_gpu^k - x_oracle^k| = {err:.2e}")
        assert err <= 1e-7, (k, err)

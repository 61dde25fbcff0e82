"""Dykstra's alternating projections, the safeguarded fallback of the
projection (paper Sec. 3.1): on its own against the oracle's Dykstra and its
exact Pi_F, and as the step projection of a whole solve against the oracle's
minimiser."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle.projection import dykstra, proj_F
from oracle.reference import exact_mv_factor
from tests.gpu_util import banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


@pytest.mark.parametrize("n,q,seed", [(7, 0.5, 1), (64, 0.8, 2), (300, 0.3, 3), (1000, 0.9, 4), (5440, 0.6, 5)])
def test_dykstra_projection_matches_oracle(npga, n, q, seed):
    rng = np.random.default_rng(500 + seed)
    mu = rng.normal(5e-4, 3e-4, size=n)
    v = rng.normal(1.0 / n, 3.0 / n, size=n)
    r = float(np.quantile(mu, q))
    x_exact, _, _ = proj_F(v, mu, r)
    y_ref, k_ref = dykstra(v, mu, r, max_iter=5000, tol=1e-14)
    x, nu, tau, k, ok = npga.project_dykstra(to_dev(v), to_dev(mu), r, max_iter=5000, tol=1e-14)
    xh = x.cpu().numpy()
    banner(f"dykstra n={n}: gpu {k} sweeps, oracle {k_ref}; |x - exact| = {np.abs(xh - x_exact).max():.1e}")
    assert xh.min() >= 0.0 and abs(xh.sum() - 1.0) <= 1e-12
    assert np.abs(xh - y_ref).max() <= 1e-11
    if ok:
        assert np.abs(xh - x_exact).max() <= 1e-9
        # multipliers fitted on the support reproduce x = max(v + nu mu - tau, 0)
        assert np.abs(np.maximum(v + nu * mu - tau, 0.0) - xh).max() <= 1e-9


@pytest.mark.parametrize("n,T,q", [(64, 256, 0.5), (300, 1000, 0.8)])
def test_solve_with_dykstra_projections(npga, n, T, q):
    """Every step projection by Dykstra's method (options.projection): the
    minimiser is the oracle's, and the result reports it."""
    spec = spec_with("c2", n, T, seed=520 + n)
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu, q))
    ref = exact_mv_factor(L, 0.0, mu, r)
    Ld, mud = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(Ld, mud, r, projection="dykstra", path="gemv")
    x_e, info_e = npga.solve(Ld, mud, r, path="gemv")
    banner(f"dykstra solve n={n}: iters {info['iters']} (exact {info_e['iters']}), refined {info['refined']}")
    assert info["status"] == 0 and info["dykstra_used"] == 1 and info_e["dykstra_used"] == 0
    xh = x.cpu().numpy().astype(np.float64)
    assert xh.min() >= 0.0 and abs(xh.sum() - 1.0) <= 1e-6 and mu @ xh >= r - 1e-6 * max(1.0, abs(r))
    assert np.abs(xh - ref["x"]).max() <= 1e-5

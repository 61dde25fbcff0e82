"""Adaptive backtracking (paper Sec. 3.1) on the GPU against the oracle's:
the same refusals, accepted steps and iterates from a trial step eight
times 1/L_f, and the oracle's minimiser at the end."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import npga as onpga
from oracle.reference import exact_mv_factor
from tests.gpu_util import banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


@pytest.mark.parametrize("n,T,q", [(64, 256, 0.6), (300, 1000, 0.8)])
def test_backtracking_trajectory_matches_oracle(npga, n, T, q):
    spec = spec_with("c2", n, T, seed=800 + n)
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu, q))
    model = onpga.FactorModel(L)
    lf = model.lipschitz_exact()
    a0, rho = 8.0 / lf, 0.5
    Ld, mud = npga.build_factor(to_dev(Rt))
    for k in (1, 2, 5, 10, 30):
        ref = onpga.npga(model, mu, r, a0, np.full(n, 1.0 / n), tol=0.0, check_every=5, max_iter=k, backtrack=rho)
        x, info = npga.solve(Ld, mud, r, alpha=a0, backtrack_rho=rho, max_iter=k, refine=False, tol=1e-300,
                             path="gemv")
        err = float(np.abs(x.cpu().numpy().astype(np.float64) - ref["x"]).max())
        banner(f"backtracking n={n} k={k}: refusals gpu {info['backtracks']} oracle {ref['rejections']}, "
               f"alpha*L_f gpu {info['alpha'] * lf:.4f} oracle {ref['alpha'] * lf:.4f}, |dx| {err:.1e}")
        assert info["iters"] == k and info["backtracks"] == ref["rejections"]
        assert info["alpha"] == pytest.approx(ref["alpha"], rel=1e-15)
        assert err <= 1e-7, (k, err)


def test_backtracking_solve_reaches_the_minimiser(npga):
    n, T = 120, 600
    spec = spec_with("c2", n, T, seed=830)
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu, 0.7))
    ref = exact_mv_factor(L, 0.0, mu, r)
    lf = onpga.FactorModel(L).lipschitz_exact()
    Ld, mud = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(Ld, mud, r, alpha=16.0 / lf, backtrack_rho=0.5, path="gemv")
    banner(f"backtracking solve: {info['iters']} iterations, {info['backtracks']} refusals, "
           f"alpha*L_f {info['alpha'] * lf:.3f}")
    assert info["status"] == 0 and info["backtracks"] >= 1
    assert 0.5 / lf <= info["alpha"] <= 16.0 / lf
    assert np.abs(x.cpu().numpy().astype(np.float64) - ref["x"]).max() <= 1e-5

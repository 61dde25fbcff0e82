"""Edge cases of the GPU path: the smallest and largest sizes, a single
feasible vertex, constant returns, the largest batch, non-finite data, and
degenerate faces for the adjoint; compared with the oracle where a
minimiser exists."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import qp
from oracle.reference import exact_mv_factor
from tests.golden.make_golden import panel_digest
from tests.gpu_util import banner, spec_with, to_dev
from tests.test_gpu_solve import _check_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


def _factor(n, T, seed, K=3):
    spec = spec_with("c2", n, T, seed=seed)
    spec = spec.__class__(**{**spec.__dict__, "K": K})
    Rt = gen.returns_TxN(spec)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    return Rt, mu_o, L_o


@pytest.mark.parametrize("n,T", [(1, 2), (1, 50), (2, 2), (3, 9), (4, 3)])
def test_tiny_problems(npga, n, T):
    Rt, mu_o, L_o = _factor(n, T, 700 + 10 * n + T, K=1)
    r = float(np.quantile(mu_o, 0.5))
    ref = exact_mv_factor(L_o, 1e-8, mu_o, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, gamma=1e-8)
    assert info["status"] == 0, info
    _check_parity(x.cpu().numpy(), info, L_o, mu_o, r, 1e-8, ref, f"{n}x{T}")
    X, infos = npga.solve_batched(L, mu, [r, float(mu_o.min())], gamma=1e-8)
    assert all(i["status"] == 0 for i in infos)
    assert np.abs(X[0].cpu().numpy() - ref["x"]).max() <= 1e-5


def test_single_asset(npga):
    """n = 1: the only feasible point is x = 1 (r <= mu_1)."""
    Rt, mu_o, L_o = _factor(1, 100, 711, K=1)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, float(mu_o[0]) - 1e-6)
    assert info["status"] == 0 and float(x[0]) == 1.0
    with pytest.raises(npga.NpgaError):
        npga.solve(L, mu, float(mu_o[0]) + 1e-6)


N8192 = os.path.join(os.path.dirname(__file__), "golden", "n8192_solution.json")


@pytest.mark.skipif(not os.path.exists(N8192), reason="n8192 golden not generated")
def test_largest_n(npga):
    """n = 8192 (the largest supported), T < n with a ridge: every slot of
    the register-resident vectors is in use; against the stored oracle
    solution (tests/golden/make_golden.py n8192)."""
    with open(N8192) as fh:
        ref = json.load(fh)
    n, T = 8192, 600
    Rt, mu_o, L_o = _factor(n, T, 712, K=5)
    assert panel_digest(Rt) == ref["panel_sha256"]
    gamma, r = ref["gamma"], ref["r"]
    L, mu = npga.build_factor(to_dev(Rt))
    banner("n=8192: solve")
    x, info = npga.solve(L, mu, r, gamma=gamma)
    banner(f"n=8192: iters {info['iters']} refine {info['refine_iters']} refined {info['refined']}")
    assert info["status"] == 0 and info["refined"] == 1
    _check_parity(x.cpu().numpy(), info, L_o, mu_o, r, gamma,
                  {"x": np.asarray(ref["x"]), "f": ref["objective"]}, "n=8192")
    X, infos = npga.solve_batched(L, mu, [r, float(np.quantile(mu_o, 0.3))], gamma=gamma)
    assert all(i["status"] == 0 for i in infos)
    assert np.abs(X[0].cpu().numpy() - np.asarray(ref["x"])).max() <= 1e-5


def test_constant_returns(npga):
    """mu constant: the return row repeats the budget row (a singular face);
    with r equal to that constant the minimiser is the minimum-variance
    portfolio."""
    Rt, mu_o, L_o = _factor(50, 400, 713)
    c = 3e-4
    Rt = (Rt - Rt.mean(axis=0, keepdims=True) + np.float32(c)).astype(np.float32)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    r = float(mu_o.min())
    ref = exact_mv_factor(L_o, 0.0, mu_o, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r)
    assert info["status"] == 0
    _check_parity(x.cpu().numpy(), info, L_o, mu_o, r, 0.0, ref, "constant mu")


def test_largest_batch(npga):
    """m = 1024 targets on a small factor: the batch limit."""
    n, T, m = 64, 256, 1024
    Rt, mu_o, L_o = _factor(n, T, 714)
    L, mu = npga.build_factor(to_dev(Rt))
    rs = np.linspace(float(np.quantile(mu_o, 0.2)), 0.95 * float(mu_o.max()), m)
    X, infos = npga.solve_batched(L, mu, rs)
    assert all(i["status"] == 0 for i in infos)
    for j in (0, 511, 1023):
        ref = exact_mv_factor(L_o, 0.0, mu_o, float(rs[j]))
        _check_parity(X[j].cpu().numpy(), infos[j], L_o, mu_o, float(rs[j]), 0.0, ref, f"target {j}")
    with pytest.raises(npga.NpgaError):
        npga.solve_batched(L, mu, np.linspace(0, 1e-4, 1025))


def test_nonfinite_factor(npga):
    """A NaN in L itself (not caught by the factor build) ends the solve with
    NPGA_ERR_NUMERIC instead of returning garbage."""
    Rt, mu_o, L_o = _factor(40, 200, 715)
    L, mu = npga.build_factor(to_dev(Rt))
    L[7, 3] = float("nan")
    with pytest.raises(npga.NpgaError) as e:
        npga.solve(L, mu, float(np.quantile(mu_o, 0.5)))
    assert e.value.code == 5


def test_adjoint_degenerate_vertex(npga):
    """r = max mu: x* is the vertex e_i; the face is a single point and the
    adjoint flags it as degenerate (|S| = 1) with finite outputs."""
    Rt, mu_o, L_o = _factor(30, 200, 716)
    L, mu = npga.build_factor(to_dev(Rt))
    r = float(mu.max().item())
    x, info = npga.solve(L, mu, r)
    xh = x.cpu().numpy()
    assert (xh > 0).sum() == 1
    g = np.random.default_rng(3).standard_normal(30).astype(np.float32)
    dmu, dL, binfo = npga.backward(L, mu, r, x, to_dev(g))
    assert binfo["degenerate"] == 1 and binfo["support"] == 1
    assert torch.isfinite(dmu).all() and torch.isfinite(dL).all()


class _FactorHessian:
    """H = 2 L L^T applied in factor form (the oracle's KKT report only
    forms H x)."""

    def __init__(self, L):
        self.L = L

    def __matmul__(self, x):
        return 2.0 * (self.L @ (self.L.T @ x))


@pytest.mark.parametrize("n,T", [(7000, 7200), (8192, 8192)])
def test_preconditioned_refinement_largest(npga, n, T):
    """The preconditioned face CG at 14 and 16 rows per thread (n > 6144 with
    cols >= n): the float64 KKT certificate of the returned x computed in
    factor form (a dense oracle solve does not finish in seconds at this
    size), at the bar of the other certificate test (float32 x: 1e-4 of the
    gradient), and the same minimiser as the plain face CG."""
    banner(f"preconditioned refinement n={n} T={T}")
    Rt, mu_o, L_o = _factor(n, T, 900 + n, K=10)
    r = float(np.quantile(mu_o, 0.6))
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, path="gemv")
    assert info["status"] == 0 and info["refined"] == 1, info
    xp, infop = npga.solve(L, mu, r, path="gemv", refine_precond=False)
    assert infop["status"] == 0 and infop["refined"] == 1, infop
    xh = x.cpu().numpy().astype(np.float64)
    rep = qp.kkt_report(_FactorHessian(L_o), np.zeros(n), mu_o, r, xh,
                        act_tol=1e-6 * max(abs(r), np.abs(mu_o).max()))
    assert rep["min_x"] >= 0.0 and rep["budget"] <= 1e-6, rep
    assert rep["ret_slack"] >= -1e-6 * max(1.0, abs(r)), rep
    assert rep["stat_support"] <= 1e-4 and rep["dual_offsupport"] >= -1e-4, rep
    assert np.abs(xh - xp.cpu().numpy()).max() <= 1e-5
    assert abs(info["objective"] - infop["objective"]) <= 1e-8 * abs(infop["objective"])
    banner(f"refine_iters {info['refine_iters']} (plain face CG {infop['refine_iters']}), "
           f"stationarity {rep['stat_support']:.1e}")

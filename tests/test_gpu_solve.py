"""GPU NPGA solves (Algorithm 1 + refinement) against the exact FP64
minimiser of eq. mv computed by the oracle.

Bar (float32 storage): relative objective error <= 1e-6 (objective of
the GPU x re-evaluated in float64 by the oracle, and the GPU's own
reported objective), ||x - x*||_inf <= 1e-5, x >= 0 exactly,
|1^T x - 1| <= 1e-6, mu^T x >= r - 1e-6 max(1, |r|).

The GPU side builds L and mu from the float32 returns with
npga_build_factor; the oracle builds them in float64 from the same
float32 returns.  The two factors differ by float32 rounding of L
(relative 6e-8), far inside the bar.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import qp
from oracle.reference import exact_mv_factor, factor_objective
from tests.gpu_util import banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


def _check_parity(x, info, L, mu, r, gamma, ref, tag):
    x64 = x.astype(np.float64)
    f_gpu = factor_objective(L, gamma, x64)
    f_ref = ref["f"]
    assert x.min() >= 0.0, tag
    assert abs(x64.sum() - 1.0) <= 1e-6, tag
    assert mu @ x64 >= r - 1e-6 * max(1.0, abs(r)), tag
    assert abs(f_gpu - f_ref) <= 1e-6 * abs(f_ref), (tag, f_gpu, f_ref)
    assert abs(info["objective"] - f_ref) <= 1e-6 * abs(f_ref), (tag, info["objective"], f_ref)
    assert np.abs(x64 - ref["x"]).max() <= 1e-5, (tag, np.abs(x64 - ref["x"]).max())


def _case(spec, q=None, gamma=0.0):
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt) if q is None else None
    mu_ref, L_ref = ofactor.build_factor(Rt.T)
    if q is not None:
        r = float(np.quantile(Rt.astype(np.float64).mean(axis=0), q))
        if q == 1.0:  # stay clear of max(mu) by more than the summation-order rounding
            r -= 1e-9 * abs(r)
    ref = exact_mv_factor(L_ref, gamma, mu_ref, r)
    return Rt, r, mu_ref, L_ref, ref


@pytest.mark.parametrize("path", ["gemv", "syrk"])
def test_c1_parity(npga, path):
    spec = gen.SPECS["c1"]
    banner(f"c1 parity path={path}")
    Rt, r, mu_ref, L_ref, ref = _case(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, path=path)
    assert info["status"] == 0 and info["refined"] == 1, info
    _check_parity(x.cpu().numpy(), info, L_ref, mu_ref, r, 0.0, ref, f"c1-{path}")
    assert info["residual"] <= 1e-6


@pytest.mark.parametrize("n,T,q,gamma,path", [
    (5, 40, 0.5, 0.0, "gemv"),
    (63, 500, 0.9, 0.0, "gemv"),
    (130, 700, 0.2, 0.0, "syrk"),
    (257, 2000, 0.6, 0.0, "gemv"),
    (257, 2000, 0.6, 0.0, "syrk"),
    (300, 200, 0.6, 1e-4, "gemv"),   # T < n: ridge makes the model strongly convex
    (1000, 6000, 0.6, 0.0, "gemv"),
    (1000, 6000, 0.0, 0.0, "gemv"),  # return constraint slack
    (777, 3000, 1.0, 0.0, "gemv"),   # r = max mu: a single feasible vertex
])
def test_parity_shapes(npga, n, T, q, gamma, path):
    banner(f"parity n={n} T={T} q={q} gamma={gamma} path={path}")
    spec = spec_with("c2", n, T, seed=31 + n)
    Rt, r, mu_ref, L_ref, ref = _case(spec, q=q)
    if gamma:
        gamma = gamma * float(np.trace(L_ref @ L_ref.T)) / n
        ref = exact_mv_factor(L_ref, gamma, mu_ref, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, gamma=gamma, path=path)
    assert info["status"] == 0, info
    _check_parity(x.cpu().numpy(), info, L_ref, mu_ref, r, gamma, ref, f"{n}x{T}")


def test_certificate_and_multipliers(npga):
    spec = spec_with("c2", 400, 3000, seed=9)
    Rt, r, mu_ref, L_ref, ref = _case(spec, q=0.7)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, refine_tol=1e-11)
    H = 2 * (L_ref @ L_ref.T)
    xg = x.cpu().numpy().astype(np.float64)
    # x is float32: the return slack is known to float32 rounding only
    rep = qp.kkt_report(H, np.zeros(400), mu_ref, r, xg, act_tol=1e-6 * max(abs(r), np.abs(mu_ref).max()))
    assert rep["support"] == int((ref["x"] > 0).sum())
    assert rep["stat_support"] <= 1e-4 and rep["dual_offsupport"] >= -1e-4, rep
    assert info["return_active"] == (ref["nu"] > 0)
    assert abs(info["nu"] - ref["nu"]) <= 1e-3 * abs(ref["nu"]) + 1e-9
    assert abs(info["lambda"] - ref["lam"]) <= 1e-3 * abs(ref["lam"])


def test_deterministic(npga):
    spec = spec_with("c2", 500, 4000, seed=12)
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    L, mu = npga.build_factor(to_dev(Rt))
    xa, ia = npga.solve(L, mu, r)
    xb, ib = npga.solve(L, mu, r)
    assert torch.equal(xa, xb)
    assert ia["iters"] == ib["iters"] and ia["objective"] == ib["objective"]


def test_errors(npga):
    spec = gen.SPECS["c1"]
    Rt = gen.returns_TxN(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    with pytest.raises(npga.NpgaError) as e:
        npga.solve(L, mu, float(mu.max().item()) + 1e-3)
    assert e.value.code == 2
    mu_bad = mu.clone()
    mu_bad[3] = float("nan")
    with pytest.raises(npga.NpgaError) as e:
        npga.solve(L, mu_bad, 0.0)
    assert e.value.code == 5
    with pytest.raises(npga.NpgaError) as e:
        npga.solve(L, mu, 0.0, tol=-1.0)
    assert e.value.code == 1
    # max_iter reached: NOT_CONVERGED, and the returned x still lies in F
    r = gen.target_return(spec, Rt)
    x, info = npga.solve(L, mu, r, max_iter=2, tol=1e-14)
    assert info["status"] == 3
    xn = x.cpu().numpy().astype(np.float64)
    assert xn.min() >= 0 and abs(xn.sum() - 1) < 1e-6
    assert mu.cpu().numpy() @ xn >= r - 1e-6 * max(1, abs(r))


def test_warm_start_from_solution(npga):
    spec = spec_with("c2", 300, 2000, seed=14)
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r)
    x2, info2 = npga.solve(L, mu, r, x0=x)
    assert info2["iters"] <= 5
    assert torch.allclose(x, x2, atol=1e-6)


@pytest.mark.parametrize("n,T,want", [(300, 3000, 2), (500, 520, 2), (500, 480, 1)])
def test_auto_path_parity(npga, n, T, want):
    """NPGA_PATH_AUTO takes the covariance path at T >> n and T ~ n (T >= n)
    and the fused sweep at T < n; either way the result matches the oracle."""
    banner(f"auto path n={n} T={T}")
    spec = spec_with("c2", n, T, seed=41 + n)
    Rt, r, mu_ref, L_ref, ref = _case(spec, q=0.6)
    gamma = 0.0
    if T < n:
        gamma = 1e-4 * float(np.trace(L_ref @ L_ref.T)) / n
        ref = exact_mv_factor(L_ref, gamma, mu_ref, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, gamma=gamma)
    assert info["status"] == 0 and info["path_used"] == want, info
    _check_parity(x.cpu().numpy(), info, L_ref, mu_ref, r, gamma, ref, f"auto {n}x{T}")


@pytest.mark.parametrize("path", ["gemv", "syrk"])
@pytest.mark.parametrize("check_every", [1, 3, 7])
def test_check_every(npga, check_every, path):
    """The stopping test every check_every iterations (Algorithm 1's KKT check):
    the iteration count is a multiple of it, the last tail of each chunk of
    check_every launches reports the chunk's state to the host, and the
    refined solution is the oracle's."""
    spec = spec_with("c2", 300, 2500, seed=33)
    banner(f"check_every={check_every} {path}")
    Rt, r, mu_ref, L_ref, ref = _case(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, check_every=check_every, path=path)
    assert info["status"] == 0 and info["refined"] == 1, info
    assert info["iters"] % check_every == 0, info["iters"]
    assert info["residual"] <= 1e-6
    _check_parity(x.cpu().numpy(), info, L_ref, mu_ref, r, 0.0, ref, f"check_every={check_every}")


def test_batched_deterministic(npga):
    """Fixed launch shapes and fixed summation orders: two batched solves
    (main phase, float64 anchors of the refinement, face steps) give the
    same bits."""
    spec = spec_with("c4", 400, 3000, seed=34)
    Rt = gen.returns_TxN(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    mu_h = mu.cpu().numpy()
    rs = list(np.linspace(float(np.quantile(mu_h, 0.5)), 0.9 * float(mu_h.max()), 70))
    for path in ("gemv", "syrk"):
        Xa, ia = npga.solve_batched(L, mu, rs, path=path)
        Xb, ib = npga.solve_batched(L, mu, rs, path=path)
        assert torch.equal(Xa, Xb), path
        assert [i["objective"] for i in ia] == [i["objective"] for i in ib], path


@pytest.mark.parametrize("n,T,q,precond", [
    (2048, 6000, 0.6, True),
    (2048, 6000, 0.6, False),
    (2600, 7800, 0.3, True),
    (2600, 7800, 0.0, True),   # return constraint slack
    (2100, 4200, 1.0, True),   # r = max mu: a single feasible vertex
])
def test_refine_preconditioned(npga, n, T, q, precond):
    """Face solves of the active-set refinement with the Nystrom
    preconditioner (n >= 2048 on the factor path) and without it: the same
    parity bar against the oracle's minimiser, and bitwise-repeatable."""
    banner(f"preconditioned refinement n={n} T={T} q={q} precond={precond}")
    spec = spec_with("c2", n, T, seed=71 + n)
    Rt, r, mu_ref, L_ref, ref = _case(spec, q=q)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, path="gemv", refine_precond=precond)
    assert info["status"] == 0 and info["refined"] == 1, info
    _check_parity(x.cpu().numpy(), info, L_ref, mu_ref, r, 0.0, ref, f"pcg {n}x{T} q={q}")
    x2, info2 = npga.solve(L, mu, r, path="gemv", refine_precond=precond)
    assert torch.equal(x, x2) and info2["refine_iters"] == info["refine_iters"], (
        float((x - x2).abs().max()), info["refine_iters"], info2["refine_iters"], info["iters"], info2["iters"],
        info["objective"], info2["objective"])
    banner(f"refine_iters {info['refine_iters']}")


def test_solve_ignores_stale_workspace(npga):
    """A solve reads nothing of its workspace before writing it: the same
    solve on a zeroed workspace and on one holding finite junk (what earlier
    calls leave behind) is bitwise identical.  Regression: the padding of
    the float32 sweep input past n was left as found by the random start
    vector of the step estimate, and shifted the step size."""
    import ctypes
    from paper_2604_02917_amd import api
    spec = spec_with("c2", 2600, 7800, seed=71 + 2600)
    Rt, r, mu_ref, L_ref, ref = _case(spec, q=0.3)
    L, mu = npga.build_factor(to_dev(Rt))
    co = api.Options(path="gemv")._c()
    Lb, n, cols, ld = api._as_colmajor(L)
    need = api._lib.npga_solve_workspace_size(n, cols, ctypes.byref(co))
    mud = mu.to(torch.float64).contiguous()
    outs = []
    for fill in ("zero", "junk"):
        ws = torch.zeros(need // 8 + 1, dtype=torch.float64, device="cuda:0")
        if fill == "junk":
            ws.uniform_(-1e-3, 1e-3)
        x = torch.empty(n, dtype=torch.float32, device="cuda:0")
        res = api._Result()
        f = api._factor(Lb, n, cols, ld, mud, 0.0)
        code = api._lib.npga_solve(ctypes.byref(f), r, ctypes.byref(co), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.byref(res), ctypes.c_void_p(ws.data_ptr()), need, api._stream())
        torch.cuda.synchronize()
        assert code == 0
        outs.append((x, res.iters, res.refine_iters))
    assert torch.equal(outs[0][0], outs[1][0]), float((outs[0][0] - outs[1][0]).abs().max())
    assert outs[0][1:] == outs[1][1:], (outs[0][1:], outs[1][1:])
    _check_parity(outs[1][0].cpu().numpy(), {"objective": ref["f"]}, L_ref, mu_ref, r, 0.0, ref, "stale workspace")

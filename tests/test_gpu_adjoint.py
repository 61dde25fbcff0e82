"""Adjoint of the solution map on the GPU (npga_backward, NPGAFunction)
against the float64 oracle (oracle/adjoint.py: dense KKT solve on the
face), which is itself pinned by finite differences.

Workload C5: n = 200, T = 2000 (seed 5), r = 60th percentile of mu; the
loss is the out-of-sample objective l(w) = w^T Sigma_test w - mu_test^T w on
a held-out block (same B and drift, fresh factor and noise draws, seed 105,
5000 periods).  The GPU runs at the oracle's exact x* (float32), so the two
sides differentiate at the same point.

The n = 2048, T = 6000 case runs the face CG with the Nystrom
preconditioner (n >= 2048 with at least as many columns as assets).

Bar: the adjoint solve uses float32 products with one float64 correction
round, so dl/dmu and dl/dL agree with the oracle to 1e-4 of their largest
entry; dl/dr and dl/dgamma to 1e-4 relative."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle.adjoint import kkt_adjoint
from oracle.reference import exact_mv
from tests.gpu_util import banner, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


def _heldout_loss(spec):
    Rt = gen.heldout_returns_TxN(spec, 5000, gen.factor_model.HELDOUT_SEED_C5)
    mu_t, L_t = ofactor.build_factor(Rt.T)
    return (lambda w: 2.0 * (L_t @ (L_t.T @ w)) - mu_t), (lambda w: float((L_t.T @ w) @ (L_t.T @ w) - mu_t @ w))


def _case(n, T, seed, q, gamma):
    spec = spec_with("c5fd", n, T, seed=seed)
    Rt = gen.returns_TxN(spec)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu_o, q)) if q is not None else float(mu_o.min()) - 1e-3
    Q = L_o @ L_o.T + gamma * np.eye(n)
    s = exact_mv(Q, mu_o, r, fista_tol=1e-12)
    grad, _ = _heldout_loss(spec)
    return Rt, mu_o, L_o, r, s, grad


def _compare(npga, Rt, mu_o, L_o, r, s, grad, gamma, tag):
    L, mu = npga.build_factor(to_dev(Rt))
    xs = s["x"].astype(np.float32)
    g = grad(xs.astype(np.float64))
    dmu, dL, info = npga.backward(L, mu, r, to_dev(xs), to_dev(g.astype(np.float32)), gamma=gamma)
    ref = kkt_adjoint(L_o, gamma, mu_o, r, xs.astype(np.float64), s["lam"], s["nu"],
                      g.astype(np.float32).astype(np.float64))
    banner(f"{tag}: cg {info['cg_iters']} support {info['support']} active {info['return_active']} "
           f"residual {info['residual']:.1e}")
    assert info["status"] == 0 and info["degenerate"] == 0, info
    assert info["support"] == len(ref["support"]) and info["return_active"] == int(ref["active"])
    dmu_h = dmu.cpu().numpy()
    sc = np.abs(ref["dmu"]).max()
    assert np.abs(dmu_h - ref["dmu"]).max() <= 1e-4 * sc + 1e-12, (np.abs(dmu_h - ref["dmu"]).max(), sc)
    dL_h = dL.cpu().numpy().T.astype(np.float64)  # n x T
    scl = np.abs(ref["dL"]).max()
    assert np.abs(dL_h - ref["dL"]).max() <= 1e-4 * scl, (np.abs(dL_h - ref["dL"]).max(), scl)
    if ref["active"]:
        assert info["dl_dr"] == pytest.approx(ref["dr"], rel=1e-4)
    else:
        assert info["dl_dr"] == 0.0 and np.all(dmu_h == 0.0)
    assert info["dl_dgamma"] == pytest.approx(ref["dgamma"], rel=1e-4, abs=1e-12 * abs(ref["dgamma"]) + 1e-14)
    return info


@pytest.mark.parametrize("n,T,seed,q,gamma", [(200, 2000, 5, 0.6, 0.0), (200, 2000, 5, 0.9, 0.0),
                                              (131, 700, 7, 0.5, 1e-5), (150, 1200, 8, None, 0.0),
                                              (300, 400, 9, 0.7, 2e-5), (2048, 6000, 12, 0.6, 1e-5)])
def test_backward_vs_oracle(npga, n, T, seed, q, gamma):
    Rt, mu_o, L_o, r, s, grad = _case(n, T, seed, q, gamma)
    _compare(npga, Rt, mu_o, L_o, r, s, grad, gamma, f"adjoint n={n} T={T} q={q} gamma={gamma}")


def test_autograd_function(npga):
    """NPGAFunction: forward = npga_solve, backward = npga_backward; the
    gradients reach mu and L through torch.autograd."""
    n, T = 120, 900
    Rt, mu_o, L_o, r, s, grad = _case(n, T, 11, 0.6, 0.0)
    L, mu = npga.build_factor(to_dev(Rt))
    mu = mu.clone().requires_grad_(True)
    Lr = L.clone().requires_grad_(True)
    x = npga.NPGAFunction.apply(mu, Lr, r)
    spec = spec_with("c5fd", n, T, seed=11)
    Rtest = gen.heldout_returns_TxN(spec, 5000, gen.factor_model.HELDOUT_SEED_C5)
    mu_t, L_t = ofactor.build_factor(Rtest.T)
    Lt = to_dev(L_t.astype(np.float32))
    ut = Lt.T.float() @ x
    loss = (ut * ut).sum() - (to_dev(mu_t.astype(np.float32)) * x).sum()
    loss.backward()
    xg = x.detach().cpu().numpy().astype(np.float64)
    assert np.abs(xg - s["x"]).max() <= 1e-5
    g = grad(xg)
    ref = kkt_adjoint(L_o, 0.0, mu_o, r, s["x"], s["lam"], s["nu"], g)
    sc = np.abs(ref["dmu"]).max()
    # differentiated at the GPU's x (within 1e-5 of x*): a looser bar
    assert np.abs(mu.grad.cpu().numpy() - ref["dmu"]).max() <= 2e-3 * sc
    scl = np.abs(ref["dL"]).max()
    assert np.abs(Lr.grad.cpu().numpy().T - ref["dL"]).max() <= 2e-3 * scl

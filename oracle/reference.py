"""Exact reference minimisers for the mean-variance problem (eq. mv).

``exact_mv`` runs Algorithm 1 (oracle.npga) with the exact Lipschitz step
alpha = 1/L_f until the projected-gradient residual is small, then finishes
with the active-set method of oracle.qp, which certifies the KKT
conditions.  The result stands in for the exact solver x^G of Sec. 5.1.
"""
import numpy as np

from . import qp
from .npga import CovarianceModel, FactorModel, npga


def exact_mv(Q, mu, r, fista_tol=1e-9, max_iter=200000, x0=None):
    """x* = argmin_{x in F} x^T Q x for a dense PSD Q (float64).

    Returns dict(x, f, lam, nu, npga_iters).  f is x^T Q x accumulated from
    the given Q.
    """
    Q = np.asarray(Q, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    n = Q.shape[0]
    model = CovarianceModel(Q)
    alpha = 1.0 / model.lipschitz_exact()
    x0 = np.full(n, 1.0 / n) if x0 is None else x0
    out = npga(model, mu, r, alpha, x0, tol=fista_tol, check_every=5,
               max_iter=max_iter, restart=True)
    H = 2.0 * Q
    x, lam, nu, _ = qp.polish(H, np.zeros(n), mu, r, out["x"])
    return dict(x=x, f=float(x @ Q @ x), lam=lam, nu=nu, npga_iters=out["iters"])


def factor_objective(L, gamma, x):
    """f(x) = ||L^T x||^2 + gamma ||x||^2 accumulated in float64
    (eq. npga-unified-grad), without forming L L^T."""
    L = np.asarray(L, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    u = L.T @ x
    return float(u @ u + gamma * (x @ x))


def exact_mv_factor(L, gamma, mu, r, **kw):
    """exact_mv for Q = L L^T + gamma I; the objective is re-evaluated in
    factor form."""
    L = np.asarray(L, dtype=np.float64)
    Q = L @ L.T
    if gamma:
        Q = Q + gamma * np.eye(L.shape[0])
    out = exact_mv(Q, mu, r, **kw)
    out["f"] = factor_objective(L, gamma, out["x"])
    return out

"""Efficient frontier of eq. mv on one covariance: the exact minimiser for
each of m target returns (the batched workload of Sec. 5, where the paper
traces frontiers by re-solving for a grid of targets).

Test infrastructure only: imported by tests/, the golden-file script and
the benchmark's CPU baseline, never by the GPU path.

    min_variance(Q, mu)        -> x_mv, r_mv: the minimiser over the simplex
                                  with the return constraint dropped, and its
                                  return; every r <= r_mv has x*(r) = x_mv.
    frontier(L, gamma, mu, rs) -> exact x*(r_j), f*(r_j), nu*(r_j) for each
                                  target, by oracle.reference.exact_mv.

Parity pins (tests/test_oracle_frontier.py): f*(r) is nondecreasing and
convex on [r_mv, max mu]; nu*(r) = d f*/dr (envelope theorem of the
Lagrangian f - lam (1^T x - 1) - nu (mu^T x - r)), bracketed by the backward
and forward difference quotients; f*(r_mv) = f(x_mv); the two-asset
frontier in closed form.
"""
import numpy as np

from .reference import exact_mv, factor_objective


def min_variance(Q, mu, fista_tol=1e-10):
    """x_mv = argmin over the simplex of x^T Q x, and r_mv = mu^T x_mv."""
    mu = np.asarray(mu, dtype=np.float64)
    r_low = float(mu.min()) - 1.0          # never binds: mu^T x >= min mu on the simplex
    out = exact_mv(Q, mu, r_low, fista_tol=fista_tol)
    x = out["x"]
    return x, float(mu @ x)


def frontier(L, gamma, mu, targets, fista_tol=1e-10):
    """Exact solutions of eq. mv for Q = L L^T + gamma I at every target."""
    L = np.asarray(L, dtype=np.float64)
    Q = L @ L.T
    if gamma:
        Q = Q + gamma * np.eye(L.shape[0])
    out = []
    for r in targets:
        s = exact_mv(Q, mu, float(r), fista_tol=fista_tol)
        out.append(dict(r=float(r), x=s["x"], f=factor_objective(L, gamma, s["x"]), nu=s["nu"],
                        lam=s["lam"]))
    return out

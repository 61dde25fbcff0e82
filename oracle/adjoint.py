"""Gradients of a loss l(x*) through the solution map x*(mu, L, r, gamma)
of eq. mv, by implicit differentiation of the KKT system on the active face.

Test infrastructure only: imported by tests/ and never by the GPU path.

On the support S of x* with the return constraint active, x*_S and the
multipliers (lam, nu) of f = x^T Q x (Q = L L^T + gamma I) solve

    2 Q_SS x_S - lam 1 - nu mu_S = 0,   1^T x_S = 1,   mu_S^T x_S = r,

i.e. F(z; theta) = 0 with z = (x_S, lam, nu) and Jacobian
    K = [[2 Q_SS, -1, -mu_S], [1^T, 0, 0], [mu_S^T, 0, 0]].
With a = K^{-T} (dl/dx_S, 0, 0), dl/dtheta = -a^T dF/dtheta, which gives
    dl/dmu_S   = nu a_x - a_nu x_S,        dl/dmu_{S^c} = 0,
    dl/dr      = a_nu,
    dl/dgamma  = -2 a_x^T x_S,
    dl/dL      = -2 (a u^T + x v^T),  u = L^T x*, v = L^T a  (a embedded in R^n).
With the return constraint inactive the nu row and column are dropped
(dl/dmu = 0, dl/dr = 0).  The formula assumes strict complementarity (the
face does not change under a small perturbation); ``face_is_stable``
reports whether it holds.

Parity pins (tests/test_oracle_adjoint.py): central finite differences of
the exact solution map, the inactive case, and the two-asset closed form.
"""
import numpy as np


def face(L, gamma, mu, r, x, nu, tol=0.0):
    """Support S = {x_i > tol} and whether the return row is in the face
    (nu > 0 at the solution)."""
    S = np.flatnonzero(np.asarray(x) > tol)
    return S, bool(nu > 0.0)


def kkt_adjoint(L, gamma, mu, r, x, lam, nu, dl_dx):
    """Adjoint gradients at the exact solution x* with multipliers (lam, nu).

    Returns dict(dmu, dL, dr, dgamma, a (n,), a_lam, a_nu, support, active).
    """
    L = np.asarray(L, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(dl_dx, dtype=np.float64)
    n = L.shape[0]
    S, active = face(L, gamma, mu, r, x, nu)
    s = len(S)
    Q_SS = L[S] @ L[S].T + gamma * np.eye(s)
    k = s + (2 if active else 1)
    K = np.zeros((k, k))
    K[:s, :s] = 2.0 * Q_SS
    K[:s, s] = -1.0
    K[s, :s] = 1.0
    if active:
        K[:s, s + 1] = -mu[S]
        K[s + 1, :s] = mu[S]
    rhs = np.zeros(k)
    rhs[:s] = g[S]
    sol = np.linalg.solve(K.T, rhs)
    a = np.zeros(n)
    a[S] = sol[:s]
    a_lam = float(sol[s])
    a_nu = float(sol[s + 1]) if active else 0.0
    dmu = np.zeros(n)
    if active:
        dmu[S] = nu * a[S] - a_nu * x[S]
    u = L.T @ x
    v = L.T @ a
    dL = -2.0 * (np.outer(a, u) + np.outer(x, v))
    return dict(dmu=dmu, dL=dL, dr=a_nu, dgamma=-2.0 * float(a[S] @ x[S]), a=a, a_lam=a_lam, a_nu=a_nu,
                support=S, active=active)


def face_is_stable(Q, mu, x, lam, nu, rel=1e-8):
    """Strict complementarity: every zero x_i has a reduced cost
    2 (Q x)_i - lam - nu mu_i bounded away from zero, and x_i > 0 on S."""
    d = 2.0 * (Q @ x) - lam - nu * mu
    scale = np.abs(2.0 * (Q @ x)).max()
    off = np.asarray(x) <= 0.0
    return bool(np.all(d[off] > rel * scale))

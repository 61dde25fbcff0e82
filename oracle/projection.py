"""Euclidean projections onto the simplex and onto F (paper Sec. 3.1).

F = Delta  intersect  H,  Delta = {x >= 0, 1^T x = 1},  H = {mu^T x >= r}.

* Simplex: find tau with sum_i max(v_i - tau, 0) = 1 (eq. simplex-tau) and
  set x_i = max(v_i - tau, 0) (eq. simplex-proj); tau from the sorted
  values by the largest j with v_(j) - (sum_{i<=j} v_(i) - 1)/j > 0.
* F: if mu^T Pi_Delta(v) >= r the simplex projection is already Pi_F(v).
  Otherwise the return constraint is active and Pi_F(v) = Pi_Delta(v + nu mu)
  for the nu >= 0 with phi(nu) = mu^T Pi_Delta(v + nu mu) = r
  (eq. projF-dualpath); phi is continuous and nondecreasing, so nu is
  bracketed by doubling nu = 1, 2, 4, ... and then bisected.

The paper stops the bisection at |phi(nu) - r| <= tau_proj max{1, |r|}.  This
oracle instead finishes exactly: once the two bracket ends share a support
S, phi is affine on the bracket (on S, tau(nu) = (sum_S v + nu sum_S mu -
1)/|S|), so the root is solved in closed form and then verified with the
sort formula.  The returned point is exact up to float64 rounding.
"""
import numpy as np


def simplex_threshold_sort(v):
    """tau of eq. simplex-tau via the sorting rule of Sec. 3.1."""
    v = np.asarray(v, dtype=np.float64)
    u = np.sort(v)[::-1]
    css = np.cumsum(u) - 1.0
    j = np.arange(1, v.size + 1, dtype=np.float64)
    cond = u - css / j > 0
    k = np.nonzero(cond)[0][-1]
    return css[k] / (k + 1.0)


def proj_simplex(v):
    """Pi_Delta(v) by eq. simplex-proj."""
    v = np.asarray(v, dtype=np.float64)
    return np.maximum(v - simplex_threshold_sort(v), 0.0)


def simplex_threshold_bisect(v, iters=200):
    """Independent tau: bisection on the decreasing map
    h(tau) = sum max(v - tau, 0) - 1 over [min v - 1, max v]."""
    v = np.asarray(v, dtype=np.float64)
    lo, hi = v.min() - 1.0, v.max()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.maximum(v - mid, 0.0).sum() - 1.0 > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _phi(v, mu, nu):
    x = proj_simplex(v + nu * mu)
    return float(mu @ x), x


def proj_F(v, mu, r, max_double=2000, max_bisect=400):
    """Pi_F(v) by the scalar dual search of Sec. 3.1.

    Returns (x, nu, tau).  Raises ValueError when F is empty (r > max mu).
    """
    v = np.asarray(v, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    if r > mu.max():
        raise ValueError("F is empty: r > max(mu)")
    tau0 = simplex_threshold_sort(v)
    x0 = np.maximum(v - tau0, 0.0)
    if mu @ x0 >= r:
        return x0, 0.0, tau0
    # bracket: phi(lo) < r <= phi(hi)
    lo, hi = 0.0, 1.0
    for _ in range(max_double):
        if _phi(v, mu, hi)[0] >= r:
            break
        lo, hi = hi, 2.0 * hi
    else:
        raise RuntimeError("bracketing failed")
    for _ in range(max_bisect):
        xlo = proj_simplex(v + lo * mu)
        xhi = proj_simplex(v + hi * mu)
        Slo, Shi = xlo > 0, xhi > 0
        if np.array_equal(Slo, Shi):
            S = Shi
            c = S.sum()
            sv, sm = v[S].sum(), mu[S].sum()
            smm, smv = (mu[S] ** 2).sum(), (mu[S] * v[S]).sum()
            slope = smm - sm * sm / c
            if slope > 0:
                # phi(nu) = smv + nu*smm - tau(nu)*sm, tau(nu) = (sv + nu*sm - 1)/c
                nu = (r - smv + sm * (sv - 1.0) / c) / slope
                if lo <= nu <= hi:
                    tau = (sv + nu * sm - 1.0) / c
                    x = np.maximum(v + nu * mu - tau, 0.0)
                    # verify with the sort formula
                    xs = proj_simplex(v + nu * mu)
                    if np.array_equal(xs > 0, S) and abs(mu @ xs - r) <= 1e-11 * np.abs(mu).max():
                        return xs, nu, simplex_threshold_sort(v + nu * mu)
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if _phi(v, mu, mid)[0] < r:
            lo = mid
        else:
            hi = mid
    x = proj_simplex(v + hi * mu)
    return x, hi, simplex_threshold_sort(v + hi * mu)


def proj_halfspace(z, mu, r):
    """Pi_H(z) for H = {x : mu^T x >= r}: z + max(0, r - mu^T z)/||mu||^2 mu."""
    z = np.asarray(z, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    s = float(mu @ z)
    if s >= r:
        return z.copy()
    return z + ((r - s) / float(mu @ mu)) * mu


def dykstra(v, mu, r, max_iter=100000, tol=1e-12):
    """Pi_F(v) by Dykstra's alternating projections onto the simplex Delta
    and the half-space H = {mu^T x >= r}, the safeguarded fallback of Sec. 3.1
    (Bauschke and Borwein, 1996).  With x_0 = v and p_0 = q_0 = 0:
        y_k = Pi_Delta(x_k + p_k),   p_{k+1} = x_k + p_k - y_k,
        x_{k+1} = Pi_H(y_k + q_k),   q_{k+1} = y_k + q_k - x_{k+1};
    both sequences converge to Pi_{Delta cap H}(v).  Stops when
    ||x_{k+1} - y_k||_2 and ||y_k - y_{k-1}||_2 are both <= tol.
    Returns (y, iterations); y lies in Delta exactly."""
    v = np.asarray(v, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    x = v.copy()
    p = np.zeros_like(v)
    q = np.zeros_like(v)
    y = np.zeros_like(v)
    for k in range(1, max_iter + 1):
        y_new = proj_simplex(x + p)
        p = x + p - y_new
        x_new = proj_halfspace(y_new + q, mu, r)
        q = y_new + q - x_new
        dy = float(np.linalg.norm(y_new - y))
        dx = float(np.linalg.norm(x_new - y_new))
        x, y = x_new, y_new
        if k > 1 and dx <= tol and dy <= tol:
            return y, k
    return y, max_iter

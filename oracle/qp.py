"""Exact solution of the constrained QP (paper eq. mv) and its KKT checks.

    minimise 1/2 x^T H x + c^T x  over  F = {x >= 0, 1^T x = 1, mu^T x >= r}.

The mean-variance problem is H = 2 Sigma, c = 0 (eq. mv, objective x^T Sigma
x with no 1/2).  The projection Pi_F(v) is H = I, c = -v.

Optimality (Sec. 3.1, "Stopping condition": x* is optimal iff
0 in grad f(x*) + N_F(x*)) is written out as the KKT system
    H x + c = lam 1 + nu mu + s,  s >= 0,  s_i x_i = 0,
    nu >= 0,  nu (mu^T x - r) = 0,  x in F.
On a fixed face (free set S, return constraint active or not) this is the
linear system
    [H_SS  -1  -mu_S] [x_S]   [-c_S]
    [1^T    0    0  ] [lam] = [  1 ]
    [mu_S^T 0    0  ] [nu ]   [  r ]      (last row/column only if active).

``brute_force`` enumerates every face (tiny n); ``active_set`` is the
textbook primal active-set method for convex QP (Nocedal and Wright,
Numerical Optimization, Alg. 16.3) started from a feasible point.
"""
import itertools

import numpy as np


def face_solve(H, c, mu, r, free, active):
    """Solve the KKT equalities on a face.  Returns (x, lam, nu) or None if
    the face system is singular."""
    n = H.shape[0]
    idx = np.nonzero(free)[0]
    k = idx.size
    m = 2 if active else 1
    K = np.zeros((k + m, k + m))
    K[:k, :k] = H[np.ix_(idx, idx)]
    K[:k, k] = -1.0
    K[k, :k] = 1.0
    rhs = np.zeros(k + m)
    rhs[:k] = -c[idx]
    rhs[k] = 1.0
    if active:
        K[:k, k + 1] = -mu[idx]
        K[k + 1, :k] = mu[idx]
        rhs[k + 1] = r
    try:
        sol = np.linalg.solve(K, rhs)
        if np.all(np.isfinite(sol)):
            # one step of iterative refinement (ill-conditioned faces, e.g. a
            # rank-ell covariance plus a small ridge)
            sol = sol + np.linalg.solve(K, rhs - K @ sol)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(sol)):
        return None
    # reject numerically singular faces: the solution must satisfy the
    # constraints and the stationarity rows to a tolerance set by the data
    xs = sol[:k]
    if abs(xs.sum() - 1.0) > 1e-9:
        return None
    mscale = max(np.abs(mu[idx]).max(), 1e-300)
    if active and abs(mu[idx] @ xs - r) > 1e-9 * mscale:
        return None
    if np.linalg.cond(K) > 1e14:
        return None
    x = np.zeros(n)
    x[idx] = sol[:k]
    lam = sol[k]
    nu = sol[k + 1] if active else 0.0
    return x, lam, nu


def multipliers(H, c, mu, r, x, act_tol=None):
    """Least-squares (lam, nu) on the support of x; nu = 0 when the return
    constraint is slack."""
    g = H @ x + c
    S = x > 0
    if act_tol is None:
        act_tol = 1e-12 * max(abs(r), np.abs(mu).max())
    if mu @ x - r > act_tol:
        lam = g[S].mean() if S.any() else 0.0
        return float(lam), 0.0
    if S.sum() == 1:
        # vertex e_s on the return face: (lam, nu) are not unique; take the
        # smallest nu >= 0 that keeps every reduced cost g_j - lam - nu mu_j >= 0
        s = int(np.nonzero(S)[0][0])
        dm = mu - mu[s]
        dg = g - g[s]
        lo = 0.0
        neg = (~S) & (dm < 0)
        if neg.any():
            lo = max(lo, float(np.max(dg[neg] / dm[neg])))
        nu = lo
        return float(g[s] - nu * mu[s]), float(nu)
    A = np.stack([np.ones(S.sum()), mu[S]], axis=1)
    sol, *_ = np.linalg.lstsq(A, g[S], rcond=None)
    return float(sol[0]), float(sol[1])


def kkt_report(H, c, mu, r, x, lam=None, nu=None, act_tol=None):
    """Residuals of every KKT condition at x (all as plain floats).

    ``act_tol`` is the slack below which the return constraint counts as
    active when the multipliers are estimated (default: float64 rounding)."""
    x = np.asarray(x, dtype=np.float64)
    if lam is None:
        lam, nu = multipliers(H, c, mu, r, x, act_tol=act_tol)
    g = H @ x + c
    d = g - lam - nu * mu
    S = x > 0
    scale = max(np.abs(g).max(), 1e-300)
    return dict(
        min_x=float(x.min()),
        budget=float(abs(x.sum() - 1.0)),
        ret_slack=float(mu @ x - r),
        nu=float(nu),
        lam=float(lam),
        compl=float(abs(nu * (mu @ x - r))),
        stat_support=float(np.abs(d[S]).max() / scale) if S.any() else 0.0,
        dual_offsupport=float(min(d[~S].min(), 0.0) / scale) if (~S).any() else 0.0,
        support=int(S.sum()),
    )


def certificate_ok(rep, tol_stat=1e-10, tol_feas=1e-12, r_scale=1.0):
    """True when a kkt_report certifies optimality at the given tolerances."""
    return (rep["min_x"] >= 0.0
            and rep["budget"] <= tol_feas
            and rep["ret_slack"] >= -tol_feas * r_scale
            and rep["nu"] >= -tol_stat
            and rep["stat_support"] <= tol_stat
            and rep["dual_offsupport"] >= -tol_stat)


def brute_force(H, c, mu, r, tol=1e-10):
    """Enumerate all faces (n <= ~14).  Returns the list of KKT points
    (x, lam, nu) found; for H positive definite on F there is one x."""
    H = np.asarray(H, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    n = H.shape[0]
    found = []
    scale = max(np.abs(H).max(), np.abs(c).max(), 1e-300)
    for k in range(1, n + 1):
        for comb in itertools.combinations(range(n), k):
            free = np.zeros(n, bool)
            free[list(comb)] = True
            for active in (False, True):
                out = face_solve(H, c, mu, r, free, active)
                if out is None:
                    continue
                x, lam, nu = out
                if x[free].min() < -tol:
                    continue
                if not active and mu @ x < r - tol * max(1.0, abs(r)):
                    continue
                if active and nu < -tol * scale:
                    continue
                d = H @ x + c - lam - nu * mu
                if (~free).any() and d[~free].min() < -tol * scale:
                    continue
                found.append((np.maximum(x, 0.0), lam, nu))
    return found


def active_set(H, c, mu, r, x0, max_iter=10000, tol=1e-13):
    """Primal active-set method (Nocedal and Wright, Alg. 16.3) for the QP
    above, from a feasible x0.  The working set holds bounds x_i = 0 and,
    possibly, the return constraint.  Returns (x, lam, nu, iterations)."""
    H = np.asarray(H, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    x = np.asarray(x0, dtype=np.float64).copy()
    n = x.size
    Z = x <= 0.0                     # bounds in the working set
    x[Z] = 0.0
    mscale = np.abs(mu).max()
    ret_in = (mu @ x - r) <= 1e-14 * max(abs(r), mscale)
    gscale = max(np.abs(H).max(), np.abs(c).max(), 1e-300)
    seen = set()
    for it in range(max_iter):
        state = (Z.tobytes(), bool(ret_in))
        out = face_solve(H, c, mu, r, ~Z, ret_in)
        if out is None and ret_in and (~Z).sum() <= 1:
            # a vertex e_i with mu_i = r: the budget row alone fixes the
            # point, so the return row is redundant in the working set
            ret_in = False
            out = face_solve(H, c, mu, r, ~Z, ret_in)
        if out is None:
            raise np.linalg.LinAlgError("singular face system")
        xh, lam, nu = out
        p = xh - x
        if np.abs(p).max() <= 1e-12 * max(1.0, np.abs(x).max()):
            d = H @ x + c - lam - nu * mu
            s = np.where(Z, d, 0.0)
            cand_i = int(np.argmin(s)) if Z.any() else -1
            worst_s = s[cand_i] if cand_i >= 0 else 0.0
            worst_nu = nu if ret_in else 0.0
            if worst_s >= -tol * gscale and worst_nu >= -tol * gscale:
                # free entries equal to zero up to rounding are clamped
                return np.maximum(xh, 0.0), lam, nu, it
            if state in seen:
                raise RuntimeError("active set cycled")
            seen.add(state)
            # drop the most violated constraint (scale nu by |mu|)
            if worst_s <= worst_nu * mscale:
                Z[cand_i] = False
            else:
                ret_in = False
            x = xh
            continue
        # step towards xh, stopping at the first blocking constraint
        alpha, block = 1.0, None
        neg = (~Z) & (p < 0)
        if neg.any():
            ratios = x[neg] / (-p[neg])
            j = int(np.argmin(ratios))
            if ratios[j] < alpha:
                alpha, block = ratios[j], ("x", np.nonzero(neg)[0][j])
        mp = mu @ p
        if not ret_in and mp < 0:
            rr = (mu @ x - r) / (-mp)
            if rr < alpha:
                alpha, block = rr, ("ret", None)
        x = x + alpha * p
        if block is not None:
            if block[0] == "x":
                Z[block[1]] = True
                x[block[1]] = 0.0
            else:
                ret_in = True
        x[Z] = 0.0
    raise RuntimeError("active set did not terminate")


def polish(H, c, mu, r, x_approx, theta_rel=1e-7):
    """Exact minimiser from an approximate feasible x: guess the face by
    thresholding, take its KKT point if it is feasible, then finish with
    the active-set method (which certifies optimality on exit)."""
    x_approx = np.asarray(x_approx, dtype=np.float64)
    theta = theta_rel * x_approx.max()
    free = x_approx > theta
    mscale = np.abs(mu).max()
    lam0, nu0 = multipliers(H, c, mu, r, np.where(free, x_approx, 0.0))
    active = (mu @ x_approx - r) <= 1e-6 * max(abs(r), mscale)
    start = x_approx
    out = face_solve(H, c, mu, r, free, active)
    if out is not None:
        xf = out[0]
        if xf.min() >= 0.0 and mu @ xf >= r - 1e-14 * max(abs(r), mscale):
            start = np.maximum(xf, 0.0)
    return active_set(H, c, mu, r, start)


def gap(f_hat, f_ref):
    """Relative objective gap of Sec. 5.1:
    max{f(x_hat) - f(x_ref), 0} / max{|f(x_ref)|, 1e-12}."""
    return max(f_hat - f_ref, 0.0) / max(abs(f_ref), 1e-12)

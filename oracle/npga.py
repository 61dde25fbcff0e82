"""Algorithm 1 (NPGA) and the power-method step size (paper Sec. 3.1).

Unified model (eq. npga-unified-grad):
    f(x) = ||L_eff^T x||^2 + gamma ||x||^2,
    grad f(x) = 2 L_eff (L_eff^T x) + 2 gamma x.
Explicit-covariance form (Sec. 3.1): grad f(x) = 2 Sigma x.

Algorithm 1: y^0 = x^0, t_0 = 1; repeat
    v^k = y^k - alpha grad f(y^k);  x^{k+1} = Pi_F(v^k);
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2;  beta_k = (t_k - 1) / t_{k+1};
    y^{k+1} = x^{k+1} + beta_k (x^{k+1} - x^k).
Stop when ||Pi_F(x^k - alpha grad f(x^k)) - x^k||_2 <= eps (Sec. 3.1
"Stopping condition"), checked every ``check_every`` iterations as in the
benchmarks of Sec. 5.1.  Fixed step 0 < alpha <= 1/L_f with
L_f = 2 ||L_eff||_2^2 + 2 gamma (Sec. 3.1 "Fixed step").

Pins: the limit (the exact QP minimiser, pinned in ``qp``), the rates, and
the trajectory itself against a scalar FISTA on the two-asset segment, where
the projection is a clamp (tests/test_oracle_factor_npga.py).
"""
import numpy as np

from .projection import proj_F


class FactorModel:
    """f(x) = ||L^T x||^2 + gamma ||x||^2 given the n x m factor L."""

    def __init__(self, L, gamma=0.0):
        self.L = np.asarray(L, dtype=np.float64)
        self.gamma = float(gamma)

    def value(self, x):
        u = self.L.T @ x
        return float(u @ u + self.gamma * (x @ x))

    def grad(self, x):
        return 2.0 * (self.L @ (self.L.T @ x)) + 2.0 * self.gamma * x

    def curv(self, d):
        """d^T Q d = ||L^T d||^2 + gamma ||d||^2: for this quadratic f,
        f(x) - f(y) - <grad f(y), x - y> equals curv(x - y) exactly."""
        u = self.L.T @ d
        return float(u @ u + self.gamma * (d @ d))

    def lipschitz_exact(self):
        """L_f = 2 ||L||_2^2 + 2 gamma."""
        s = np.linalg.norm(self.L, 2)
        return 2.0 * s * s + 2.0 * self.gamma


class CovarianceModel:
    """f(x) = x^T Sigma x (explicit covariance, Sec. 3.1)."""

    def __init__(self, Sigma):
        self.S = np.asarray(Sigma, dtype=np.float64)

    def value(self, x):
        return float(x @ (self.S @ x))

    def grad(self, x):
        return 2.0 * (self.S @ x)

    def curv(self, d):
        """d^T Sigma d (= f(x) - f(y) - <grad f(y), x - y> with d = x - y)."""
        return float(d @ (self.S @ d))

    def lipschitz_exact(self):
        return 2.0 * float(np.linalg.eigvalsh(self.S)[-1])


def power_method(L, iters, u0):
    """Remark "Power method": u <- L(L^T u)/||L(L^T u)||, u^0 = r/||r||.

    Returns the Rayleigh values ||L^T u^t||_2 for t = 0..iters (each is a
    lower bound on ||L||_2 that rises towards it) and the final vector.
    """
    L = np.asarray(L, dtype=np.float64)
    u = np.asarray(u0, dtype=np.float64)
    u = u / np.linalg.norm(u)
    ray = [float(np.linalg.norm(L.T @ u))]
    for _ in range(iters):
        w = L @ (L.T @ u)
        u = w / np.linalg.norm(w)
        ray.append(float(np.linalg.norm(L.T @ u)))
    return np.array(ray), u


def constant_momentum(alpha, m_f):
    """beta = (1 - sqrt(alpha m_f)) / (1 + sqrt(alpha m_f)): the constant
    momentum of the strongly convex specialization (Sec. 3.1; Thm. npga-
    convergence (b)), with m_f a lower curvature bound (m_f >= 2 gamma)."""
    q = np.sqrt(alpha * m_f)
    return float((1.0 - q) / (1.0 + q))


def npga(model, mu, r, alpha, x0, tol=1e-6, check_every=5, max_iter=100000,
         restart=False, record=False, beta_const=None, backtrack=None):
    """Algorithm 1 with the fixed step ``alpha``.

    ``x0`` is projected onto F first (Algorithm 1 requires x^0 in F).
    Returns dict(x, iters, residual, converged, trace).  ``iters`` counts
    gradient evaluations at y^k.  The residual is checked at k = 0, c, 2c...
    before the k-th step, using grad f(x^k).  ``restart`` applies the
    gradient-based adaptive restart of O'Donoghue and Candes (resets t to 1
    when (y^k - x^{k+1})^T (x^{k+1} - x^k) > 0); it is off by default.
    ``beta_const`` replaces the t_k sequence by a constant momentum (used
    from the second step on; the first step has beta = 0).
    ``backtrack = rho`` (0 < rho < 1) turns on the adaptive backtracking of
    Sec. 3.1: starting from the previous accepted step (``alpha`` at k = 0),
    the trial step is multiplied by rho until the point
    x^{k+1} = Pi_F(y^k - alpha_k grad f(y^k)) satisfies
    f(x^{k+1}) <= f(y^k) + <grad f(y^k), x^{k+1} - y^k>
                 + ||x^{k+1} - y^k||^2 / (2 alpha_k).
    The steps are then nonincreasing; the returned dict adds ``alpha`` (the
    last accepted step) and ``rejections`` (trial steps refused).  f is
    quadratic, so the test is evaluated in its exact rearranged form
    curv(d) <= ||d||^2 / (2 alpha_k), d = x^{k+1} - y^k (curv(d) = d^T Q d is
    f(x^{k+1}) - f(y^k) - <grad f(y^k), d>), which avoids the cancellation
    of the direct form once the steps are small.
    """
    mu = np.asarray(mu, dtype=np.float64)
    x, _, _ = proj_F(np.asarray(x0, dtype=np.float64), mu, r)
    x_prev = x.copy()
    t, beta = 1.0, 0.0
    trace = []
    res = np.inf
    k = 0
    rejections = 0
    while True:
        if k % check_every == 0:
            gx = model.grad(x)
            p, _, _ = proj_F(x - alpha * gx, mu, r)
            res = float(np.linalg.norm(p - x))
            if record:
                trace.append((k, res))
            if res <= tol:
                return dict(x=x, iters=k, residual=res, converged=True, trace=trace, alpha=alpha,
                            rejections=rejections)
        if k >= max_iter:
            return dict(x=x, iters=k, residual=res, converged=False, trace=trace, alpha=alpha,
                        rejections=rejections)
        y = x + beta * (x - x_prev)
        gy = model.grad(y)
        v = y - alpha * gy
        x_new, _, _ = proj_F(v, mu, r)
        if backtrack is not None:
            while True:
                d = x_new - y
                if model.curv(d) <= (d @ d) / (2.0 * alpha):
                    break
                alpha *= backtrack
                rejections += 1
                x_new, _, _ = proj_F(y - alpha * gy, mu, r)
        if restart and (y - x_new) @ (x_new - x) > 0:
            t = 1.0
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        beta = (t - 1.0) / t_new if beta_const is None else beta_const
        t = t_new
        x_prev, x = x, x_new
        k += 1

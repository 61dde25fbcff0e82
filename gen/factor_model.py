"""Seeded factor-model return panels shaped like the paper's workloads.

The paper's real panel (5-minute A-share returns, n=5440 assets, T=48374
training periods; Sec. 5.1) is proprietary, and its synthetic generator is
only described as "geometrically decaying singular values" (Sec. 5.1).  The
stand-in used everywhere here is a K-factor model with heavy-tailed
idiosyncratic noise and a per-asset drift:

    R[:, t] = B f_t + c_t * e_t + d,   f_t ~ N(0, 0.01^2 I_K),
    e_t[i] ~ Student-t(4) iid,         d_i ~ N(drift_mean, drift_sd^2),
    B[i, k] ~ N(0, 1).

Draw order (numpy ``default_rng(seed)``, PCG64): B (n x K, row-major), then
d (n), then F as a (T x K) array, then E as a (T x n) array consumed in
period order.  Chunked draws consume the stream exactly as one large draw,
so the panel is bit-identical however it is chunked.

Layout: the panel is returned as a C-contiguous (T, n) float32 array, i.e.
period t's n-vector is contiguous.  Read as an n x T matrix this is the
column-major layout (leading dimension n) that the HIP library expects.
The float32 values are the workload: both sides treat them as exact.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class FactorModelSpec:
    name: str
    n: int
    T: int
    K: int
    t_scale: float
    drift_mean: float
    drift_sd: float
    seed: int
    target_rule: str  # "median" or "pct60"

    def scaled(self, n: int, T: int, name: str | None = None) -> "FactorModelSpec":
        return dataclasses.replace(self, n=n, T=T, name=name or f"{self.name}-{n}x{T}")


# The five workloads.  Distribution parameters follow the stated recipes;
# "N(m, s)" for the drift is read as (mean, standard deviation) and
# "Student-t(4) scaled c" as c * t_4.
SPECS = {
    # Plain NPGA parity case: n=64, T=256, 3 factors.
    "c1": FactorModelSpec("c1", 64, 256, 3, 0.02, 5e-4, 2e-4, 1, "median"),
    # Unreduced full model at the paper's headline shape.
    "c2": FactorModelSpec("c2", 5440, 48374, 10, 0.015, 4e-4, 3e-4, 2, "pct60"),
    # Batched frontier: n=2000, T=20000, 5 factors, c2 distributions.
    "c4": FactorModelSpec("c4", 2000, 20000, 5, 0.015, 4e-4, 3e-4, 4, "pct60"),
    # Adjoint finite-difference case: n=200, T=2000.
    "c5fd": FactorModelSpec("c5fd", 200, 2000, 10, 0.015, 4e-4, 3e-4, 5, "pct60"),
}

SKETCH_SEED_C3 = 3
HELDOUT_SEED_C5 = 105


def returns_TxN(spec: FactorModelSpec, chunk: int = 4096) -> np.ndarray:
    """Return the (T, n) float32 panel for ``spec`` (see module docstring)."""
    rng = np.random.default_rng(spec.seed)
    n, T, K = spec.n, spec.T, spec.K
    B = rng.standard_normal((n, K))
    d = rng.normal(spec.drift_mean, spec.drift_sd, n)
    F = rng.normal(0.0, 0.01, (T, K))
    out = np.empty((T, n), dtype=np.float32)
    for t0 in range(0, T, chunk):
        t1 = min(T, t0 + chunk)
        E = rng.standard_t(4.0, (t1 - t0, n))
        blk = F[t0:t1] @ B.T
        blk += spec.t_scale * E
        blk += d[None, :]
        out[t0:t1] = blk
    return out


def heldout_returns_TxN(spec: FactorModelSpec, T_test: int, seed: int) -> np.ndarray:
    """A held-out (T_test, n) float32 block: same B and drift as ``spec``,
    fresh factor and idiosyncratic draws from ``seed``."""
    rng = np.random.default_rng(spec.seed)
    n, K = spec.n, spec.K
    B = rng.standard_normal((n, K))
    d = rng.normal(spec.drift_mean, spec.drift_sd, n)
    rng2 = np.random.default_rng(seed)
    F = rng2.normal(0.0, 0.01, (T_test, K))
    E = rng2.standard_t(4.0, (T_test, n))
    return (F @ B.T + spec.t_scale * E + d[None, :]).astype(np.float32)


def target_return(spec: FactorModelSpec, R_TxN: np.ndarray) -> float:
    """Target return r from the per-asset sample means of the float32 panel.

    "median" -> numpy.median; "pct60" -> numpy.percentile(., 60) (linear).
    The row means are summed in float64 over the float32 values.
    """
    m = np.asarray(R_TxN, dtype=np.float64).mean(axis=0)
    if spec.target_rule == "median":
        return float(np.median(m))
    if spec.target_rule == "pct60":
        return float(np.percentile(m, 60))
    raise ValueError(spec.target_rule)


def frontier_targets_from_mv(r_mv: float, mu_max: float, m: int = 128) -> np.ndarray:
    """m targets evenly spaced from the min-variance return to 0.95 * max mu."""
    return np.linspace(r_mv, 0.95 * mu_max, m)


def gaussian_sketch(T: int, k: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Dense sketch S (T x k), entries N(0, 1/k), returned C-contiguous as a
    (k, T) array: row j is sketch column j, i.e. S is column-major T x k."""
    rng = np.random.default_rng(seed)
    out = np.empty((k, T), dtype=dtype)
    sd = 1.0 / np.sqrt(k)
    for j0 in range(0, k, 256):
        j1 = min(k, j0 + 256)
        out[j0:j1] = rng.normal(0.0, sd, (j1 - j0, T))
    return out


def countsketch(T: int, k: int, seed: int):
    """CountSketch draws (Sec. 2.3): bucket h(t) uniform on [0, k) and sign
    s(t) = +-1 for each period t.  Returns (h int32 (T,), s float32 (T,))."""
    rng = np.random.default_rng(seed)
    h = rng.integers(0, k, T).astype(np.int32)
    s = (2 * rng.integers(0, 2, T) - 1).astype(np.float32)
    return h, s


def random_vector(n: int, seed: int, kind: str = "normal", scale: float = 1.0) -> np.ndarray:
    """Random float64 test vectors (projection inputs, warm starts)."""
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return scale * rng.standard_normal(n)
    if kind == "uniform":
        return scale * rng.random(n)
    if kind == "ties":  # many exactly repeated values
        return scale * rng.integers(-3, 4, n).astype(np.float64) / 4.0
    raise ValueError(kind)

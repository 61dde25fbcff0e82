"""Sample mean and centered covariance factor (paper Sec. 2.1 and Sec. 1).

mu = (1/T) R 1_T,   L = (R - mu 1_T^T) / sqrt(T - 1),   Sigma = L L^T
(the unbiased sample covariance).
"""
import numpy as np


def build_factor(R_nxT):
    """Return (mu, L) in float64 for an n x T return panel (Sec. 2.1)."""
    R = np.asarray(R_nxT, dtype=np.float64)
    T = R.shape[1]
    if T < 2:
        raise ValueError("need T >= 2 periods")
    mu = R.sum(axis=1) / T
    L = (R - mu[:, None]) / np.sqrt(T - 1.0)
    return mu, L


def covariance(L):
    """Sigma = L L^T (Sec. 2.1)."""
    L = np.asarray(L, dtype=np.float64)
    return L @ L.T

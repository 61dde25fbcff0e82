"""Sketch, truncation and ridge (paper Sec. 2.3-2.6 and App. D).

* Sketch stage (Sec. 2.5): L_tilde = L Phi with Phi T x s, Gaussian JL
  entries N(0, 1/s) (Sec. 2.3); Sigma_tilde = L_tilde L_tilde^T.
* Truncation stage (Sec. 2.5): thin SVD L_tilde = U S V^T, keep the
  leading ell triplets.
* Ridge stage (Sec. 2.5): Sigma_hat = L_ell L_ell^T + gamma I, whose
  spectrum is {sigma_i^2 + gamma} (i <= ell) and gamma (n - ell times).
* App. D "Relation between STR and sketching": (L Phi V_ell)(L Phi V_ell)^T
  = U_ell S_ell^2 U_ell^T, so the n x ell factor L_eff = U_ell S_ell
  = L_tilde V_ell defines the same Sigma_hat as the n x s form.
* Ridge rule of the STR workload: gamma = c * trace(L_tilde L_tilde^T) / n
  with the untruncated sketch (c = 1e-4).  The paper's own rule,
  gamma = sigma_1^2 / (kappa_tar - 1) (App. D), is ``gamma_kappa_target``.
* CountSketch (Sec. 2.3): one +-1 per row of Phi at a hashed column.
"""
import numpy as np


def sketch(L, Phi):
    """L_tilde = L Phi (Sec. 2.5, sketch stage)."""
    return np.asarray(L, dtype=np.float64) @ np.asarray(Phi, dtype=np.float64)


def countsketch_apply(L, h, sgn, s):
    """L Phi for the CountSketch Phi(i, h(i)) = sgn_i (Sec. 2.3)."""
    L = np.asarray(L, dtype=np.float64)
    out = np.zeros((L.shape[0], s))
    for t in range(L.shape[1]):
        out[:, h[t]] += sgn[t] * L[:, t]
    return out


def truncate(Y, ell):
    """Thin SVD of Y and the leading ell triplets (Sec. 2.5)."""
    U, sig, Vt = np.linalg.svd(np.asarray(Y, dtype=np.float64), full_matrices=False)
    return U[:, :ell], sig[:ell], Vt[:ell].T, sig


def str_factor(Y, ell, ridge_coef):
    """Return (L_eff = U_ell S_ell, sigma (all), gamma) for the STR model.

    gamma = ridge_coef * ||Y||_F^2 / n  (= ridge_coef * trace(Y Y^T) / n).
    """
    Y = np.asarray(Y, dtype=np.float64)
    n = Y.shape[0]
    U, s_ell, V, sig = truncate(Y, ell)
    L_eff = U * s_ell[None, :]
    gamma = ridge_coef * float(np.sum(Y * Y)) / n
    return L_eff, sig, gamma


def str_covariance(L_eff, gamma):
    """Sigma_hat = L_eff L_eff^T + gamma I (Sec. 2.5, ridge stage)."""
    n = L_eff.shape[0]
    return L_eff @ L_eff.T + gamma * np.eye(n)


def gamma_kappa_target(sigma1, kappa_tar):
    """App. D: gamma = sigma_1^2 / (kappa_tar - 1)."""
    return sigma1 * sigma1 / (kappa_tar - 1.0)


def ell_knee(lam_tilde, tau, rho):
    """App. D knee rule: the largest i with lam_i/lam_1 >= tau and
    lam_{i+1}/lam_i <= rho (1-based i).  Returns 0 if none qualifies."""
    lt = np.asarray(lam_tilde, dtype=np.float64)
    best = 0
    for i in range(len(lt) - 1):
        if lt[i] / lt[0] >= tau and lt[i + 1] / lt[i] <= rho:
            best = i + 1
    return best


def embedding_epsilon(L, Phi):
    """Smallest eps with (1-eps)||L^T x||^2 <= ||(L Phi)^T x||^2 <= (1+eps)||L^T x||^2
    on range(L) (Def. of subspace embedding, Sec. 4).  Computed as the
    spectral distance of Q^T Phi Phi^T Q from I, with Q an orthonormal basis
    of range(L^T)."""
    L = np.asarray(L, dtype=np.float64)
    Q, _ = np.linalg.qr(L.T)
    M = Q.T @ np.asarray(Phi, dtype=np.float64)
    ev = np.linalg.eigvalsh(M @ M.T)
    return float(max(ev[-1] - 1.0, 1.0 - ev[0]))

"""GPU parity of the step-level entry points against the FP64 oracle:
projection (Sec. 3.1), fused gradient sweep (eq. npga-unified-grad),
power-method step size (Sec. 3.1 Remark), factor build (Sec. 2.1) and the
MFMA SYRK (explicit-covariance form of Sec. 3.1)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle import projection as oproj
from tests.gpu_util import U32, banner, dev, spec_with, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


PROJ_SIZES = [1, 2, 3, 7, 64, 255, 256, 257, 1000, 4099, 5440, 8192]


@pytest.mark.parametrize("n", PROJ_SIZES)
def test_projection_matches_oracle(npga, n):
    banner(f"projection n={n}")
    rng = np.random.default_rng(n)
    for trial in range(6):
        kind = ["normal", "uniform", "ties"][trial % 3]
        v = gen.random_vector(n, 1000 * n + trial, kind, scale=rng.choice([1e-3, 0.1, 3.0]))
        mu = rng.normal(4e-4, 3e-4, n)
        q = [0.0, 0.5, 0.9, 1.0, 0.99, 0.3][trial]
        r = float(np.quantile(mu, q))
        x_ref, nu_ref, tau_ref = oproj.proj_F(v, mu, r)
        x, nu, tau = npga.project(to_dev(v), to_dev(mu), r)
        x = x.cpu().numpy()
        assert x.min() >= 0.0
        scale = max(np.abs(v).max(), 1.0)
        np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-12 * scale * max(1, n / 100))
        assert abs(x.sum() - 1.0) <= 1e-12 * max(1, n / 100)
        assert mu @ x >= r - 1e-12 * max(abs(r), np.abs(mu).max())
        assert (nu > 0) == (nu_ref > 0) or abs(mu @ x_ref - r) < 1e-15


def test_projection_infeasible(npga):
    mu = np.array([1e-3, 2e-3, 3e-3])
    with pytest.raises(npga.NpgaError) as e:
        npga.project(to_dev(np.zeros(3)), to_dev(mu), 4e-3)
    assert e.value.code == 2


@pytest.mark.parametrize("n,T", [(64, 256), (5, 33), (257, 1031), (1000, 4000), (5440, 3000), (8192, 700)])
def test_gradient_matches_oracle(npga, n, T):
    banner(f"gradient n={n} T={T}")
    spec = spec_with("c2", n, T, seed=7 + n)
    Rt = gen.returns_TxN(spec)           # any matrix is a valid L_eff
    x = gen.random_vector(n, 3 + n, "uniform")
    x = (x / x.sum()).astype(np.float32)
    gamma = 1e-4
    g, f = npga.gradient(to_dev(Rt), to_dev(x), gamma)
    g = g.cpu().numpy()
    L = Rt.T.astype(np.float64)
    xd = x.astype(np.float64)
    u = L.T @ xd
    g_ref = 2 * (L @ u) + 2 * gamma * xd
    f_ref = u @ u + gamma * xd @ xd
    # float32 products, float32 dot of n terms, float32 accumulation of the
    # columns handled by one wavefront, float64 beyond: worst-case bound
    # (n + cols) u32 on the absolute-value sum
    B = 2 * (np.abs(L) @ (np.abs(L).T @ np.abs(xd))) + 2 * gamma * np.abs(xd)
    assert np.all(np.abs(g - g_ref) <= (n + T) * U32 * B + 1e-300)
    assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    assert abs(f - f_ref) <= 1e-5 * f_ref


def test_spectral_norm_estimate(npga):
    spec = spec_with("c2", 300, 2000, seed=11)
    Rt = gen.returns_TxN(spec)
    L = Rt.T.astype(np.float64)
    lmax = np.linalg.eigvalsh(L @ L.T)[-1]
    est = npga.spectral_norm_sq(to_dev(Rt), iters=60, seed=3)
    assert est <= lmax * (1 + 1e-5)      # a Rayleigh value is a lower bound
    assert est >= 0.98 * lmax


@pytest.mark.parametrize("n,T,K", [(300, 2000, 10), (2000, 6000, 5), (517, 3001, 3)])
def test_lanczos_estimate(npga, n, T, K):
    """Lanczos on L L^T: the largest Ritz value is a lower bound of
    lambda_max that reaches it to float32-product accuracy within the step
    cap, while the power method with as many steps is still short of it on
    the clustered top spectrum of a factor model."""
    spec = spec_with("c2", n, T, seed=20 + n)
    spec = spec.__class__(**{**spec.__dict__, "K": K})
    Rt = gen.returns_TxN(spec)
    L = Rt.T.astype(np.float64)
    lmax = np.linalg.eigvalsh(L @ L.T)[-1]
    est, steps = npga.spectral_norm_sq(to_dev(Rt), iters=40, seed=5, method="lanczos", return_steps=True)
    pw = npga.spectral_norm_sq(to_dev(Rt), iters=steps, seed=5, method="power")
    banner(f"lanczos n={n} K={K}: {steps} steps, rel err {(lmax - est) / lmax:.1e}; power {(lmax - pw) / lmax:.1e}")
    assert est <= lmax * (1 + 1e-6)
    assert est >= lmax * (1 - 1e-6)
    assert steps < 40


@pytest.mark.parametrize("n,T", [(64, 256), (1000, 3001), (5440, 2000), (37, 100)])
def test_build_factor_matches_oracle(npga, n, T):
    banner(f"build_factor n={n} T={T}")
    spec = spec_with("c2", n, T, seed=100 + n)
    Rt = gen.returns_TxN(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    mu_ref, L_ref = ofactor.build_factor(Rt.T)
    mu = mu.cpu().numpy()
    Lt = L.cpu().numpy().T.astype(np.float64)
    scale = np.abs(Rt).max()
    assert np.abs(mu - mu_ref).max() <= 4 * np.finfo(np.float64).eps * T * scale
    # L is the float32 rounding of the float64 value: within one float32 ulp
    assert np.all(np.abs(Lt - L_ref) <= 2 * U32 * np.abs(L_ref) + 1e-30)


def test_build_factor_nan(npga):
    spec = spec_with("c1", 64, 128, seed=1)
    Rt = gen.returns_TxN(spec).copy()
    Rt[17, 5] = np.nan
    with pytest.raises(npga.NpgaError) as e:
        npga.build_factor(to_dev(Rt))
    assert e.value.code == 5


@pytest.mark.parametrize("n,T", [(64, 256), (130, 1000), (1000, 5000), (259, 77)])
def test_syrk_matches_oracle(npga, n, T):
    banner(f"syrk n={n} T={T}")
    spec = spec_with("c2", n, T, seed=200 + n)
    Rt = gen.returns_TxN(spec)
    S = npga.syrk(to_dev(Rt)).cpu().numpy().astype(np.float64)
    L = Rt.T.astype(np.float64)
    S_ref = L @ L.T
    B = np.abs(L) @ np.abs(L).T
    # float32 products accumulated in float32 over 256-period chunks,
    # float64 across chunks, final rounding to float32
    assert np.all(np.abs(S - S_ref) <= (256 + 2) * U32 * B + U32 * np.abs(S_ref))
    assert np.array_equal(S, S.T)


@pytest.mark.parametrize("n,T", [(64, 256), (130, 1000), (1000, 5000), (259, 77), (5440, 3000)])
def test_syrk_split_matches_oracle(npga, n, T):
    """Sigma from three bfloat16 planes per entry on the bfloat16 matrix
    cores: the three dropped plane products weigh at most 3 2^-24 (plus the
    planes' own rounding, 2^-25), the kept ones are exact in float32 and are
    accumulated in float32 over 256-period chunks (six per period), float64
    across chunks; the result is within the float32 kernel's bound and as
    close to the exact Sigma as the float32 kernel's."""
    banner(f"syrk split n={n} T={T}")
    spec = spec_with("c2", n, T, seed=210 + n)
    Rt = gen.returns_TxN(spec)
    Ld = to_dev(Rt)
    S = npga.syrk(Ld, method="split").cpu().numpy().astype(np.float64)
    S32 = npga.syrk(Ld).cpu().numpy().astype(np.float64)
    L = Rt.T.astype(np.float64)
    S_ref = L @ L.T
    B = np.abs(L) @ np.abs(L).T
    assert np.all(np.abs(S - S_ref) <= (256 + 2) * U32 * B + U32 * np.abs(S_ref))
    assert np.array_equal(S, S.T)
    e_split = np.abs(S - S_ref).max() / np.abs(S_ref).max()
    e_f32 = np.abs(S32 - S_ref).max() / np.abs(S_ref).max()
    banner(f"  max rel error: split {e_split:.2e}, float32 {e_f32:.2e}")
    assert e_split <= 4 * e_f32 + 4 * U32

"""The paper's variants on the GPU against the oracle: the constant
momentum of the strongly convex specialization (Sec. 3.1), and the STR
options of App. D (on-device Gaussian sketch, CountSketch, knee-rule ell,
kappa_tar ridge)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle.reference import exact_mv_factor
from tests.gpu_util import banner, spec_with, to_dev
from tests.test_gpu_solve import _check_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def npga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as p
    return p


@pytest.mark.parametrize("n,T,ridge", [(300, 100, 1e-3), (1000, 400, 1e-4), (257, 257, 1e-2), (2000, 300, 1e-5)])
def test_constant_momentum(npga, n, T, ridge):
    spec = spec_with("c2", n, T, seed=500 + n)
    Rt = gen.returns_TxN(spec)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    gamma = ridge * float(np.sum(L_o * L_o)) / n
    r = float(np.quantile(mu_o, 0.6))
    ref = exact_mv_factor(L_o, gamma, mu_o, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, gamma=gamma, momentum="constant")
    x_f, info_f = npga.solve(L, mu, r, gamma=gamma)
    banner(f"constant momentum n={n} T={T}: iters {info['iters']} refine {info['refine_iters']} "
           f"(t_k sequence: {info_f['iters']} refine {info_f['refine_iters']})")
    for xx, ii, tag in ((x, info, "constant"), (x_f, info_f, "t_k")):
        assert ii["status"] == 0 and ii["refined"] == 1, (tag, ii)
        _check_parity(xx.cpu().numpy(), ii, L_o, mu_o, r, gamma, ref, f"n={n} {tag}")


def test_constant_momentum_needs_ridge(npga):
    spec = spec_with("c1", 64, 256, seed=3)
    Rt = gen.returns_TxN(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    with pytest.raises(npga.NpgaError) as e:
        npga.solve(L, mu, float(mu.median()), momentum="constant")
    assert e.value.code == 1


def test_philox_sketch_bit_exact(npga):
    """Raw Philox words bit-exact against the oracle generator; the float32
    entries within one float32 rounding (the two sides' float64 log/cos may
    differ in the last bit)."""
    from oracle.philox import gaussian_sketch_philox, philox4x32_10
    T, k, seed = 1000, 300, 12345678901
    S, R = npga.philox_sketch(T, k, seed, raw=True)
    Rh = R.cpu().numpy().view(np.uint32)
    t = np.arange(T, dtype=np.uint64)[None, :]
    j = np.arange(k, dtype=np.uint64)[:, None]
    z = np.zeros((1, 1), dtype=np.uint64)
    o = philox4x32_10(np.broadcast_to(t, (k, T)), np.broadcast_to(j, (k, T)), z, z, seed & 0xFFFFFFFF, seed >> 32)
    np.testing.assert_array_equal(Rh[:, :, 0], o[0])
    np.testing.assert_array_equal(Rh[:, :, 1], o[1])
    S_ref = gaussian_sketch_philox(T, k, seed)
    Sh = S.cpu().numpy()
    assert np.all(np.abs(Sh - S_ref) <= 2.0 ** -23 * np.abs(S_ref) + 1e-30)


def _str_case(n, T, seed):
    spec = spec_with("c2", n, T, seed=seed)
    Rt = gen.returns_TxN(spec)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    r = float(np.quantile(mu_o, 0.6))
    return Rt, mu_o, L_o, r


def _check_str(npga, Rt, mu_o, L_o, r, Y_o, ell, Leff, sigma, gamma, gamma_ref, tag):
    from oracle import sketch as osk
    Le_o, sig_o, _ = osk.str_factor(Y_o, ell, 0.0)
    np.testing.assert_allclose(sigma.cpu().numpy(), sig_o[:ell], rtol=1e-5)
    assert gamma == pytest.approx(gamma_ref, rel=1e-6)
    ref = exact_mv_factor(Le_o, gamma, mu_o, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(Leff, mu, r, gamma=gamma)
    banner(f"{tag}: sigma_1 {float(sigma[0]):.4e} gamma {gamma:.3e} iters {info['iters']}")
    _check_parity(x.cpu().numpy(), info, Le_o, mu_o, r, gamma, ref, tag)


def test_str_philox_sketch(npga):
    from oracle import sketch as osk
    from oracle.philox import gaussian_sketch_philox
    n, T, k, ell, seed = 200, 2000, 256, 32, 77
    Rt, mu_o, L_o, r = _str_case(n, T, 610)
    L, _ = npga.build_factor(to_dev(Rt))
    Leff, sigma, gamma, e = npga.sketch_str_ex(L, k, ell, sketch="gaussian", seed=seed, ridge_coef=1e-4)
    assert e == ell
    Y_o = osk.sketch(L_o, gaussian_sketch_philox(T, k, seed).astype(np.float64).T)
    _check_str(npga, Rt, mu_o, L_o, r, Y_o, ell, Leff, sigma, gamma, 1e-4 * float(np.sum(Y_o * Y_o)) / n,
               "STR philox")


def test_str_countsketch(npga):
    from oracle import sketch as osk
    n, T, k, ell = 200, 3000, 300, 40
    Rt, mu_o, L_o, r = _str_case(n, T, 611)
    h, s = gen.countsketch(T, k, 612)
    L, _ = npga.build_factor(to_dev(Rt))
    Leff, sigma, gamma, e = npga.sketch_str_ex(L, k, ell, sketch="count", h=to_dev(h), sgn=to_dev(s),
                                               ridge_coef=1e-4)
    Y_o = osk.countsketch_apply(L_o, h, s, k)
    _check_str(npga, Rt, mu_o, L_o, r, Y_o, ell, Leff, sigma, gamma, 1e-4 * float(np.sum(Y_o * Y_o)) / n,
               "STR countsketch")
    bad = h.copy()
    bad[17] = k                                  # bucket out of range
    with pytest.raises(npga.NpgaError) as err:
        npga.sketch_str_ex(L, k, ell, sketch="count", h=to_dev(bad), sgn=to_dev(s))
    assert err.value.code == 1


def test_str_knee_and_kappa(npga):
    """Knee rule (App. D) over the ell_cap + 1 leading eigenvalues and the
    kappa_tar ridge gamma = sigma_1^2/(kappa_tar - 1)."""
    from oracle import sketch as osk
    n, T, k, cap = 300, 3000, 400, 60
    Rt, mu_o, L_o, r = _str_case(n, T, 613)
    L, _ = npga.build_factor(to_dev(Rt))
    S = gen.gaussian_sketch(T, k, 614)
    Y_o = osk.sketch(L_o, S.astype(np.float64).T)
    lam_o = np.linalg.svd(Y_o, compute_uv=False) ** 2
    tau, rho = 1e-3, 0.9
    ell_o = osk.ell_knee(lam_o[:cap + 1], tau, rho)
    # the decision is not marginal at these thresholds
    i = ell_o - 1
    assert ell_o > 0 and lam_o[i + 1] / lam_o[i] < rho - 1e-6 and lam_o[i] / lam_o[0] > tau * (1 + 1e-6)
    kappa = 200.0
    Leff, sigma, gamma, e = npga.sketch_str_ex(L, k, cap, sketch="gaussian", S_kxT=to_dev(S), ell_rule="knee",
                                               tau=tau, rho=rho, kappa_tar=kappa)
    banner(f"knee: ell {e} (oracle {ell_o}), gamma {gamma:.3e}")
    assert e == ell_o
    g_ref = osk.gamma_kappa_target(float(np.sqrt(lam_o[0])), kappa)
    _check_str(npga, Rt, mu_o, L_o, r, Y_o, e, Leff, sigma, gamma, g_ref, "STR knee + kappa")
    # kappa(Sigma_hat) = (sigma_1^2 + gamma)/gamma = kappa_tar
    assert (float(sigma[0]) ** 2 + gamma) / gamma == pytest.approx(kappa, rel=1e-5)

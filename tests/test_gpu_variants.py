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


@pytest.mark.parametrize("n,T,ridge", [(300, 100, 1e-3), (1000, 400, 1e-4), (257, 257, 1e-2)])
def test_constant_momentum(npga, n, T, ridge):
    spec = spec_with("c2", n, T, seed=500 + n)
    Rt = gen.returns_TxN(spec)
    mu_o, L_o = ofactor.build_factor(Rt.T)
    gamma = ridge * float(np.sum(L_o * L_o)) / n
    r = float(np.quantile(mu_o, 0.6))
    ref = exact_mv_factor(L_o, gamma, mu_o, r)
    L, mu = npga.build_factor(to_dev(Rt))
    x, info = npga.solve(L, mu, r, gamma=gamma, momentum="constant")
    _, info_f = npga.solve(L, mu, r, gamma=gamma)
    banner(f"constant momentum n={n} T={T}: iters {info['iters']} (t_k sequence: {info_f['iters']})")
    assert info["status"] == 0 and info["refined"] == 1
    _check_parity(x.cpu().numpy(), info, L_o, mu_o, r, gamma, ref, f"n={n}")


def test_constant_momentum_needs_ridge(npga):
    spec = spec_with("c1", 64, 256, seed=3)
    Rt = gen.returns_TxN(spec)
    L, mu = npga.build_factor(to_dev(Rt))
    with pytest.raises(npga.NpgaError) as e:
        npga.solve(L, mu, float(mu.median()), momentum="constant")
    assert e.value.code == 1

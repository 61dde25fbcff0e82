"""Full-size parity at the headline workload (n=5440, T=48374) in the
launch configuration the benchmark times, against the stored oracle
solution tests/golden/c2_solution.json (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from oracle.reference import factor_objective
from tests.golden.make_golden import panel_digest
from tests.gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_solution.json")


@pytest.fixture(scope="module")
def c2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as npga
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    spec = gen.SPECS["c2"]
    banner("c2: generating the panel")
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"], "regenerated panel differs from the stored one"
    r = gen.target_return(spec, Rt)
    assert r == ref["r"]
    mu_o, L_o = ofactor.build_factor(Rt.T)
    R = to_dev(Rt)
    L, mu = npga.build_factor(R)
    return npga, ref, L, mu, L_o, mu_o, r


@pytest.mark.parametrize("path", ["gemv", "syrk"])
def test_c2_parity(c2, path):
    npga, ref, L, mu, L_o, mu_o, r = c2
    banner(f"c2 solve path={path}")
    x, info = npga.solve(L, mu, r, path=path)
    banner(f"c2 {path}: status={info['status_name']} iters={info['iters']} refine={info['refine_iters']} "
           f"res={info['final_residual']:.2e} ms={info['time_ms']:.1f}")
    assert info["status"] == 0 and info["refined"] == 1
    assert info["residual"] <= 1e-6
    xs = np.asarray(ref["x"])
    xg = x.cpu().numpy().astype(np.float64)
    f_ref = ref["objective"]
    f_gpu = factor_objective(L_o, 0.0, xg)
    assert xg.min() >= 0.0
    assert abs(xg.sum() - 1.0) <= 1e-6
    assert mu_o @ xg >= r - 1e-6 * max(1.0, abs(r))
    assert abs(f_gpu - f_ref) <= 1e-6 * f_ref, (f_gpu, f_ref)
    assert abs(info["objective"] - f_ref) <= 1e-6 * f_ref, (info["objective"], f_ref)
    assert np.abs(xg - xs).max() <= 1e-5, np.abs(xg - xs).max()
    assert info["support"] == ref["support"]

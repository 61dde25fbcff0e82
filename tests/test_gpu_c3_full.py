"""Full-size STR workload (n=5440, T=48374, k=4096, ell=512) against the
stored oracle STR solution tests/golden/c3_solution.json (oracle-only
script tests/golden/make_golden.py), from the identical float32 sketch."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from tests.golden.make_golden import panel_digest
from tests.gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_solution.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="c3 golden not generated")
def test_c3_str_parity():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as npga
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    spec = gen.SPECS["c2"]
    banner("c3: generating panel and sketch")
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    r = gen.target_return(spec, Rt)
    S = gen.gaussian_sketch(spec.T, ref["k"], seed=ref["sketch_seed"])
    assert panel_digest(S) == ref["sketch_sha256"]
    L, mu = npga.build_factor(to_dev(Rt))
    Sd = to_dev(S)
    del S
    banner("c3: sketch-truncate-ridge")
    Leff, sigma, gamma = npga.sketch_str(L, Sd, ref["ell"], ridge_coef=ref["ridge_coef"])
    del Sd
    sig = sigma.cpu().numpy().astype(np.float64)
    sig_ref = np.asarray(ref["sigma"])
    np.testing.assert_allclose(sig, sig_ref, rtol=1e-5)
    assert abs(gamma - ref["gamma"]) <= 1e-6 * ref["gamma"]
    banner("c3: STR solve")
    x, info = npga.solve(Leff, mu, r, gamma=gamma)
    banner(f"c3: status={info['status_name']} iters={info['iters']} refine={info['refine_iters']} "
           f"obj={info['objective']:.6e} ref={ref['objective']:.6e}")
    assert info["status"] == 0
    xg = x.cpu().numpy().astype(np.float64)
    xs = np.asarray(ref["x"])
    assert xg.min() >= 0 and abs(xg.sum() - 1) <= 1e-6
    assert abs(info["objective"] - ref["objective"]) <= 1e-6 * ref["objective"]
    assert np.abs(xg - xs).max() <= 1e-5, np.abs(xg - xs).max()
    # full-model objective of the STR portfolio (fused sweep on L) -> gap of Sec. 5.1
    _, f_full = npga.gradient(L, x, 0.0)
    assert abs(f_full - ref["full_model_objective_of_str_x"]) <= 1e-5 * ref["full_model_objective_of_str_x"]

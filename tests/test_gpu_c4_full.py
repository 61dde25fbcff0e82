"""Full-size frontier (n = 2000, T = 20000, 128 targets) against the stored
oracle solutions tests/golden/c4_frontier.json (oracle-only script
tests/golden/make_golden.py): every target's objective, and the minimiser
at a sample of targets, in the launch configuration the benchmark uses."""
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c4_frontier.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="c4 golden not generated")
def test_c4_frontier_parity():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as npga
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    spec = gen.SPECS["c4"]
    banner("c4: generating panel")
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    mu_o, L_o = ofactor.build_factor(Rt.T)
    L, mu = npga.build_factor(to_dev(Rt))
    rs = ref["targets"]
    best, _ = npga.batched_tune(L, len(rs))
    banner(f"c4: batched solve of {len(rs)} targets (config {best})")
    X, infos = npga.solve_batched(L, mu, rs, batch_config=best)
    Xh = X.cpu().numpy().astype(np.float64)
    worst = 0.0
    for p in ref["points"]:
        j = p["j"]
        assert infos[j]["status"] == 0, (j, infos[j])
        x = Xh[j]
        assert x.min() >= 0 and abs(x.sum() - 1) <= 1e-6
        assert mu_o @ x >= rs[j] - 1e-6 * max(1.0, abs(rs[j]))
        f = factor_objective(L_o, 0.0, x)
        rel = abs(f - p["objective"]) / p["objective"]
        worst = max(worst, rel)
        assert rel <= 1e-6, (j, f, p["objective"])
        assert abs(infos[j]["objective"] - p["objective"]) <= 1e-6 * p["objective"], j
        if "x" in p:
            assert np.abs(x - np.asarray(p["x"])).max() <= 1e-5, j
    banner(f"c4: worst relative objective error {worst:.2e}; iters max {max(i['iters'] for i in infos)}")
    # bfloat16 storage of the same factor: solver parity is covered at small
    # sizes; here the quantisation gap against the float32 frontier
    Xb, infos_b = npga.solve_batched(npga.to_bf16(L), mu, rs)
    Xbh = Xb.cpu().numpy().astype(np.float64)
    gaps = []
    for p in ref["points"]:
        j = p["j"]
        assert infos_b[j]["status"] == 0
        gaps.append((factor_objective(L_o, 0.0, Xbh[j]) - p["objective"]) / p["objective"])
    banner(f"c4 bf16: quantisation gap max {max(gaps):.2e} median {sorted(gaps)[len(gaps) // 2]:.2e}")
    assert min(gaps) >= -1e-6 and max(gaps) <= 1e-2

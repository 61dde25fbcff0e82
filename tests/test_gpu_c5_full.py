"""Full-size adjoint (n = 5440, T = 48374) at the stored C2 minimiser
against the stored oracle adjoint tests/golden/c5_adjoint.json (dense
float64 KKT solve on the face; oracle-only script
tests/golden/make_golden.py): dl/dmu everywhere, dl/dL at 256 sampled
entries, dl/dr and dl/dgamma; bar 1e-4 of the largest entry."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import gen
from oracle import factor as ofactor
from tests.golden.make_golden import panel_digest
from tests.gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(__file__), "golden")
GOLDEN = os.path.join(HERE, "c5_adjoint.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="c5 golden not generated")
def test_c5_adjoint_full_size():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_02917_amd as npga
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    with open(os.path.join(HERE, "c2_solution.json")) as fh:
        c2 = json.load(fh)
    spec = gen.SPECS["c2"]
    banner("c5: generating panels")
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == c2["panel_sha256"]
    x = np.asarray(c2["x"]).astype(np.float32)
    Rtest = gen.heldout_returns_TxN(spec, ref["test_periods"], ref["heldout_seed"])
    mu_t, L_t = ofactor.build_factor(Rtest.T)
    g = (2.0 * (L_t @ (L_t.T @ x.astype(np.float64))) - mu_t).astype(np.float32)
    L, mu = npga.build_factor(to_dev(Rt))
    del Rt
    banner("c5: backward")
    dmu, dL, info = npga.backward(L, mu, ref["r"], to_dev(x), to_dev(g))
    banner(f"c5: cg {info['cg_iters']} support {info['support']} residual {info['residual']:.1e} "
           f"time {info['time_ms']:.1f} ms")
    assert info["status"] == 0 and info["degenerate"] == 0
    assert info["support"] == ref["support"] and info["return_active"] == int(ref["active"])
    dmu_ref = np.asarray(ref["dmu"])
    err = np.abs(dmu.cpu().numpy() - dmu_ref).max()
    assert err <= 1e-4 * np.abs(dmu_ref).max(), (err, np.abs(dmu_ref).max())
    dLh = dL.cpu()
    for i, t, v in ref["dL_samples"]:
        assert abs(float(dLh[t, i]) - v) <= 1e-4 * ref["dL_max"], (i, t, float(dLh[t, i]), v)
    assert float(dL.abs().max()) == pytest.approx(ref["dL_max"], rel=1e-3)
    assert info["dl_dr"] == pytest.approx(ref["dr"], rel=1e-4)
    assert info["dl_dgamma"] == pytest.approx(ref["dgamma"], rel=1e-4)

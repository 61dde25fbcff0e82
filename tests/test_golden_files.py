"""CPU checks of the stored oracle solution: it belongs to the regenerated
panel and is a feasible point of eq. mv with the stored objective."""
import json
import os

import numpy as np
import pytest

import gen
from oracle import factor as ofactor
from oracle.reference import factor_objective
from tests.golden.make_golden import panel_digest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_solution.json")


@pytest.mark.slow
def test_c2_golden_consistent():
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    spec = gen.SPECS["c2"]
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    r = gen.target_return(spec, Rt)
    assert r == ref["r"]
    mu, L = ofactor.build_factor(Rt.T)
    x = np.asarray(ref["x"])
    assert x.min() >= 0 and abs(x.sum() - 1) <= 1e-12
    assert mu @ x >= r - 1e-14
    assert factor_objective(L, 0.0, x) == pytest.approx(ref["objective"], rel=1e-12)
    k = ref["kkt"]
    assert k["stat_support"] <= 1e-9 and k["dual_offsupport"] >= -1e-9


GOLDEN_C3 = os.path.join(os.path.dirname(__file__), "golden", "c3_solution.json")


@pytest.mark.slow
def test_c3_golden_consistent():
    """Stored STR solution: feasible for eq. mv on the regenerated panel,
    with a valid KKT certificate and the gap recorded against c2."""
    with open(GOLDEN_C3) as fh:
        ref = json.load(fh)
    with open(GOLDEN) as fh:
        ref2 = json.load(fh)
    spec = gen.SPECS["c2"]
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    assert gen.target_return(spec, Rt) == ref["r"]
    mu, L = ofactor.build_factor(Rt.T)
    x = np.asarray(ref["x"])
    assert x.min() >= 0 and abs(x.sum() - 1) <= 1e-12
    assert mu @ x >= ref["r"] - 1e-14
    # the STR portfolio is feasible for the full model, so it cannot beat x*
    f_full = factor_objective(L, 0.0, x)
    assert f_full == pytest.approx(ref["full_model_objective_of_str_x"], rel=1e-12)
    assert f_full >= ref2["objective"] * (1 - 1e-12)
    sig = np.asarray(ref["sigma"])
    assert np.all(np.diff(sig) <= 0) and sig[-1] >= ref["sigma_513"]
    k = ref["kkt"]
    assert k["stat_support"] <= 1e-9 and k["dual_offsupport"] >= -1e-9


GOLDEN_C4 = os.path.join(os.path.dirname(__file__), "golden", "c4_frontier.json")


@pytest.mark.slow
def test_c4_golden_consistent():
    """Stored frontier: regenerated panel, stored minimisers feasible with
    the stored objectives, f* nondecreasing and convex along the targets."""
    with open(GOLDEN_C4) as fh:
        ref = json.load(fh)
    spec = gen.SPECS["c4"]
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    mu, L = ofactor.build_factor(Rt.T)
    rs = np.asarray(ref["targets"])
    np.testing.assert_allclose(rs, gen.frontier_targets_from_mv(ref["r_mv"], float(mu.max()), 128), rtol=0,
                               atol=0)
    f = np.array([p["objective"] for p in ref["points"]])
    assert np.all(np.diff(f) >= 0) and np.all(f[:-2] - 2 * f[1:-1] + f[2:] >= -1e-12 * f.max())
    assert f[0] == pytest.approx(ref["f_mv"], rel=1e-9)
    for p in ref["points"]:
        if "x" not in p:
            continue
        x = np.asarray(p["x"])
        assert x.min() >= 0 and abs(x.sum() - 1) <= 1e-12
        assert mu @ x >= p["r"] - 1e-14
        assert factor_objective(L, 0.0, x) == pytest.approx(p["objective"], rel=1e-12)


GOLDEN_C5 = os.path.join(os.path.dirname(__file__), "golden", "c5_adjoint.json")


@pytest.mark.slow
def test_c5_golden_consistent():
    """Stored full-size adjoint: zero off the support, and the constraint
    rows of the adjoint system (1^T a = 0, mu_S^T a = 0) give
    sum(dl/dmu) = -dl/dr and mu^T dl/dmu = -r dl/dr."""
    with open(GOLDEN_C5) as fh:
        ref = json.load(fh)
    with open(GOLDEN) as fh:
        c2 = json.load(fh)
    x = np.asarray(c2["x"])
    dmu = np.asarray(ref["dmu"])
    assert np.all(dmu[x <= 0] == 0.0) and ref["support"] == int((x > 0).sum()) and ref["active"]
    spec = gen.SPECS["c2"]
    Rt = gen.returns_TxN(spec)
    mu = Rt.astype(np.float64).mean(axis=0)
    assert dmu.sum() == pytest.approx(-ref["dr"], rel=1e-8)
    assert mu @ dmu == pytest.approx(-ref["r"] * ref["dr"], rel=1e-6)


GOLDEN_N8192 = os.path.join(os.path.dirname(__file__), "golden", "n8192_solution.json")


def test_n8192_golden_consistent():
    """Stored solution at the largest n (8192 assets, 600 periods, ridge):
    it belongs to the regenerated panel, is feasible, and its KKT conditions
    hold when recomputed here in factor form (gradient 2 L (L^T x) + 2 gamma x)."""
    from tests.gpu_util import spec_with
    with open(GOLDEN_N8192) as fh:
        ref = json.load(fh)
    spec = spec_with("c2", 8192, 600, seed=712)
    spec = spec.__class__(**{**spec.__dict__, "K": 5})
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    mu, L = ofactor.build_factor(Rt.T)
    gamma, r = ref["gamma"], ref["r"]
    assert gamma == pytest.approx(1e-3 * float(np.sum(L * L)) / 8192, rel=1e-12)
    x = np.asarray(ref["x"])
    assert x.min() >= 0 and abs(x.sum() - 1) <= 1e-12
    assert mu @ x >= r - 1e-14
    assert factor_objective(L, gamma, x) == pytest.approx(ref["objective"], rel=1e-12)
    g = 2.0 * (L @ (L.T @ x)) + 2.0 * gamma * x
    d = g - ref["lambda"] - ref["nu"] * mu  # reduced costs
    S = x > 0
    scale = np.abs(g).max()
    assert np.abs(d[S]).max() <= 1e-9 * scale
    assert d[~S].min() >= -1e-8 * scale
    assert ref["nu"] >= 0 and ref["nu"] * (mu @ x - r) <= 1e-12 * scale


GOLDEN_C4_BF16 = os.path.join(os.path.dirname(__file__), "golden", "c4_frontier_bf16.json")


@pytest.mark.slow
def test_c4_bf16_golden_consistent():
    """Stored frontier on the bfloat16 factor: same panel and targets as the
    float32 frontier, f* nondecreasing along the targets, and at the stored
    minimisers feasibility, the stored objective and the KKT conditions
    recomputed here in factor form on bf16(float32(L))."""
    from oracle import quantize as oq
    with open(GOLDEN_C4_BF16) as fh:
        ref = json.load(fh)
    with open(GOLDEN_C4) as fh:
        c4 = json.load(fh)
    assert ref["panel_sha256"] == c4["panel_sha256"] and ref["targets"] == c4["targets"]
    spec = gen.SPECS["c4"]
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == ref["panel_sha256"]
    mu, L = ofactor.build_factor(Rt.T)
    Lq = oq.round_to_bf16(L.astype(np.float32))
    f = np.array([p["objective"] for p in ref["points"]])
    assert np.all(np.diff(f) >= -1e-12 * f.max())
    for p in ref["points"]:
        if "x" not in p:
            continue
        x = np.asarray(p["x"])
        assert x.min() >= 0 and abs(x.sum() - 1) <= 1e-12
        assert mu @ x >= p["r"] - 1e-14
        assert factor_objective(Lq, 0.0, x) == pytest.approx(p["objective"], rel=1e-12)
        g = 2.0 * (Lq @ (Lq.T @ x))
        d = g - p["lambda"] - p["nu"] * mu
        S = x > 0
        scale = np.abs(g).max()
        assert np.abs(d[S]).max() <= 1e-9 * scale and d[~S].min() >= -1e-9 * scale

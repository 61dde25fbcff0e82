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

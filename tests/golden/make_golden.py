"""Writes the stored oracle solutions used by the full-size GPU parity tests.

Calls only the oracle (and the seeded generator).  Usage:
    python -m tests.golden.make_golden c2
Output: tests/golden/<name>_solution.json with the exact minimiser x* of
eq. mv for the workload, its objective, multipliers, the target r and a
SHA-256 of the float32 return panel (so a test can tell that its
regenerated input is the one the solution belongs to).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
from oracle import factor as ofactor  # noqa: E402
from oracle import qp  # noqa: E402
from oracle.reference import exact_mv, factor_objective  # noqa: E402


def panel_digest(Rt):
    return hashlib.sha256(np.ascontiguousarray(Rt).tobytes()).hexdigest()


def make(name):
    spec = gen.SPECS[name]
    t0 = time.time()
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    mu, L = ofactor.build_factor(Rt.T)
    Q = L @ L.T
    print(f"{name}: data + covariance {time.time() - t0:.1f}s", flush=True)
    out = exact_mv(Q, mu, r, fista_tol=1e-9)
    x = out["x"]
    rep = qp.kkt_report(2 * Q, np.zeros(spec.n), mu, r, x, out["lam"], out["nu"])
    assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=np.abs(mu).max()), rep
    f = factor_objective(L, 0.0, x)
    doc = {
        "workload": name, "n": spec.n, "T": spec.T, "seed": spec.seed, "r": r,
        "panel_sha256": panel_digest(Rt),
        "objective": f, "lambda": out["lam"], "nu": out["nu"],
        "support": int((x > 0).sum()), "npga_iters": out["npga_iters"],
        "kkt": rep, "x": [float(v) for v in x],
    }
    path = os.path.join(HERE, f"{name}_solution.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path}: f*={f:.6e} support={doc['support']} ({time.time() - t0:.1f}s)", flush=True)


if __name__ == "__main__":
    make(sys.argv[1] if len(sys.argv) > 1 else "c2")

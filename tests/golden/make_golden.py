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


def make_c3():
    """STR workload: the c2 factor, Gaussian sketch k = 4096 (seed 3),
    ell = 512, gamma = 1e-4 trace(Y Y^T)/n; oracle STR model from the same S."""
    from oracle import sketch as osketch
    spec = gen.SPECS["c2"]
    t0 = time.time()
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    mu, L = ofactor.build_factor(Rt.T)
    S = gen.gaussian_sketch(spec.T, 4096, seed=gen.factor_model.SKETCH_SEED_C3)
    s_digest = panel_digest(S)
    Y = osketch.sketch(L, S.astype(np.float64).T)
    del S
    print(f"c3: sketch {time.time() - t0:.1f}s", flush=True)
    L_eff, sig, gamma = osketch.str_factor(Y, 512, 1e-4)
    print(f"c3: svd {time.time() - t0:.1f}s", flush=True)
    Q = L_eff @ L_eff.T + gamma * np.eye(spec.n)
    out = exact_mv(Q, mu, r, fista_tol=1e-10)
    x = out["x"]
    rep = qp.kkt_report(2 * Q, np.zeros(spec.n), mu, r, x, out["lam"], out["nu"])
    assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=np.abs(mu).max()), rep
    f_str = factor_objective(L_eff, gamma, x)
    f_full_at_str = factor_objective(L, 0.0, x)
    with open(os.path.join(HERE, "c2_solution.json")) as fh:
        f_full = json.load(fh)["objective"]
    doc = {
        "workload": "c3", "n": spec.n, "T": spec.T, "k": 4096, "ell": 512, "ridge_coef": 1e-4,
        "sketch_seed": gen.factor_model.SKETCH_SEED_C3, "r": r,
        "panel_sha256": panel_digest(Rt), "sketch_sha256": s_digest,
        "gamma": gamma, "sigma": [float(v) for v in sig[:512]], "sigma_513": float(sig[512]),
        "objective": f_str, "lambda": out["lam"], "nu": out["nu"],
        "support": int((x > 0).sum()), "kkt": rep,
        "full_model_objective_of_str_x": f_full_at_str, "full_model_gap": qp.gap(f_full_at_str, f_full),
        "x": [float(v) for v in x],
    }
    path = os.path.join(HERE, "c3_solution.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path}: f*={f_str:.6e} gap={doc['full_model_gap']:.4f} ({time.time() - t0:.1f}s)", flush=True)


C4_SAMPLED = [0, 1, 16, 32, 48, 64, 80, 96, 112, 127]


def make_c4():
    """Frontier workload: n = 2000, T = 20000, 128 targets from r_mv to
    0.95 max mu; exact objective and multipliers at every target, the
    minimiser itself at a sample of the targets."""
    from oracle.frontier import min_variance
    spec = gen.SPECS["c4"]
    t0 = time.time()
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    Q = L @ L.T
    x_mv, r_mv = min_variance(Q, mu)
    rs = gen.frontier_targets_from_mv(r_mv, float(mu.max()), 128)
    print(f"c4: min-variance r_mv={r_mv:.6e} ({time.time() - t0:.1f}s)", flush=True)
    pts = []
    for j in range(len(rs)):
        out = exact_mv(Q, mu, float(rs[j]), fista_tol=1e-10)
        x = out["x"]
        rep = qp.kkt_report(2 * Q, np.zeros(spec.n), mu, float(rs[j]), x, out["lam"], out["nu"])
        assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=np.abs(mu).max()), rep
        p = {"j": j, "r": float(rs[j]), "objective": factor_objective(L, 0.0, x), "nu": out["nu"],
             "lambda": out["lam"], "support": int((x > 0).sum())}
        if j in C4_SAMPLED:  # minimisers stored at a sample of the targets only (file size)
            p["x"] = [float(v) for v in x]
        pts.append(p)
        print(f"c4: target {j} f*={p['objective']:.6e} ({time.time() - t0:.1f}s)", flush=True)
    doc = {"workload": "c4", "n": spec.n, "T": spec.T, "seed": spec.seed, "m": 128,
           "panel_sha256": panel_digest(Rt), "r_mv": r_mv, "f_mv": factor_objective(L, 0.0, x_mv),
           "targets": [float(v) for v in rs], "points": pts}
    path = os.path.join(HERE, "c4_frontier.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path} ({time.time() - t0:.1f}s)", flush=True)


def make_c4_bf16():
    """The frontier workload on a bfloat16 factor: the oracle's float64 L
    rounded to float32 (the precision the device builds it in), then to
    bfloat16 by round-to-nearest-even (oracle.quantize), at the 128 targets
    of c4_frontier.json.  The exact minimiser of every target on that
    factor is the reference of the bfloat16 frontier's solver error; the
    float32 frontier's stored objectives give its quantisation error."""
    from oracle import quantize as oq
    spec = gen.SPECS["c4"]
    t0 = time.time()
    with open(os.path.join(HERE, "c4_frontier.json")) as fh:
        c4 = json.load(fh)
    Rt = gen.returns_TxN(spec)
    assert panel_digest(Rt) == c4["panel_sha256"]
    mu, L = ofactor.build_factor(Rt.T)
    del Rt
    Lq = oq.round_to_bf16(L.astype(np.float32))
    del L
    Q = Lq @ Lq.T
    rs = c4["targets"]
    pts = []
    for j, r in enumerate(rs):
        out = exact_mv(Q, mu, float(r), fista_tol=1e-10)
        x = out["x"]
        rep = qp.kkt_report(2 * Q, np.zeros(spec.n), mu, float(r), x, out["lam"], out["nu"])
        assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=np.abs(mu).max()), rep
        p = {"j": j, "r": float(r), "objective": factor_objective(Lq, 0.0, x), "nu": out["nu"],
             "lambda": out["lam"], "support": int((x > 0).sum())}
        if j in C4_SAMPLED:
            p["x"] = [float(v) for v in x]
        pts.append(p)
        print(f"c4_bf16: target {j} f*={p['objective']:.6e} ({time.time() - t0:.1f}s)", flush=True)
    doc = {"workload": "c4_bf16", "n": spec.n, "T": spec.T, "seed": spec.seed, "m": len(rs),
           "panel_sha256": c4["panel_sha256"], "factor": "bf16(float32(L)), round to nearest even",
           "targets": rs, "points": pts}
    path = os.path.join(HERE, "c4_frontier_bf16.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path} ({time.time() - t0:.1f}s)", flush=True)


def make_c5():
    """Adjoint at full size: the out-of-sample loss l(w) = w^T Sigma_test w -
    mu_test^T w (held-out block: same B and drift, fresh draws, seed 105,
    5000 periods) differentiated at the stored C2 minimiser."""
    from oracle.adjoint import kkt_adjoint
    spec = gen.SPECS["c2"]
    t0 = time.time()
    with open(os.path.join(HERE, "c2_solution.json")) as fh:
        c2 = json.load(fh)
    x = np.asarray(c2["x"]).astype(np.float32).astype(np.float64)  # the point the GPU is handed
    Rtest = gen.heldout_returns_TxN(spec, 5000, gen.factor_model.HELDOUT_SEED_C5)
    mu_t, L_t = ofactor.build_factor(Rtest.T)
    g = (2.0 * (L_t @ (L_t.T @ x)) - mu_t).astype(np.float32).astype(np.float64)
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    del Rt
    print(f"c5: data {time.time() - t0:.1f}s", flush=True)
    adj = kkt_adjoint(L, 0.0, mu, c2["r"], x, c2["lambda"], c2["nu"], g)
    print(f"c5: adjoint {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(55)
    idx_i = rng.integers(0, spec.n, 256)
    idx_t = rng.integers(0, spec.T, 256)
    a, u, v = adj["a"], L.T @ x, L.T @ adj["a"]
    samples = [[int(i), int(t), float(-2.0 * (a[i] * u[t] + x[i] * v[t]))] for i, t in zip(idx_i, idx_t)]
    dL_max = 0.0
    for t0_ in range(0, spec.T, 4096):
        blk = -2.0 * (np.outer(a, u[t0_:t0_ + 4096]) + np.outer(x, v[t0_:t0_ + 4096]))
        dL_max = max(dL_max, float(np.abs(blk).max()))
    doc = {"workload": "c5", "n": spec.n, "T": spec.T, "test_periods": 5000,
           "heldout_seed": gen.factor_model.HELDOUT_SEED_C5, "r": c2["r"],
           "support": int(len(adj["support"])), "active": bool(adj["active"]),
           "dr": adj["dr"], "dgamma": adj["dgamma"], "dmu": [float(v_) for v_ in adj["dmu"]],
           "dL_samples": samples, "dL_max": dL_max}
    path = os.path.join(HERE, "c5_adjoint.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path} ({time.time() - t0:.1f}s)", flush=True)


def make_n8192():
    """Largest supported n: n = 8192, T = 600, K = 5 (C2 distributions,
    seed 712), ridge 1e-3 tr(L L^T)/n, r = 60th percentile of mu."""
    from tests.gpu_util import spec_with
    t0 = time.time()
    spec = spec_with("c2", 8192, 600, seed=712)
    spec = spec.__class__(**{**spec.__dict__, "K": 5})
    Rt = gen.returns_TxN(spec)
    mu, L = ofactor.build_factor(Rt.T)
    gamma = 1e-3 * float(np.sum(L * L)) / spec.n
    r = float(np.quantile(mu, 0.6))
    Q = L @ L.T + gamma * np.eye(spec.n)
    out = exact_mv(Q, mu, r, fista_tol=1e-10)
    x = out["x"]
    rep = qp.kkt_report(2 * Q, np.zeros(spec.n), mu, r, x, out["lam"], out["nu"])
    assert qp.certificate_ok(rep, tol_stat=1e-9, tol_feas=1e-12, r_scale=np.abs(mu).max()), rep
    doc = {"workload": "n8192", "n": spec.n, "T": spec.T, "K": 5, "seed": 712, "gamma": gamma, "r": r,
           "panel_sha256": panel_digest(Rt), "objective": factor_objective(L, gamma, x),
           "lambda": out["lam"], "nu": out["nu"], "support": int((x > 0).sum()), "kkt": rep,
           "x": [float(v) for v in x]}
    path = os.path.join(HERE, "n8192_solution.json")
    with open(path, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {path}: f*={doc['objective']:.6e} support={doc['support']} ({time.time() - t0:.1f}s)", flush=True)


def make(name):
    if name == "n8192":
        return make_n8192()
    if name == "c5":
        return make_c5()
    if name == "c3":
        return make_c3()
    if name == "c4":
        return make_c4()
    if name == "c4_bf16":
        return make_c4_bf16()
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

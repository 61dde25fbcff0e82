#!/usr/bin/env python3
"""NPGA benchmark on one MI355X: time-to-1e-6 at n=5440, T=48374.

Workload: the unreduced full model at the paper's headline shape
(Sec. 5.4: n = 5440 assets, T = 48374 periods), on synthetic 10-factor
returns with Student-t(4) idiosyncratic noise (gen.SPECS["c2"]), target
r = 60th percentile of the asset means.

One step = npga_build_factor (mu, L from the float32 returns already in
HBM) + npga_solve (power-method step size, NPGA to residual 1e-6, float64
refinement).  ``value`` is the median over the timed steps of the GPU time
from npga_solve entry until the stopping test first passed (residual
<= 1e-6), in seconds; ``ms_per_step`` is the wall time of a whole step.

Prints ONE JSON line.  --gpus N with N > 1 exits: the solver runs on one GPU.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--path", default="gemv", choices=["gemv", "syrk", "auto"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-syrk-compare", action="store_true")
    ap.add_argument("--no-str", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-restart-compare", action="store_true")
    ap.add_argument("--no-frontier", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-probe-gb", type=float, default=0.0,
                    help="run one plain device copy of this size first (calibrates HBM byte counters)")
    ap.add_argument("--frontier-seq", type=int, default=4,
                    help="single solves timed for the one-at-a-time comparison")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def sweep_traffic(path_used):
    """HBM bytes per sweep launch from the committed counter passes
    (profiles/k_sweep_c2_traffic.json), or None when the fused sweep's
    source has changed since they were taken (or another path ran)."""
    import hashlib
    import re
    if path_used != 1:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", "k_sweep_c2_traffic.json")) as fh:
            doc = json.load(fh)
        src = open(os.path.join(ROOT, doc["source_file"])).read()
    except (OSError, ValueError, KeyError):
        return None
    m = re.search(r"template <int E, typename TL>\n__global__ __launch_bounds__\(256\) void k_sweep\(SolveArgs a\) "
                  r"\{.*?\n\}\n", src, re.S)
    if not m:
        return None
    # the kernel's text and the device helpers it calls (wave sums, loads)
    h = hashlib.sha256(m.group(0).encode())
    for extra in doc.get("helper_files", []):
        try:
            h.update(open(os.path.join(ROOT, extra)).read().encode())
        except OSError:
            return None
    if h.hexdigest() != doc["source_sha256"]:
        return None
    return doc["traffic_bytes_per_launch"]


def cpu_baseline(Rt, r, gpu_grad_evals, budget_s):
    """The FP64 oracle's Algorithm 1 timed on a bounded sample: a few
    iterations on the full factor, scaled to the GPU's gradient count."""
    import numpy as np
    from oracle import factor as ofactor
    from oracle import npga as onpga
    try:
        from threadpoolctl import threadpool_info
        cores = sum(int(p.get("num_threads", 0)) for p in threadpool_info()
                    if p.get("user_api") == "blas") or os.cpu_count()
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    mu, L = ofactor.build_factor(Rt.T)
    model = onpga.FactorModel(L)
    n = L.shape[0]
    alpha = 1.0 / (2.0 * float(np.sum(L * L)))  # ||L||_2^2 <= ||L||_F^2: a safe fixed step
    x0 = np.full(n, 1.0 / n)
    t0 = time.perf_counter()
    onpga.npga(model, mu, r, alpha, x0, tol=1e-300, check_every=5, max_iter=1)
    t1 = time.perf_counter()
    per_first = t1 - t0
    k = max(5, min(2000, int(budget_s / max(per_first / 2.0, 1e-3))))
    t0 = time.perf_counter()
    onpga.npga(model, mu, r, alpha, x0, tol=1e-300, check_every=5, max_iter=k)
    dt = time.perf_counter() - t0
    # npga(max_iter=k) evaluates k step gradients + (k // 5 + 1) check gradients
    per_grad = dt / (k + k // 5 + 1)
    return {
        "value": per_grad * gpu_grad_evals,
        "unit": "s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": (f"{k} iterations of the float64 oracle Algorithm 1 on the full "
                   f"n={n}, T={L.shape[1]} factor ({dt:.1f} s, {per_grad * 1e3:.1f} ms per "
                   f"gradient), scaled to the {gpu_grad_evals} gradient evaluations the GPU "
                   f"needed to reach residual 1e-6"),
    }


def adjoint_section(npga, gen, torch, dev, spec, R, x, r):
    """npga_backward at the C2 solution with l(w) = w^T Sigma_test w -
    mu_test^T w: float64 face gradient, projected CG, dl/dmu and the n x T
    dl/dL (a 1.05 GB write)."""
    Rtest = torch.from_numpy(gen.heldout_returns_TxN(spec, 5000, gen.factor_model.HELDOUT_SEED_C5)).to(dev)
    Lt, mut = npga.build_factor(Rtest)
    del Rtest
    xd = x.to(torch.float64)
    Ltd = Lt.to(torch.float64)
    g = (2.0 * (Ltd.T @ (Ltd @ xd)) - mut).to(torch.float32)
    del Ltd, Lt
    L, mu = npga.build_factor(R)
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dmu, dL, info = npga.backward(L, mu, r, x, g)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    n, T = spec.n, spec.T
    return {"workload": "dl/dmu and dl/dL at the n=5440, T=48374 solution; held-out loss (5000 periods, seed 105)",
            "backward_ms": times[-1], "cg_iters": info["cg_iters"], "support": info["support"],
            "return_active": info["return_active"], "residual": info["residual"],
            "dl_dL_write_GB": 4.0 * n * T / 1e9, "status": info["status_name"]}


def frontier_section(npga, gen, torch, dev, n_seq):
    """Efficient frontier at n = 2000, T = 20000 (5 factors, seed 4): m = 128
    targets r_j = r_mv + j (0.95 max mu - r_mv)/127, all solved by one batched
    call; frontier solves/s = m / GPU time until the last target's stopping
    test passed.  r_mv comes from a GPU solve with a slack return target."""
    spec = gen.SPECS["c4"]
    Rt = gen.returns_TxN(spec)
    R4 = torch.from_numpy(Rt).to(dev)
    del Rt
    L4, mu4 = npga.build_factor(R4)
    del R4
    mu_h = mu4.cpu().numpy()
    x_mv, _ = npga.solve(L4, mu4, float(mu_h.min()) - 1.0)
    r_mv = float(mu_h @ x_mv.cpu().numpy().astype("float64"))
    rs = gen.frontier_targets_from_mv(r_mv, float(mu_h.max()), 128)
    n, T, m = spec.n, spec.T, len(rs)
    flops = 4.0 * n * T * m            # U = L^T X and G = L U: 2 n T m each
    sec = {"workload": "frontier n=2000, T=20000, m=128 targets (seed 4)", "m": m}
    for name, Lx in (("f32", L4), ("bf16", npga.to_bf16(L4))):
        best, cfg_ms = npga.batched_tune(Lx, m)
        runs = []
        for _ in range(2):
            X, infos = npga.solve_batched(Lx, mu4, rs, batch_config=best)
            runs.append(infos)
        infos = runs[-1]
        t_all = max(i["time_to_tol_ms"] for i in infos) / 1e3
        gemm_ms = infos[0]["sweep_ms"]
        sec[name] = {
            "frontier_solves_per_s": m / t_all,
            "time_to_tol_all_s": t_all,
            "solve_ms_incl_refinement": infos[0]["time_ms"],
            "setup_ms": infos[0]["setup_ms"],
            "iters_max": max(i["iters"] for i in infos),
            "iters_median": sorted(i["iters"] for i in infos)[m // 2],
            "refine_iters_max": max(i["refine_iters"] for i in infos),
            "all_ok": all(i["status"] == 0 for i in infos),
            "all_refined": all(i["refined"] == 1 for i in infos),
            "config": best,
            "config_ms": cfg_ms,
            "gemm_pair_ms": gemm_ms,
            "gemm_TFLOPs": flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms else None,
            "objectives_nondecreasing": all(infos[j + 1]["objective"] >= infos[j]["objective"] * (1 - 1e-6)
                                            for j in range(m - 1)),
        }
    # adaptive momentum restart (an option; Algorithm 1 itself has none)
    best16 = sec["bf16"]["config"]
    Lb16 = npga.to_bf16(L4)
    npga.solve_batched(Lb16, mu4, rs, batch_config=best16, restart=True)
    _, inf_r = npga.solve_batched(Lb16, mu4, rs, batch_config=best16, restart=True)
    t_r = max(i["time_to_tol_ms"] for i in inf_r) / 1e3
    sec["bf16_restart"] = {"frontier_solves_per_s": m / t_r, "time_to_tol_all_s": t_r,
                           "iters_max": max(i["iters"] for i in inf_r),
                           "iters_median": sorted(i["iters"] for i in inf_r)[m // 2],
                           "all_ok": all(i["status"] == 0 for i in inf_r)}
    del Lb16
    # the same targets one solve at a time (a sample, scaled to m)
    seq = []
    idx = [int(round(v)) for v in (i * (m - 1) / max(n_seq - 1, 1) for i in range(n_seq))]
    for j in idx:
        npga.solve(L4, mu4, float(rs[j]))
        _, inf1 = npga.solve(L4, mu4, float(rs[j]))
        seq.append(inf1["time_to_tol_ms"] / 1e3)
    t_seq = sum(seq) / len(seq) * m
    sec["one_at_a_time"] = {"targets_timed": idx, "time_to_tol_s_mean": sum(seq) / len(seq),
                            "frontier_solves_per_s": m / t_seq}
    sec["speedup_batched_f32_vs_one_at_a_time"] = sec["f32"]["frontier_solves_per_s"] / (m / t_seq)
    return sec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    import paper_2604_02917_amd as npga

    spec = gen.SPECS["c2"]
    t_gen = time.perf_counter()
    Rt = gen.returns_TxN(spec)
    r = gen.target_return(spec, Rt)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    R = torch.from_numpy(Rt).to(dev)
    torch.cuda.synchronize()
    n, T = spec.n, spec.T

    if args.copy_probe_gb > 0:
        nel = int(args.copy_probe_gb * 1e9) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        L, mu = npga.build_factor(R)
        x, info = npga.solve(L, mu, r, path=args.path)
        return x, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3

    tol_s = statistics.median(i["time_to_tol_ms"] for i in infos) / 1e3
    solve_ms = statistics.median(i["time_ms"] for i in infos)
    sweep_ms = statistics.median(i["sweep_ms"] for i in infos)
    last = infos[-1]
    bytes_per_launch = 4.0 * n * (T if last["path_used"] == 1 else n)
    achieved = bytes_per_launch / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    iters = last["iters"]
    # gradient evaluations to the stopping point: step-size estimate + iterations 0..iters
    grad_evals = last["step_sweeps"] + iters + 1

    xh = x.cpu().numpy().astype(np.float64)
    feas = {
        "min_x": float(xh.min()),
        "budget_err": float(abs(xh.sum() - 1.0)),
    }
    out = {
        "metric": "time-to-1e-6 (s) at n=5440,T=48374",
        "value": tol_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "full model n=5440, T=48374: 10-factor returns with Student-t(4) noise, "
                        "r = 60th percentile of mu (seed 2)",
            "n": n, "T": T, "path": "gemv" if last["path_used"] == 1 else "syrk", "tol": 1e-6,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": sweep_traffic(last["path_used"]),
            "kernel": "k_sweep (fused L^T x and L u, one read of L)" if last["path_used"] == 1
                      else "k_symv_tail",
            "bytes_per_launch": bytes_per_launch,
            "launch_ms": sweep_ms,
        },
        "solve": {
            "iters_to_tol": iters,
            "refine_iters": last["refine_iters"],
            "residual_at_stop": last["residual"],
            "final_residual": last["final_residual"],
            "objective": last["objective"],
            "support": last["support"],
            "return_active": last["return_active"],
            "solve_ms_incl_refinement": solve_ms,
            "setup_ms": last["setup_ms"],
            "step_estimate_sweeps": last["step_sweeps"],
            "ms_per_iteration": (tol_s * 1e3 - last["setup_ms"]) / max(iters, 1),
            "status": last["status_name"],
            "feasibility": feas,
        },
        "generator_s": t_gen,
    }
    # Algorithm 1 with the adaptive momentum restart option (not the paper's
    # default; reported beside the timed path)
    if not args.no_restart_compare:
        L, mu = npga.build_factor(R)
        npga.solve(L, mu, r, restart=True)
        _, info_r = npga.solve(L, mu, r, restart=True)
        out["restart_variant"] = {"time_to_tol_s": info_r["time_to_tol_ms"] / 1e3, "iters_to_tol": info_r["iters"],
                                  "objective": info_r["objective"], "status": info_r["status_name"]}
    # the covariance path (Sigma = L L^T by MFMA, then a SYMV per iteration),
    # reported beside the timed path; not part of the timed steps
    if args.path == "gemv" and not args.no_syrk_compare:
        L, mu = npga.build_factor(R)
        sy = []
        for _ in range(2):
            _, info_s = npga.solve(L, mu, r, path="syrk")
            sy.append(info_s)
        s_last = sy[-1]
        out["syrk_path"] = {
            "time_to_tol_s": s_last["time_to_tol_ms"] / 1e3,
            "solve_ms_incl_refinement": s_last["time_ms"],
            "setup_ms_incl_syrk": s_last["setup_ms"],
            "iters_to_tol": s_last["iters"],
            "refine_iters": s_last["refine_iters"],
            "symv_ms": s_last["sweep_ms"],
            "symv_effective_GBs": 4.0 * n * n / (s_last["sweep_ms"] * 1e-3) / 1e9 if s_last["sweep_ms"] else None,
            "objective": s_last["objective"],
            "status": s_last["status_name"],
        }
    # bfloat16 storage of L (float32 accumulation): the same solve reading
    # half the bytes; quantisation gap measured in the float32 model
    if not args.no_bf16:
        L, mu = npga.build_factor(R)
        Lb = npga.to_bf16(L)
        bi = []
        for _ in range(2):
            xb, info_b = npga.solve(Lb, mu, r)
            bi.append(info_b)
        b_last = bi[-1]
        _, f32_at_b = npga.gradient(L, xb, 0.0)
        out["bf16_path"] = {
            "time_to_tol_s": b_last["time_to_tol_ms"] / 1e3,
            "solve_ms_incl_refinement": b_last["time_ms"],
            "iters_to_tol": b_last["iters"],
            "refine_iters": b_last["refine_iters"],
            "sweep_ms": b_last["sweep_ms"],
            "sweep_GBs": 2.0 * n * T / (b_last["sweep_ms"] * 1e-3) / 1e9 if b_last["sweep_ms"] else None,
            "objective_bf16_model": b_last["objective"],
            "quantisation_gap_vs_f32_model": max(f32_at_b - last["objective"], 0.0) / last["objective"],
            "max_abs_x_diff_vs_f32": float((xb - x).abs().max().item()),
            "status": b_last["status_name"],
        }
        del Lb
    # Sketch-truncate-ridge workload (k = 4096, ell = 512, gamma = 1e-4 tr(YY^T)/n):
    # build time, STR solve and the full-model gap of Sec. 5.1, beside the timed path
    if not args.no_str:
        from gen.factor_model import SKETCH_SEED_C3
        S = gen.gaussian_sketch(T, 4096, seed=SKETCH_SEED_C3)
        Sd = torch.from_numpy(S).to(dev)
        del S
        L, mu = npga.build_factor(R)
        builds = []
        for _ in range(2):
            torch.cuda.synchronize()
            tb = time.perf_counter()
            Leff, sigma, gamma = npga.sketch_str(L, Sd, 512, ridge_coef=1e-4)
            torch.cuda.synchronize()
            builds.append((time.perf_counter() - tb) * 1e3)
        del Sd
        xs_, info_str = npga.solve(Leff, mu, r, gamma=gamma)
        _, f_full_str = npga.gradient(L, xs_, 0.0)
        f_full = last["objective"]
        # the same build with S drawn on the device (Philox), and with a
        # CountSketch (k = 4096 buckets, draws seed 3)
        variants = {}
        hc, sc = gen.countsketch(T, 4096, 3)
        hcd, scd = torch.from_numpy(hc).to(dev), torch.from_numpy(sc).to(dev)
        for name, kw in (("philox_gaussian", dict(sketch="gaussian", seed=3)),
                         ("countsketch", dict(sketch="count", h=hcd, sgn=scd))):
            tv = []
            for _ in range(2):
                torch.cuda.synchronize()
                tb = time.perf_counter()
                Le_v, sig_v, g_v, _ = npga.sketch_str_ex(L, 4096, 512, ridge_coef=1e-4, **kw)
                torch.cuda.synchronize()
                tv.append((time.perf_counter() - tb) * 1e3)
            xv, inf_v = npga.solve(Le_v, mu, r, gamma=g_v)
            _, f_full_v = npga.gradient(L, xv, 0.0)
            variants[name] = {"build_ms": tv[-1], "time_to_tol_s": inf_v["time_to_tol_ms"] / 1e3,
                              "sigma_1": float(sig_v[0].item()),
                              "full_model_gap": max(f_full_v - last["objective"], 0.0) / max(abs(last["objective"]), 1e-12),
                              "status": inf_v["status_name"]}
            del Le_v
        out["str"] = {
            "variants": variants,
            "workload": "c2 factor, Gaussian sketch k=4096 (seed 3), ell=512, gamma=1e-4 tr(YY^T)/n",
            "build_ms": builds[-1],
            "time_to_tol_s": info_str["time_to_tol_ms"] / 1e3,
            "solve_ms_incl_refinement": info_str["time_ms"],
            "iters_to_tol": info_str["iters"],
            "refine_iters": info_str["refine_iters"],
            "sweep_ms": info_str["sweep_ms"],
            "gamma": gamma,
            "sigma_1": float(sigma[0].item()),
            "sigma_512": float(sigma[-1].item()),
            "objective_str": info_str["objective"],
            "full_model_gap": max(f_full_str - f_full, 0.0) / max(abs(f_full), 1e-12),
            "status": info_str["status_name"],
        }
    # adjoint of the solution map at the benchmark's solution: out-of-sample
    # loss on a held-out block (5000 periods, seed 105), dl/dmu and dl/dL
    if not args.no_adjoint:
        out["adjoint"] = adjoint_section(npga, gen, torch, dev, spec, R, x, r)
    if not args.no_frontier:
        out["frontier"] = frontier_section(npga, gen, torch, dev, args.frontier_seq)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Rt, r, grad_evals, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

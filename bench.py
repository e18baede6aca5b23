"""Benchmark: iterative Vecchia-Laplace inference on one MI355X.

One step = one full pass of the hot path over the n = 100,000 workload
(Matern-3/2 range 0.05, m = 20, Bernoulli-logit, 50 Rademacher probes, CG
tolerance 1e-3, predictions at 10,000 test locations with s = 2000 simulated
samples), inputs resident in HBM before the timed region:
  vl_build_vecchia  neighbour search + Vecchia factor (with derivatives)
  vl_find_mode      Newton mode finding with VADU-preconditioned CG
  vl_neg_log_marglik SLQ negative log-marginal likelihood + STE gradient
  vl_predict        predictive means and simulated variances
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Laplace marginal-likelihood evals/s at n=1e5,m=20; B-SpMM HBM GB/s; p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KINDS = ("spmm_b", "spmm_bt", "trsm_lower", "trsm_upper", "dense_lower", "dense_upper",
         "level_lower", "level_upper", "level_upper_split", "level_upper_fold", "dense_wide")
KERNEL_NAMES = {"spmm_b": "spmm_ell_kernel", "spmm_bt": "spmm_csr_t_kernel",
                "trsm_lower": "trsm_kernel<lower>", "trsm_upper": "trsm_kernel<upper>",
                "dense_lower": "dense_part_kernel", "dense_upper": "dense_fold_kernel",
                "level_lower": "trsm_level_lower_kernel",
                "level_upper": "trsm_level_upper_kernel",
                "level_upper_split": "trsm_level_split_kernel",
                "level_upper_fold": "trsm_fold_kernel", "dense_wide": "dense_gemm_kernel"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2_n1e5.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2_n1e5")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--forms", default="all",
                    help="comma-separated forms to run after the timed steps (default all)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision, batching and serving measurements")
    ap.add_argument("--batch-problems", type=int, default=32)
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="one 512 MiB device-to-device copy before the steps (the known-size "
                         "kernel that scales the HBM byte counters)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2310_12000_amd as P
    import synth

    P.lib()
    w = synth.make(args.workload, seed=args.seed)
    d = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    coords, y, F = d(w["coords"]), d(w["y"]), d(w["F"])
    coords_p, Fp = d(w["coords_pred"]), d(w["Fp"])
    opts = P.vl_default_opts(cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"],
                             num_probes=w["t"], num_pred_samples=w["s"], seed=args.seed)
    theta = (w["sigma2"], w["rho"])
    torch.cuda.synchronize()

    ktime = {k: [0.0, 0, 0.0] for k in KINDS}
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    timed_kinds = [None]  # kernel classes recorded in the timed steps (None = all)

    def step(rec, timed=False):
        t0 = time.perf_counter()
        g = P.VecchiaLaplace(coords, w["m"], w["kind"], theta, want_deriv=True)
        if timed:
            P.vl_timing_enable(g.h, True, timed_kinds[0])
        t1 = time.perf_counter()
        mode, st = g.find_mode(y, F, w["lik"], None, opts)
        t2 = time.perf_counter()
        nll, grad, nst = g.neg_log_marglik(opts, want_grad=True)
        t3 = time.perf_counter()
        mean, var, pst = g.predict(coords_p, Fp, opts)
        t4 = time.perf_counter()
        rec.append({"build_ms": 1e3 * (t1 - t0), "mode_ms": 1e3 * (t2 - t1),
                    "nll_grad_ms": 1e3 * (t3 - t2), "predict_ms": 1e3 * (t4 - t3),
                    "newton_iters": st.newton_iters, "newton_cg_total": st.cg_iters_total,
                    "slq_cg_max": nst.cg_iters_max, "pred_cg_max": pst.cg_iters_max,
                    "nll": nll, "grad": grad})
        if timed:
            for k in (KINDS if timed_kinds[0] is None else timed_kinds[0]):
                ms, cnt, by = P.vl_timing_read(g.h, k)
                ktime[k][0] += ms
                ktime[k][1] += cnt
                ktime[k][2] += by
        g.close()

    # The warm-up steps time every class once; the timed steps record events
    # around the launches of the dominant class only (events around every
    # launch would slow the step itself).
    warm = []
    for k in range(args.warmup):
        step(warm, timed=(k == args.warmup - 1))
        log(args, f"warmup {k}: {warm[-1]}")
    if args.warmup > 0:
        dom_w = max(KINDS, key=lambda k: ktime[k][0])
        out_warm = {k: ktime[k][0] for k in KINDS}
        warm_k = {k: list(ktime[k]) for k in KINDS}
        for k in KINDS:
            ktime[k] = [0.0, 0, 0.0]
        timed_kinds[0] = [dom_w]
    else:
        out_warm = None
        warm_k = None
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(rec, timed=True)
        log(args, f"step {k}: {rec[-1]}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    phases = {k: sum(r[k] for r in rec) / len(rec)
              for k in ("build_ms", "mode_ms", "nll_grad_ms", "predict_ms")}
    out = {
        "metric": METRIC, "value": args.steps / elapsed, "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={w['n']}, m={w['m']}, Matern-3/2 "
                   f"rho={w['rho']}, Bernoulli-logit, t={w['t']} probes, CG tol {w['cg_tol']}, "
                   f"{w['n_pred']} test points, s={w['s']}; one eval = build + mode + "
                   "SLQ NLL + gradient + predict",
                   "n": w["n"], "m": w["m"], "probes": w["t"], "n_pred": w["n_pred"],
                   "pred_samples": w["s"]},
        "phases_ms": phases,
        "iterations": {k: rec[-1][k] for k in ("newton_iters", "newton_cg_total", "slq_cg_max",
                                               "pred_cg_max")},
        "nll": rec[-1]["nll"],
    }
    # dominant kernel class by time; achieved = algorithmic bytes / kernel time
    dom = max(KINDS, key=lambda k: ktime[k][0])
    ms_d, cnt_d, by_d = ktime[dom]
    ach = by_d / (ms_d * 1e-3) / 1e9 if ms_d > 0 else 0.0
    out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS,
                       "traffic": measured_traffic(KERNEL_NAMES[dom], args.workload),
                       "kernel": KERNEL_NAMES[dom], "launches": cnt_d,
                       "avg_launch_us": 1e3 * ms_d / max(cnt_d, 1),
                       "alg_bytes_per_launch": by_d / max(cnt_d, 1)}
    out["kernel_time_ms"] = out_warm if out_warm is not None else \
        {k: ktime[k][0] / args.steps for k in KINDS}
    # B-SpMM (all block widths of the step), from the step that timed every class
    ms_b, cnt_b, by_b = (warm_k or ktime)["spmm_b"]
    out["b_spmm"] = {"achieved_GBps": by_b / (ms_b * 1e-3) / 1e9 if ms_b > 0 else 0.0,
                     "frac": (by_b / (ms_b * 1e-3) / 1e9) / HBM_PEAK_GBS if ms_b > 0 else 0.0,
                     "launches": cnt_b, "avg_launch_us": 1e3 * ms_b / max(cnt_b, 1)}
    # The likelihood evaluation alone, as an estimation loop calls it: new
    # theta on a built model (factor only; neighbours and schedules kept),
    # mode from zero, SLQ NLL.
    g = P.VecchiaLaplace(coords, w["m"], w["kind"], theta)
    g.set_theta(theta)
    g.find_mode(y, F, w["lik"], None, opts)
    g.neg_log_marglik(opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        g.set_theta(theta)
        g.find_mode(y, F, w["lik"], None, opts)
        g.neg_log_marglik(opts)
    torch.cuda.synchronize()
    out["nll_evals_per_s"] = {"value": 3 / (time.perf_counter() - t0),
                              "what": "vl_set_theta + vl_find_mode + vl_neg_log_marglik "
                                      "(no gradient, no prediction) on a built model"}
    g.close()
    log(args, f"nll-only evals/s: {out['nll_evals_per_s']['value']:.3f}")
    if not args.no_forms:
        out["forms"] = {}
        for name, fn in (("mixed", lambda: form_mixed(P, torch, w, coords, y, F, coords_p, Fp,
                                                       theta, opts, args)),
                         ("mixed_c3_shape", lambda: form_mixed_c3(P, torch, synth, args)),
                         ("preconditioners", lambda: form_preconditioners(
                             P, torch, w, coords, y, F, theta, opts, args)),
                         ("pred_variance_methods",
                          lambda: form_pred_variance_methods(P, torch, synth, args)),
                         ("batch", lambda: form_batch(P, torch, synth, args)),
                         ("serving", lambda: form_serving(P, torch, synth, args))):
            if args.forms != "all" and name not in args.forms.split(","):
                continue
            print(f"form: {name}", file=sys.stderr, flush=True)
            out["forms"][name] = fn()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, rec[-1], args)
        out["small_workload_timed"] = small_workload_both_sides(P, torch, synth, args)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def form_mixed(P, torch, w, coords, y, F, coords_p, Fp, theta, opts, args, grad=True):
    """The same evaluation in the mixed form (FP32 preconditioner solves with
    FP64 sums inside the FP64 PCG, for blocks wider than 64 columns: the
    prediction's sample block), against the FP64 run of the same inputs and
    probes; per-phase times of both."""
    import copy
    om = copy.copy(opts)
    om.precision = P.VL_MIXED
    res = {}
    for name, o in (("fp64", opts), ("mixed", om)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = P.VecchiaLaplace(coords, w["m"], w["kind"], theta, want_deriv=grad)
        g.find_mode(y, F, w["lik"], None, o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nll, gr, _ = g.neg_log_marglik(o, want_grad=grad)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        mean, var, _ = g.predict(coords_p, Fp, o)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        res[name] = (t3 - t0, nll, gr, mean.cpu().numpy(), var.cpu().numpy(),
                     {"build_mode_s": t1 - t0, "nll_s": t2 - t1, "predict_s": t3 - t2})
        g.close()
    import numpy as np
    f, m = res["fp64"], res["mixed"]
    rel = lambda a, b: float(np.max(np.abs(np.asarray(a) - np.asarray(b))) /
                             max(np.max(np.abs(np.asarray(b))), 1e-300))
    log(args, f"mixed: {m[0]:.2f} s vs fp64 {f[0]:.2f} s")
    out = {"evals_per_s": 1.0 / m[0], "fp64_evals_per_s": 1.0 / f[0],
           "speedup": f[0] / m[0], "phases_s": {"fp64": f[5], "mixed": m[5]},
           "nll_rel_err_vs_fp64": abs(m[1] - f[1]) / abs(f[1]),
           "var_rel_err_vs_fp64": rel(m[4], f[4]), "mean_rel_err_vs_fp64": rel(m[3], f[3])}
    if grad:
        out["grad_rel_err_vs_fp64"] = rel(m[2], f[2])
    return out


def form_mixed_c3(P, torch, synth, args):
    """The mixed form on the shape of the n = 2e6 precision workload (Matern-3/2
    range 0.02, m = 20, Poisson with offset 1, 64 probes, CG tolerance 1e-2,
    10,000 test points, s = 256) at n = 2e5, the largest size this library
    runs."""
    w = synth.make("c3_n2e6", seed=args.seed, n=200000)
    d = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    opts = P.vl_default_opts(cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"],
                             num_probes=w["t"], num_pred_samples=w["s"], seed=args.seed)
    out = form_mixed(P, torch, w, d(w["coords"]), d(w["y"]), d(w["F"]), d(w["coords_pred"]),
                     d(w["Fp"]), (w["sigma2"], w["rho"]), opts, args, grad=False)
    out["workload"] = ("n=200000 (the 2e6 workload's shape), Matern-3/2 rho=0.02, m=20, Poisson "
                       "with offset 1, t=64, CG tol 1e-2, 10000 test points, s=256; one eval = "
                       "build + mode + NLL + predict")
    return out


def form_preconditioners(P, torch, w, coords, y, F, theta, opts, args):
    """The likelihood evaluation (set theta, mode from zero, SLQ NLL) with
    each preconditioner on the same workload and probes: time, CG
    iterations, and the probe standard error of the log-determinant estimate
    (sample sd of r0^T z0 e_1^T log(T) e_1 over the t probes / sqrt t), the
    variance the preconditioners of Sec. 3.1 are compared on."""
    import copy
    import numpy as np
    res = {}
    for name, pc in (("VADU", P.VL_PREC_VADU), ("LVA", P.VL_PREC_LVA), ("LRAC", P.VL_PREC_LRAC),
                     ("P1", P.VL_PREC_DIAG)):
        o = copy.copy(opts)
        o.precond = pc
        g = P.VecchiaLaplace(coords, w["m"], w["kind"], theta, want_deriv=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.set_theta(theta)
        _, st = g.find_mode(y, F, w["lik"], None, o, allow_no_conv=True)
        t1 = time.perf_counter()
        nll, _, nst = g.neg_log_marglik(o, allow_no_conv=True)
        t2 = time.perf_counter()
        terms = g.export("slq_r0z0").cpu().numpy() * g.export("slq_quad").cpu().numpy()
        res[name] = {"mode_ms": 1e3 * (t1 - t0), "nll_ms": 1e3 * (t2 - t1), "nll": nll,
                     "newton_cg_total": st.cg_iters_total, "slq_cg_max": nst.cg_iters_max,
                     "hit_cap": bool(nst.cg_iters_max >= o.max_cg or st.hit_cap),
                     "logdet_probe_se": float(np.std(terms, ddof=1) / np.sqrt(len(terms)))}
        if pc in (P.VL_PREC_VADU, P.VL_PREC_LRAC):  # the STE formulas the paper gives
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            _, grad, _ = g.neg_log_marglik(o, want_grad=True, allow_no_conv=True)
            res[name]["nll_grad_ms"] = 1e3 * (time.perf_counter() - t3)
            res[name]["grad"] = grad
        g.close()
        log(args, f"preconditioner {name}: {res[name]}")
    return res


def form_pred_variance_methods(P, torch, synth, args):
    """Simulated (Alg. simAlgo) versus preconditioned-Lanczos (Sec. 3.3.2)
    predictive variances at n = n_p = 5,000 (Matern-3/2 range 0.05, m = 20,
    Bernoulli-logit): time on the GPU and the relative RMSE and largest
    relative error against the exact variances D_p + diag(A_p A^{-1} A_p^T),
    computed densely on the host from the device's own factor, mode and
    prediction rows (so that only the variance method differs)."""
    import copy
    import numpy as np
    w = synth.make("c2_n1e5", seed=args.seed, n=5000, n_pred=5000)
    d = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    coords, y, F, cp, Fp = (d(w["coords"]), d(w["y"]), d(w["F"]), d(w["coords_pred"]),
                            d(w["Fp"]))
    base = P.vl_default_opts(cg_tol=1e-8, pred_cg_tol=1e-3, seed=args.seed)
    g = P.VecchiaLaplace(coords, w["m"], w["kind"], (w["sigma2"], w["rho"]))
    g.find_mode(y, F, w["lik"], None, base)
    g.predict(cp, Fp, base, want_var=False)
    h = lambda name: g.export(name).cpu().numpy()
    n, m, npred = w["n"], w["m"], w["n_pred"]
    nbr, bval, D, W = h("nbr").reshape(n, m), h("bval").reshape(n, m), h("D"), h("W")
    pnbr, pval, Dp = h("pred_nbr").reshape(npred, m), h("pred_bval").reshape(npred, m), h("pred_D")
    # dense exact reference: A = W + B^T D^{-1} B, B = I - (A_i entries) in ELL
    B = np.eye(n)
    Ap = np.zeros((npred, n))
    for i in range(n):
        ok = nbr[i] >= 0
        B[i, nbr[i][ok]] = bval[i][ok]
    for j in range(npred):
        ok = pnbr[j] >= 0
        Ap[j, pnbr[j][ok]] = pval[j][ok]
    A = np.diag(W) + B.T @ (B / D[:, None])
    exact = Dp + np.einsum("pi,pi->p", Ap, np.linalg.solve(A, Ap.T).T)
    res = {"workload": "n=n_p=5000, Matern-3/2 rho=0.05, m=20, Bernoulli-logit; simulation "
                       "CG tol 1e-3", "methods": {}}

    def run(label, o):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, var, _ = g.predict(cp, Fp, o, allow_no_conv=True)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        v = var.cpu().numpy()
        rel = (v - exact) / exact
        res["methods"][label] = {"ms": ms, "rel_rmse": float(np.sqrt(np.mean(rel ** 2))),
                                 "max_rel_err": float(np.max(np.abs(rel))),
                                 "mean_rel_bias": float(np.mean(rel))}
        log(args, f"variance method {label}: {res['methods'][label]}")

    for s in (100, 500, 2000):
        o = copy.copy(base)
        o.num_pred_samples = s
        run(f"simulation s={s}", o)
    for method, tag in ((P.VL_PRED_LANCZOS_L1, "L1"), (P.VL_PRED_LANCZOS_L2, "L2")):
        for k in (50, 200, 500):
            o = copy.copy(base)
            o.pred_method = method
            o.lanczos_rank = k
            run(f"lanczos P_{tag} k={k}", o)
    g.close()
    return res


def form_batch(P, torch, synth, args):
    """Uneven problems (n log-uniform, m in {10, 20, 30}, exponential or
    Matern-3/2, range U(0.02, 0.2), Bernoulli-logit, 32 probes) fitted
    together, against solo runs of a sample of them.  The library's batch
    limit (32 problems, 65536 rows) caps the sizes at n in [1e3, 2e3]."""
    probs = synth.batch_problems(count=args.batch_problems, seed=args.seed, n_lo=1000,
                                 n_hi=2000)
    o = P.vl_default_opts(num_probes=32, cg_tol=1e-2)
    items = [dict(coords=p["coords"], y=p["y"], F=p["F"], m=p["m"], cov=p["kind"],
                  theta=(p["sigma2"], p["rho"]), seed=1000 + k) for k, p in enumerate(probs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = P.VecchiaLaplaceBatch(items)
    t1 = time.perf_counter()
    nll = b.fit(o)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    paths = [b.tuned_path(c) for c in range(2)]
    b.close()
    # solo runs of every 4th problem, scaled to all problems by their sizes
    sample = list(range(0, len(probs), 4))
    ts = 0.0
    for k in sample:
        p = probs[k]
        o.seed = 1000 + k
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        g = P.VecchiaLaplace(torch.as_tensor(p["coords"], device="cuda"), p["m"], p["kind"],
                             (p["sigma2"], p["rho"]))
        g.find_mode(torch.as_tensor(p["y"], device="cuda"), torch.as_tensor(p["F"], device="cuda"),
                    p["lik"], None, o)
        g.neg_log_marglik(o)
        torch.cuda.synchronize()
        ts += time.perf_counter() - s0
        g.close()
    n_all = sum(p["n"] for p in probs)
    n_s = sum(probs[k]["n"] for k in sample)
    solo_est = ts * n_all / n_s
    log(args, f"batch: build {t1 - t0:.2f} s fit {t2 - t1:.2f} s; solo estimate {solo_est:.2f} s")
    return {"problems": len(probs), "total_n": n_all, "build_s": t1 - t0, "fit_s": t2 - t1,
            "problems_per_s": len(probs) / (t2 - t0),
            "solo_estimate_s": solo_est, "speedup_vs_solo": solo_est / (t2 - t0),
            "solo_sample": len(sample), "autotuned_paths": {"t=1": paths[0], "t=32": paths[1]},
            "all_finite": bool(all(map(lambda v: v == v, nll)))}


def form_serving(P, torch, synth, args):
    """Fit + predict requests arriving as a Poisson process at 100 req/s (n
    log-uniform in [2e3, 2e5], 1e3..2e4 test points, m = 20, Bernoulli or
    Poisson), served by the continuous-batching loop with 4 slots under a
    200 GB HBM budget; t = 50 probes, s = 2000 samples in tiles of 500."""
    import numpy as np
    reqs = synth.serving_requests(args.serve_requests, seed=args.seed)
    o = P.vl_default_opts(num_probes=50, num_pred_samples=2000, pred_tile=500, cg_tol=1e-2,
                          pred_cg_tol=1e-3)
    srv = P.Server(4, 200e9, o)
    items = [dict(coords=r["coords"], y=r["y"], F=r["F"], m=r["m"], cov=r["kind"],
                  theta=(r["sigma2"], r["rho"]), lik=r["lik"], seed=500 + k,
                  coords_p=r["coords_pred"], Fp=r["Fp"]) for k, r in enumerate(reqs)]
    t0 = time.perf_counter()
    tickets = []
    for r, it in zip(reqs, items):
        delay = r["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(it))
    lat = []
    for tk in tickets:
        nll, mean, var, st, qms = srv.wait(tk)
        lat.append(st["t_ms"])
    wall = time.perf_counter() - t0
    peak_bytes, peak_running = srv.info()
    srv.close()
    lat = np.array(lat)
    log(args, f"serving: {len(reqs)} requests in {wall:.2f} s; p50 {np.percentile(lat, 50):.0f} ms "
              f"p99 {np.percentile(lat, 99):.0f} ms")
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "req_per_s": len(reqs) / wall,
            "slots": 4, "hbm_budget_gb": 200, "peak_running": peak_running,
            "peak_admitted_gb": peak_bytes / 1e9,
            "n_range": [int(min(r["n"] for r in reqs)), int(max(r["n"] for r in reqs))]}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed PMC summary (FETCH_SIZE
    + WRITE_SIZE, scaled by the same counters on a copy of known size), or None
    when no summary covers this kernel and workload."""
    if workload != "c2_n1e5" or not os.path.exists(TRAFFIC_FILE):
        return None
    import re
    pat = re.compile(r"^- (\S+): ([0-9.eE+-]+) bytes per launch")
    with open(TRAFFIC_FILE) as f:
        for line in f:
            mm = pat.match(line.strip())
            if mm and mm.group(1) == kernel:
                return float(mm.group(2))
    return None


def cpu_baseline(w, it, args):
    """The FP64 oracle timed on a bounded sample of the same workload.

    Every piece is an oracle call timed end to end on the full n = 1e5 data:
    the model (neighbour search + Vecchia factor with derivatives), the first
    Newton step (its whole CG solve), the SLQ likelihood with its gradient on
    2 of the t probe columns, and the prediction (test-point factor, means and
    2 of the s sample columns).  One evaluation is then: build + Newton steps
    x the device's Newton count + likelihood x t/2 + prediction x s/2 (probe
    and sample columns are independent CG runs of the same operator)."""
    from threadpoolctl import threadpool_info

    from oracle import laplace as OL

    y, F, lik = w["y"], w["F"], w["lik"]
    t0 = time.perf_counter()
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]), deriv=True)
    t_build = time.perf_counter() - t0
    o = OL.Opts(cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"], num_probes=2,
                num_pred_samples=2, seed=args.seed, max_newton=1)
    t0 = time.perf_counter()
    b, W, st = OL.find_mode(model, y, F, lik, None, o)
    t_newton = time.perf_counter() - t0
    t0 = time.perf_counter()
    OL.neg_log_marglik(model, y, F, lik, None, b, o, want_grad=True)
    t_nll2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    OL.predict(model, w["coords_pred"], w["Fp"], b, W, o)
    t_pred2 = time.perf_counter() - t0
    k_newton = max(it["newton_iters"], 1)
    t_eval = (t_build + k_newton * t_newton + t_nll2 * w["t"] / 2 + t_pred2 * w["s"] / 2)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {"value": 1.0 / t_eval, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle calls timed end to end on the same n={w['n']} workload: build "
                       f"{t_build:.1f} s, first Newton step {t_newton:.1f} s "
                       f"({st['cg_iters'][0]} CG iterations) x {k_newton} steps, SLQ likelihood "
                       f"+ gradient on 2 probes {t_nll2:.1f} s x {w['t']}/2, prediction with 2 "
                       f"samples {t_pred2:.1f} s x {w['s']}/2"),
            "est_eval_s": t_eval, "timed_s": t_build + t_newton + t_nll2 + t_pred2,
            "host_cpus": os.cpu_count()}


def small_workload_both_sides(P, torch, synth, args):
    """The n = 2,000 workload (exponential range 0.1, m = 10, Bernoulli-logit,
    t = 50, CG tolerance 1e-8, 500 test points, s = 64), where the oracle
    finishes in seconds: one whole evaluation (build + mode + NLL + gradient
    + predict) timed on both sides, the oracle replaying nothing."""
    from threadpoolctl import threadpool_info

    from oracle import laplace as OL

    w = synth.make("c1_n2000", seed=args.seed)
    d = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    coords, y, F, cp, Fp = d(w["coords"]), d(w["y"]), d(w["F"]), d(w["coords_pred"]), d(w["Fp"])
    opts = P.vl_default_opts(cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"],
                             num_probes=w["t"], num_pred_samples=w["s"], seed=args.seed)

    def gpu_eval():
        g = P.VecchiaLaplace(coords, w["m"], w["kind"], (w["sigma2"], w["rho"]), want_deriv=True)
        g.find_mode(y, F, w["lik"], None, opts)
        nll, _, _ = g.neg_log_marglik(opts, want_grad=True)
        g.predict(cp, Fp, opts)
        g.close()
        return nll

    gpu_eval()
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        nll_g = gpu_eval()
    torch.cuda.synchronize()
    t_gpu = (time.perf_counter() - t0) / reps
    o = OL.Opts(cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"], num_probes=w["t"],
                num_pred_samples=w["s"], seed=args.seed)
    t0 = time.perf_counter()
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]), deriv=True)
    b, W, _ = OL.find_mode(model, w["y"], w["F"], w["lik"], None, o)
    nll_o, _ = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o, want_grad=True)
    OL.predict(model, w["coords_pred"], w["Fp"], b, W, o)
    t_cpu = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    log(args, f"n=2000: gpu {t_gpu * 1e3:.1f} ms/eval, oracle {t_cpu:.2f} s/eval")
    return {"workload": "c1_n2000: n=2000, exponential rho=0.1, m=10, Bernoulli-logit, t=50, "
                        "CG tol 1e-8, 500 test points, s=64; one eval = build + mode + NLL + "
                        "gradient + predict",
            "gpu_evals_per_s": 1.0 / t_gpu, "oracle_evals_per_s": 1.0 / t_cpu,
            "oracle_cores": threads, "nll_gpu": nll_g, "nll_oracle": nll_o}


if __name__ == "__main__":
    main()

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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2_n1e5")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
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

    def step(rec):
        t0 = time.perf_counter()
        g = P.VecchiaLaplace(coords, w["m"], w["kind"], theta, want_deriv=True)
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
        g.close()

    warm = []
    for k in range(args.warmup):
        step(warm)
        log(args, f"warmup {k}: {warm[-1]}")
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(rec)
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

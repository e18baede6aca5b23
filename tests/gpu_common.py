"""Helpers shared by the GPU parity tests: device transfer, oracle runs with
optional replay of the device's iteration counts, and error metrics."""
import sys

import numpy as np
import torch

from oracle import laplace as OL

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """max |a - b| / max(|b|) (vector-relative, robust to zero entries)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)


def rel_err_elem(a, b):
    """max_i |a_i - b_i| / |b_i| (element-wise relative; for quantities
    bounded away from zero, e.g. variances)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def opts_pair(P, **kw):
    """The same options for the oracle and the device library."""
    o = OL.Opts(**kw)
    g = P.vl_default_opts(max_newton=o.max_newton, newton_tol=o.newton_tol, max_cg=o.max_cg,
                          cg_tol=o.cg_tol, pred_cg_tol=o.pred_cg_tol,
                          num_probes=o.num_probes, num_pred_samples=o.num_pred_samples,
                          seed=o.seed, precond=o.precond, lrac_rank=o.lrac_rank)
    return o, g


def oracle_mode_matching(model, y, F, lik, aux, opts, gpu_newton_cg, L=None, gpu_halvings=None):
    """Oracle mode; replays the device's Newton/CG (and step-halving) counts if
    they differ."""
    b, W, st = OL.find_mode(model, y, F, lik, aux, opts, L=L)
    same = list(st["cg_iters"]) == list(gpu_newton_cg)
    if gpu_halvings is not None:
        same = same and list(st["halvings"]) == list(gpu_halvings)
    if same:
        return b, W, st, False
    replay = {"newton_iters": len(gpu_newton_cg), "cg_iters": list(gpu_newton_cg)}
    if gpu_halvings is not None:
        replay["halvings"] = list(gpu_halvings)
    b, W, st = OL.find_mode(model, y, F, lik, aux, opts, L=L, replay=replay)
    return b, W, st, True

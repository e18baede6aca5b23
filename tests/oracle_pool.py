"""Runs the oracle's neighbour search and Vecchia factor over row ranges in
separate processes, for workloads too large for one process to finish in
seconds.  Each row of the result is computed by the oracle functions alone,
exactly as the single-process call would compute it; this module only splits
the rows and joins the pieces."""
import multiprocessing as mp
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from oracle import vecchia as V


def _rows_job(args):
    coords, m, kind, theta, r0, r1 = args
    rows = np.arange(r0, r1)
    nbr = V.neighbours_rows(coords, m, rows)
    A, D = V.factor(coords, nbr, kind, theta, coords_self=coords[r0:r1])
    return r0, nbr.astype(np.int32), A, D


def neighbours_and_factor(coords, m, kind, theta, workers=None, pieces=64):
    """(nbr int32 n x m, A n x m, D n) for every row, computed in `pieces`
    row ranges by at most `workers` processes (default: the CPU count, at
    most 16).  Processes are started with 'spawn' so that none inherits a
    GPU context."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[0]
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    cuts = np.linspace(0, n, pieces + 1).astype(np.int64)
    nbr = np.empty((n, m), dtype=np.int32)
    A = np.empty((n, m))
    D = np.empty(n)
    jobs = [(coords, m, kind, tuple(theta), int(a), int(b))
            for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for done, (r0, nb, a, d) in enumerate(ex.map(_rows_job, jobs), 1):
            r1 = r0 + nb.shape[0]
            nbr[r0:r1], A[r0:r1], D[r0:r1] = nb, a, d
            if done % 8 == 0:
                print(f"oracle factor rows: {done}/{len(jobs)} pieces", file=sys.stderr,
                      flush=True)
    return nbr, A, D


def _cov_variant(d2, kind, theta):
    """The covariance functions of Sec. 4.1 evaluated in another, equally
    valid, order of operations (entries differ from the oracle's by a few
    units in the last place, as any two implementations' do)."""
    sigma2, rho = float(theta[0]), float(theta[1])
    d = np.sqrt(d2)
    if kind == 0:
        return np.exp(-d * (1.0 / rho)) * sigma2
    a = d * (np.sqrt(3.0) / rho)
    e = np.exp(-a)
    return sigma2 * e + sigma2 * a * e


def _cholesky_rows_job(args):
    """A_i by Cholesky factorisation and two substitutions, with the
    covariances evaluated in another order, instead of the oracle's LU solve:
    a second correct FP64 implementation of Sigma_N(i) A_i = Sigma_N(i),i,
    whose spread against the oracle measures how far the conditioning lets
    two correct implementations drift apart."""
    coords, nbr, kind, theta, r0, r1 = args
    nb = nbr[r0:r1]
    A = np.zeros(nb.shape)
    D = np.full(nb.shape[0], float(theta[0]))
    cnt = (nb >= 0).sum(axis=1)
    for k in np.unique(cnt):
        if k == 0:
            continue
        rows = np.nonzero(cnt == k)[0]
        P = coords[nb[rows, :k]]
        q = coords[r0 + rows]
        S = _cov_variant(V.sqdist(P[:, :, None, :], P[:, None, :, :]), kind, theta)
        c = _cov_variant(V.sqdist(P, q[:, None, :]), kind, theta)
        Lc = np.linalg.cholesky(S)
        z = np.zeros_like(c)
        for j in range(k):  # L z = c
            z[:, j] = (c[:, j] - np.einsum("rl,rl->r", Lc[:, j, :j], z[:, :j])) / Lc[:, j, j]
        a = np.zeros_like(c)
        for j in range(k - 1, -1, -1):  # L^T a = z
            a[:, j] = (z[:, j] - np.einsum("rl,rl->r", Lc[:, j + 1:, j], a[:, j + 1:])) / Lc[:, j, j]
        A[rows, :k] = a
        D[rows] = float(theta[0]) - np.einsum("rk,rk->r", c, a)
    return r0, A, D


def factor_cholesky(coords, nbr, kind, theta, workers=None, pieces=64):
    """(A n x m, D n) of every row by the Cholesky variant, over row ranges."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n, m = nbr.shape
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    cuts = np.linspace(0, n, pieces + 1).astype(np.int64)
    A = np.empty((n, m))
    D = np.empty(n)
    jobs = [(coords, nbr, kind, tuple(theta), int(a), int(b))
            for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for done, (r0, a, d) in enumerate(ex.map(_cholesky_rows_job, jobs), 1):
            if done % 8 == 0:
                print(f"oracle second factor: {done}/{len(jobs)} pieces", file=sys.stderr, flush=True)
            A[r0:r0 + a.shape[0]] = a
            D[r0:r0 + a.shape[0]] = d
    return A, D


def _slq_job(args):
    from oracle import laplace as L
    model, y, F, lik, b, opts, c0, c1, replay = args
    o = L.Opts(**{k: getattr(opts, k) for k in vars(opts)})
    o.num_probes = c1 - c0
    _, info = L.neg_log_marglik(model, y, F, lik, None, b, o, col0=c0,
                                replay_cg=None if replay is None else replay[c0:c1])
    return c0, info["quad"], info["r0z0"], info["cg_iters"]


def slq_columns(model, y, F, lik, b, opts, t, replay=None, workers=None):
    """Per-probe SLQ quadratures, weights and CG counts of probe columns
    0..t-1, each slice of columns run by the oracle in its own process."""
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    cuts = np.linspace(0, t, min(t, 4 * workers) + 1).astype(np.int64)
    quad, r0z0, iters = np.empty(t), np.empty(t), np.empty(t, dtype=np.int64)
    jobs = [(model, y, F, lik, b, opts, int(a), int(c), replay)
            for a, c in zip(cuts[:-1], cuts[1:]) if c > a]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for done, (c0, q, r, it) in enumerate(ex.map(_slq_job, jobs), 1):
            print(f"oracle probe columns: {done}/{len(jobs)} pieces", file=sys.stderr, flush=True)
            k = q.shape[0]
            quad[c0:c0 + k], r0z0[c0:c0 + k], iters[c0:c0 + k] = q, r, it
    return quad, r0z0, iters


def _pred_job(args):
    from oracle import laplace as L
    model, coords_p, Fp, b, W, opts, c0, c1, replay = args
    o = L.Opts(**{k: getattr(opts, k) for k in vars(opts)})
    o.num_pred_samples = c1 - c0
    _, _, info = L.predict(model, coords_p, Fp, b, W, o, col0=c0,
                           replay_cg=None if replay is None else replay[c0:c1])
    return c0, info["acc"], info["Dp"], info["cg_iters"]


def pred_columns(model, coords_p, Fp, b, W, opts, s, replay=None, workers=None):
    """Simulated predictive variances D_p + (1/s) sum over sample columns
    0..s-1 of (A_p u_i)^2 (Alg. simAlgo), the columns split over processes;
    returns (var, per-column CG counts)."""
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    cuts = np.linspace(0, s, min(s, 4 * workers) + 1).astype(np.int64)
    acc, Dp, iters = None, None, np.empty(s, dtype=np.int64)
    jobs = [(model, coords_p, Fp, b, W, opts, int(a), int(c), replay)
            for a, c in zip(cuts[:-1], cuts[1:]) if c > a]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for done, (c0, a, dp, it) in enumerate(ex.map(_pred_job, jobs), 1):
            print(f"oracle sample columns: {done}/{len(jobs)} pieces", file=sys.stderr, flush=True)
            acc = a if acc is None else acc + a
            Dp = dp
            iters[c0:c0 + it.shape[0]] = it
    return Dp + acc / s, iters

"""Runs the oracle's neighbour search and Vecchia factor over row ranges in
separate processes, for workloads too large for one process to finish in
seconds.  Each row of the result is computed by the oracle functions alone,
exactly as the single-process call would compute it; this module only splits
the rows and joins the pieces."""
import multiprocessing as mp
import os
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
        for r0, nb, a, d in ex.map(_rows_job, jobs):
            r1 = r0 + nb.shape[0]
            nbr[r0:r1], A[r0:r1], D[r0:r1] = nb, a, d
    return nbr, A, D

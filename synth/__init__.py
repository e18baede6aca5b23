"""Seeded synthetic workloads for iterative Vecchia-Laplace inference.

This module only draws inputs: locations, latent fields, responses, offsets
and test locations.  It holds none of the method's arithmetic (no Vecchia
factor, no solver), so that the oracle and the HIP library can both consume
its output without sharing code.

The workloads follow the paper's simulation setting (Sec. 4.1): locations
i.i.d. uniform on [0,1]^2 (their generation order is the random ordering of
the Vecchia approximation), a zero-mean GP latent field with exponential or
Matern-3/2 covariance and sigma^2 = 1, and Bernoulli-logit or Poisson
log-link responses; the Gamma log-link response (Sec. 5) is drawn with a
given shape a and mean e^mu.

Latent fields:
  * n <= 5000: exact draw, dense Cholesky of the covariance matrix.
  * larger n: random Fourier features with K = 2048 frequencies drawn from the
    Matern spectral density (a bivariate Student-t with 2 nu degrees of freedom
    scaled by 1/rho; nu = 1/2 exponential, nu = 3/2 Matern-3/2).  The field
    only shapes the responses; no result is compared against it.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

COV_EXPONENTIAL = 0
COV_MATERN32 = 1
LIK_BERNOULLI_LOGIT = 0
LIK_POISSON = 1
LIK_GAUSSIAN = 2
LIK_GAMMA = 3


def _rng(seed, stream):
    return np.random.default_rng([int(seed), int(stream)])


def locations(n, seed, stream=0):
    """n x 2 locations uniform on [0,1]^2 (float64, C-contiguous)."""
    return np.ascontiguousarray(_rng(seed, 100 + stream).uniform(size=(n, 2)))


def _cov_dense(d, kind, sigma2, rho):
    if kind == COV_EXPONENTIAL:
        return sigma2 * np.exp(-d / rho)
    a = math.sqrt(3.0) * d / rho
    return sigma2 * (1.0 + a) * np.exp(-a)


def latent_field(coords, kind, sigma2, rho, seed, nfeat=2048, chunk=1 << 16):
    """A zero-mean GP draw at coords (see module docstring)."""
    n = coords.shape[0]
    g = _rng(seed, 200)
    if n <= 5000:
        diff = coords[:, None, :] - coords[None, :, :]
        d = np.sqrt(np.sum(diff * diff, axis=-1))
        C = _cov_dense(d, kind, sigma2, rho)
        L = np.linalg.cholesky(C + 1e-10 * sigma2 * np.eye(n))
        return L @ g.standard_normal(n)
    nu = 0.5 if kind == COV_EXPONENTIAL else 1.5
    dof = 2.0 * nu
    z = g.standard_normal((nfeat, 2))
    chi = g.chisquare(dof, size=nfeat)
    omega = z / np.sqrt(chi / dof)[:, None] / rho
    phase = g.uniform(0.0, 2.0 * np.pi, size=nfeat)
    amp = math.sqrt(2.0 * sigma2 / nfeat)
    out = np.empty(n)

    def fill(s):
        e = min(n, s + chunk)
        out[s:e] = amp * np.cos(coords[s:e] @ omega.T + phase).sum(axis=1)

    # Chunks are independent and numpy releases the GIL inside them, so a
    # thread pool gives the same values as a serial loop.
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fill, range(0, n, chunk)))
    return out


def responses(lik, mu, seed, tau2=None, shape=None):
    g = _rng(seed, 300)
    if lik == LIK_BERNOULLI_LOGIT:
        p = 1.0 / (1.0 + np.exp(-mu))
        return (g.uniform(size=mu.shape) < p).astype(np.float64)
    if lik == LIK_POISSON:
        return g.poisson(np.exp(mu)).astype(np.float64)
    if lik == LIK_GAUSSIAN:
        return mu + math.sqrt(tau2) * g.standard_normal(mu.shape)
    if lik == LIK_GAMMA:
        return g.gamma(shape, np.exp(mu) / shape)
    raise ValueError("unknown likelihood")


# Workload descriptions.  Sizes follow the configurations the library is
# measured on; `small` variants keep the same structure at sizes the oracle
# finishes in seconds.
WORKLOADS = {
    # n = 2,000, exponential, range 0.1, m = 10, Bernoulli-logit, exact field,
    # CG tolerance 1e-8, 50 probes
    "c1_n2000": dict(n=2000, m=10, kind=COV_EXPONENTIAL, sigma2=1.0, rho=0.1,
                     lik=LIK_BERNOULLI_LOGIT, F=0.0, t=50, cg_tol=1e-8,
                     n_pred=500, s=64, pred_cg_tol=1e-8),
    # n = 100,000, Matern-3/2, range 0.05, m = 20, Bernoulli-logit, 50 probes,
    # CG tolerance 1e-3, predictions at 10,000 test points with s = 2000
    "c2_n1e5": dict(n=100000, m=20, kind=COV_MATERN32, sigma2=1.0, rho=0.05,
                    lik=LIK_BERNOULLI_LOGIT, F=0.0, t=50, cg_tol=1e-3,
                    n_pred=10000, s=2000, pred_cg_tol=1e-3),
    # n = 2,000,000, Matern-3/2, range 0.02, m = 20, Poisson with latent mean
    # 1.0, 64 probes, CG tolerance 1e-2 (the paper's NLL tolerance)
    "c3_n2e6": dict(n=2000000, m=20, kind=COV_MATERN32, sigma2=1.0, rho=0.02,
                    lik=LIK_POISSON, F=1.0, t=64, cg_tol=1e-2,
                    n_pred=10000, s=256, pred_cg_tol=1e-3),
}


def make(name=None, seed=0, **override):
    """Build one workload: dict with coords, y, F, coords_pred, Fp and the
    parameters of WORKLOADS[name] (overridable, e.g. n=5000)."""
    spec = dict(WORKLOADS[name]) if name is not None else {}
    spec.update(override)
    n = spec["n"]
    coords = locations(n, seed)
    b = latent_field(coords, spec["kind"], spec["sigma2"], spec["rho"], seed)
    F = np.full(n, float(spec.get("F", 0.0)))
    y = responses(spec["lik"], F + b, seed, spec.get("tau2"), spec.get("shape"))
    npred = spec.get("n_pred", 0)
    spec.update(coords=coords, y=y, F=F, b_true=b,
                coords_pred=locations(npred, seed, stream=1),
                Fp=np.full(npred, float(spec.get("F", 0.0))),
                seed=seed, name=name)
    return spec


def batch_problems(count=256, seed=0, n_lo=1000, n_hi=50000):
    """Many uneven problems: n log-uniform in [n_lo, n_hi], m in {10,20,30},
    exponential or Matern-3/2 with probability 1/2, range U(0.02, 0.2),
    Bernoulli-logit, 32 probes each."""
    g = _rng(seed, 400)
    out = []
    for p in range(count):
        n = int(math.floor(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(g.choice([10, 20, 30]))
        kind = int(g.integers(0, 2))
        rho = float(g.uniform(0.02, 0.2))
        out.append(make(None, seed=seed * 100003 + p, n=n, m=m, kind=kind,
                        sigma2=1.0, rho=rho, lik=LIK_BERNOULLI_LOGIT, F=0.0,
                        t=32, cg_tol=1e-2, n_pred=0))
    return out


def serving_requests(count, seed=0, rate=100.0, n_lo=2000, n_hi=200000,
                     np_lo=1000, np_hi=20000):
    """Poisson-arrival fit+predict requests: arrival times (s), n log-uniform
    in [n_lo, n_hi], n_pred uniform in [np_lo, np_hi], m = 20, Bernoulli or
    Poisson with probability 1/2 each, Matern-3/2 range 0.05."""
    g = _rng(seed, 500)
    t = 0.0
    reqs = []
    for r in range(count):
        t += g.exponential(1.0 / rate)
        n = int(math.floor(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        n_pred = int(g.integers(np_lo, np_hi + 1))
        lik = int(g.integers(0, 2))
        spec = make(None, seed=seed * 1000003 + r, n=n, m=20, kind=COV_MATERN32,
                    sigma2=1.0, rho=0.05, lik=lik,
                    F=(0.0 if lik == LIK_BERNOULLI_LOGIT else 1.0), t=50,
                    cg_tol=1e-2, n_pred=n_pred, s=64, pred_cg_tol=1e-3)
        spec["arrival"] = t
        reqs.append(spec)
    return reqs

"""Iterative Vecchia-Laplace inference (oracle side).  TEST INFRASTRUCTURE ONLY.

Plain FP64 NumPy/SciPy, following the paper step by step:

  likelihoods      Sec. 2 (log-concave p(y|mu)); Bernoulli-logit of Sec. 4.1,
                   Poisson log-link, Gaussian (exact-Laplace special case),
                   Gamma log-link with shape xi (Sec. 5); derivatives in
                   mu and in the auxiliary parameter xi
  pcg              appendix algorithm "Preconditioned conjugate gradient
                   algorithm with Lanczos tridiagonal matrix", run column by
                   column (each probe has its own recurrence)
  slq_quadrature   e_1^T log(T~) e_1 from the CG coefficients, eq. (def_SLQ)
  find_mode        Newton iteration eq. (newton) with CG solves, eq. (pcls1)
                   for VADU, LVA (Sec. 3.1.1) and the diagonal P_1 (Sec.
                   3.1.4), eq. (pcls2) for LRAC
  neg_log_marglik  eq. (VLA_loss) with the log-determinant split
                   eq. (logdetsplit) (VADU, Sec. 3.1.1) or eq. (logdetsplit2)
                   (LRAC, Sec. 3.1.2) and SLQ for the last term
  grad_theta       App. "Gradients of Vecchia-Laplace approximations" with the
                   VADU or LRAC STE / control-variate formulas of the appendix
                   "Derivatives of log-determinants ... Preconditioner VADU /
                   LRAC" (LRAC with the forward-mode derivative of the
                   pivoted Cholesky factor);
                   also the gradient in the offset F (for F = X beta the
                   beta-gradient is X^T of it) and in the likelihood's
                   auxiliary parameter xi (Gaussian tau^2, Gamma shape)
  predict          eq. (latentpostpredictive) with B_p = I and the simulation
                   algorithm (Sec. 3.3.1, Alg. simAlgo)
  predict_lanczos  the same means with preconditioned Lanczos variances (Sec.
                   3.3.2, P_L1 and P_L2, complete reorthogonalization)

Readings of silent or ambiguous points:
  * CG stops when the unpreconditioned residual 2-norm is below `cg_tol`
    (absolute), u_0 = 0, at most `max_cg` iterations.
  * Newton starts at b = 0 and stops when
    |Psi_new - Psi_old| <= newton_tol * |Psi_old|, Psi(b) = log p(y|F+b)
    - b^T Sigma~^{-1} b / 2; a step that lowers Psi by more than
    HALVING_SLACK |Psi| is halved, at most MAX_HALVINGS times (no halving can
    help: keep b and stop); W for the marginal likelihood is taken at the
    final mode.
  * SLQ uses Rademacher probes eps; for VADU z = B^T (W+D^{-1})^{1/2} eps so
    that Cov(z) = P; the weight ||P^{-1/2} z||^2 is r_0^T z_0 of the CG run
    (first form of eq. def_SLQ).  For LRAC z = L_k eps_k + W^{-1/2} eps_n.
  * Control-variate weight c = sample Cov(h, r) / sample Var(r) over the t
    probes; c = 0 when Var(r) <= 1e-10 mean(r)^2 (then r is constant and the
    c-terms cancel exactly).  For the mu-derivative one c per component.
  * The full negative log-likelihood is used (log y! for Poisson and the
    Gaussian constants included).
  * Prediction: m nearest training points, Gaussian z^(1), z^(2).

Parity: see the pins in tests/test_oracle_laplace.py.  Large-n absolute
values have no pin beyond these (parity unpinned at n >= 1e5 except through
the small-n pins of the same code).
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular
from scipy.special import digamma, gammaln

from . import rng as _rng
from . import vecchia as _vec

LIK_BERNOULLI_LOGIT = 0
LIK_POISSON = 1
LIK_GAUSSIAN = 2
LIK_GAMMA = 3  # log link, mean exp(mu), shape aux (Sec. 5)

PRECOND_VADU = 0
PRECOND_LRAC = 1
PRECOND_LVA = 2    # P = B^T D^{-1} B (Sec. 3.1.1)
PRECOND_DIAG = 3   # P_1 = diag(W + B^T D^{-1} B) (Sec. 3.1.4)


# ----------------------------------------------------------------------------
# likelihoods: log p, d/dmu, W = -d2/dmu2, dW/dmu = -d3/dmu3
# ----------------------------------------------------------------------------
def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def lik_logp(lik, y, mu, aux=None):
    if lik == LIK_BERNOULLI_LOGIT:
        # y mu - log(1 + e^mu)
        return y * mu - np.logaddexp(0.0, mu)
    if lik == LIK_POISSON:
        return y * mu - np.exp(mu) - gammaln(y + 1.0)
    if lik == LIK_GAUSSIAN:
        tau2 = float(aux)
        return -0.5 * (y - mu) ** 2 / tau2 - 0.5 * np.log(2.0 * np.pi * tau2)
    if lik == LIK_GAMMA:
        # shape a, rate a e^{-mu}: a log a - log Gamma(a) + (a - 1) log y - a mu - a y e^{-mu}
        a = float(aux)
        return a * np.log(a) - gammaln(a) + (a - 1.0) * np.log(y) - a * mu - a * y * np.exp(-mu)
    raise ValueError("unknown likelihood")


def lik_grad(lik, y, mu, aux=None):
    if lik == LIK_BERNOULLI_LOGIT:
        return y - _sigmoid(mu)
    if lik == LIK_POISSON:
        return y - np.exp(mu)
    if lik == LIK_GAUSSIAN:
        return (y - mu) / float(aux)
    if lik == LIK_GAMMA:
        return float(aux) * (y * np.exp(-mu) - 1.0)
    raise ValueError("unknown likelihood")


def lik_W(lik, y, mu, aux=None):
    if lik == LIK_BERNOULLI_LOGIT:
        p = _sigmoid(mu)
        return p * (1.0 - p)
    if lik == LIK_POISSON:
        return np.exp(mu)
    if lik == LIK_GAUSSIAN:
        return np.full_like(mu, 1.0 / float(aux))
    if lik == LIK_GAMMA:
        return float(aux) * y * np.exp(-mu)
    raise ValueError("unknown likelihood")


def lik_dW(lik, y, mu, aux=None):
    """d W_ii / d mu_i = -d^3 log p / d mu^3."""
    if lik == LIK_BERNOULLI_LOGIT:
        p = _sigmoid(mu)
        return p * (1.0 - p) * (1.0 - 2.0 * p)
    if lik == LIK_POISSON:
        return np.exp(mu)
    if lik == LIK_GAUSSIAN:
        return np.zeros_like(mu)
    if lik == LIK_GAMMA:
        return -float(aux) * y * np.exp(-mu)
    raise ValueError("unknown likelihood")


def lik_has_aux(lik):
    """Whether the likelihood has an auxiliary parameter xi (Sec. 2)."""
    return lik in (LIK_GAUSSIAN, LIK_GAMMA)


def lik_dlogp_dxi(lik, y, mu, aux):
    """d log p(y_i | mu_i, xi) / d xi per row (Gaussian xi = tau^2, Gamma xi =
    shape a)."""
    if lik == LIK_GAUSSIAN:
        tau2 = float(aux)
        return 0.5 * (y - mu) ** 2 / tau2 ** 2 - 0.5 / tau2
    if lik == LIK_GAMMA:
        a = float(aux)
        return np.log(a) + 1.0 - digamma(a) + np.log(y) - mu - y * np.exp(-mu)
    raise ValueError("likelihood without an auxiliary parameter")


def lik_dgrad_dxi(lik, y, mu, aux):
    """d^2 log p / d xi d mu per row."""
    if lik == LIK_GAUSSIAN:
        return -(y - mu) / float(aux) ** 2
    if lik == LIK_GAMMA:
        return y * np.exp(-mu) - 1.0
    raise ValueError("likelihood without an auxiliary parameter")


def lik_dW_dxi(lik, y, mu, aux):
    """d W_ii / d xi = -d^3 log p / d xi d mu^2 per row."""
    if lik == LIK_GAUSSIAN:
        return np.full_like(mu, -1.0 / float(aux) ** 2)
    if lik == LIK_GAMMA:
        return y * np.exp(-mu)
    raise ValueError("likelihood without an auxiliary parameter")


# ----------------------------------------------------------------------------
# the model: Vecchia factor plus sparse operators
# ----------------------------------------------------------------------------
class Model:
    """Vecchia factor of one data set at one theta (Sec. 2.1)."""

    def __init__(self, coords, m, kind, theta, nbr=None, deriv=False, factor=None):
        """nbr and factor = (A, D) may be passed in when they were already
        computed by the neighbour search and factor functions (for example
        over row ranges); otherwise they are computed here."""
        self.coords = np.asarray(coords, dtype=np.float64)
        self.n = self.coords.shape[0]
        self.m = m
        self.kind = kind
        self.theta = (float(theta[0]), float(theta[1]))
        self.nbr = _vec.neighbours(self.coords, m) if nbr is None else nbr
        if factor is not None and deriv:
            raise ValueError("a precomputed factor carries no derivatives")
        out = factor if factor is not None else _vec.factor(self.coords, self.nbr, kind,
                                                             self.theta, deriv=deriv)
        if deriv:
            self.A, self.D, self.dA, self.dD = out
            self.dB = [_vec.sparse_dB(self.dA[k], self.nbr) for k in range(2)]
        else:
            self.A, self.D = out
        self.Dinv = 1.0 / self.D
        self.B = _vec.sparse_B(self.A, self.nbr)
        self.Bt = self.B.T.tocsr()

    # B^{-1} x and B^{-T} x by sparse triangular solves
    def solve_B(self, x):
        return spsolve_triangular(self.B, x, lower=True, unit_diagonal=True)

    def solve_Bt(self, x):
        return spsolve_triangular(self.Bt, x, lower=False, unit_diagonal=True)

    def prec_apply(self, x):
        """Sigma~^{-1} x = B^T D^{-1} B x."""
        return self.Bt @ (_col(self.Dinv, x) * (self.B @ x))

    def cov_apply(self, x):
        """Sigma~ x = B^{-1} D B^{-T} x (two triangular solves, Sec. 3)."""
        return self.solve_B(_col(self.D, x) * self.solve_Bt(x))


def _col(v, x):
    """Broadcast a length-n vector against x (n or n x t)."""
    return v if x.ndim == 1 else v[:, None]


# ----------------------------------------------------------------------------
# preconditioned CG with Lanczos coefficients (appendix algorithm)
# ----------------------------------------------------------------------------
class CGResult:
    def __init__(self, U, alphas, betas, iters, r0z0, Z0):
        self.U = U              # approximate solutions, n x t
        self.alphas = alphas    # list per column of alpha_1..alpha_l
        self.betas = betas      # list per column of beta_1..beta_l
        self.iters = iters      # iterations per column
        self.r0z0 = r0z0        # r_0^T z_0 per column
        self.Z0 = Z0            # z_0 = P^{-1} r_0, n x t


def pcg(apply_A, apply_Pinv, rhs, tol, max_iter, forced_iters=None):
    """Preconditioned CG on every column of `rhs` independently.

    Literal reading of the appendix algorithm: u_0 = 0, r_0 = b, z_0 = P^{-1}
    r_0, h_0 = z_0; per iteration l: v = A h, alpha = r^T z / h^T v,
    u += alpha h, r -= alpha v, stop flag if ||r||_2 < tol, z = P^{-1} r,
    beta = r_new^T z_new / r^T z, h = z + beta h.  A column that stopped keeps
    its state.  `forced_iters` (per column) replaces the stopping test by a
    fixed iteration count (replay of another run's counts)."""
    X = rhs if rhs.ndim == 2 else rhs[:, None]
    n, t = X.shape
    U = np.zeros((n, t))
    R = X.copy()
    Z = apply_Pinv(R)
    H = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    r0z0 = rz.copy()
    Z0 = Z.copy()
    active = np.ones(t, dtype=bool)
    iters = np.zeros(t, dtype=np.int64)
    alphas = [[] for _ in range(t)]
    betas = [[] for _ in range(t)]
    for it in range(max_iter):
        if forced_iters is not None:
            active &= iters < np.asarray(forced_iters)
        if not active.any():
            break
        cols = np.nonzero(active)[0]
        Hc = H[:, cols]
        V = apply_A(Hc)
        alpha = rz[cols] / np.einsum("ij,ij->j", Hc, V)
        U[:, cols] += alpha * Hc
        R[:, cols] -= alpha * V
        rnorm = np.sqrt(np.einsum("ij,ij->j", R[:, cols], R[:, cols]))
        Znew = apply_Pinv(R[:, cols])
        rz_new = np.einsum("ij,ij->j", R[:, cols], Znew)
        beta = rz_new / rz[cols]
        H[:, cols] = Znew + beta * Hc
        rz[cols] = rz_new
        for q, c in enumerate(cols):
            alphas[c].append(alpha[q])
            betas[c].append(beta[q])
            iters[c] += 1
        if forced_iters is None:
            stop = rnorm < tol
            active[cols[stop]] = False
    if rhs.ndim == 1:
        U = U[:, 0]
    return CGResult(U, alphas, betas, iters, r0z0, Z0)


def lanczos_tridiag(alphas, betas):
    """T~ from CG coefficients (appendix algorithm): T_{1,1} = 1/alpha_1,
    T_{j,j} = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j-1,j} = T_{j,j-1} = sqrt(beta_{j-1})/alpha_{j-1}."""
    L = len(alphas)
    T = np.zeros((L, L))
    for j in range(L):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j > 0:
            T[j - 1, j] = T[j, j - 1] = np.sqrt(betas[j - 1]) / alphas[j - 1]
    return T


def slq_quadrature(alphas, betas):
    """e_1^T log(T~) e_1 = sum_j V_{1j}^2 log(lambda_j) (eq. def_SLQ)."""
    T = lanczos_tridiag(alphas, betas)
    lam, V = np.linalg.eigh(T)
    return float(np.sum(V[0, :] ** 2 * np.log(lam)))


# ----------------------------------------------------------------------------
# operators of the two CG forms
# ----------------------------------------------------------------------------
def vadu_ops(model, W):
    """A = W + B^T D^{-1} B and P_VADU^{-1} = B^{-1} (W + D^{-1})^{-1} B^{-T}
    (eq. pcls1, eq. P_VADU)."""
    wd = W + model.Dinv

    def apply_A(X):
        return _col(W, X) * X + model.prec_apply(X)

    def apply_Pinv(X):
        return model.solve_B(model.solve_Bt(X) / _col(wd, X))

    return apply_A, apply_Pinv


def lva_ops(model, W):
    """A = W + B^T D^{-1} B and P_LVA^{-1} = B^{-1} D B^{-T} (Sec. 3.1.1)."""
    def apply_A(X):
        return _col(W, X) * X + model.prec_apply(X)

    def apply_Pinv(X):
        return model.solve_B(model.solve_Bt(X) * _col(model.D, X))

    return apply_A, apply_Pinv


def diag_p1(model, W):
    """(P_1)_ii = (W + B^T D^{-1} B)_ii = W_i + sum_j B_ji^2 / D_j (Sec. 3.1.4)."""
    B2 = model.B.multiply(model.B)
    return W + B2.T @ model.Dinv


def diag_ops(model, W):
    """A = W + B^T D^{-1} B and P_1^{-1} = diag(P_1)^{-1}."""
    p1 = diag_p1(model, W)

    def apply_A(X):
        return _col(W, X) * X + model.prec_apply(X)

    def apply_Pinv(X):
        return X / _col(p1, X)

    return apply_A, apply_Pinv


def sparse_precond_ops(model, W, precond):
    """Operator and preconditioner of eq. (pcls1) for VADU, LVA or P_1."""
    if precond == PRECOND_VADU:
        return vadu_ops(model, W)
    if precond == PRECOND_LVA:
        return lva_ops(model, W)
    if precond == PRECOND_DIAG:
        return diag_ops(model, W)
    raise ValueError("not a preconditioner of eq. (pcls1)")


def pivoted_cholesky(coords, kind, theta, k, pivots=None):
    """Rank-k pivoted Cholesky of the original covariance matrix Sigma
    (Sec. 3.1.2): pivot = largest remaining diagonal (first index on ties).

    pivots: optional sequence that replaces the argmax choices (replay of
    another implementation's pivots when two residual diagonals tie to
    rounding); the arithmetic is unchanged."""
    sigma2, rho = theta
    n = coords.shape[0]
    k = min(k, n)
    L = np.zeros((n, k))
    d = np.full(n, float(sigma2))
    for j in range(k):
        p = int(np.argmax(d)) if pivots is None else int(pivots[j])
        col = _vec.covariance(_vec.sqdist(coords, coords[p]), kind, sigma2, rho)
        L[:, j] = (col - L[:, :j] @ L[p, :j]) / np.sqrt(d[p])
        d = d - L[:, j] ** 2
    return L


def pivoted_cholesky_deriv(coords, kind, theta, k, pivots=None):
    """L_k of pivoted_cholesky and its derivatives dL[q] = d L_k / d theta_q
    (q = 0: sigma2, 1: rho), the forward-mode derivative of the same steps
    with the pivots held fixed (they are piecewise constant in theta).  The
    paper leaves d L_k / d theta open (App. "Preconditioner LRAC"); with
    d_p = Sigma_pp - sum_{l<j} L_pl^2 and column j = (Sigma[:, p] - L L_p^T) /
    sqrt(d_p):
      d col_j = (dSigma[:, p] - dL L_p^T - L dL_p^T - col_j d(sqrt d_p)) / sqrt(d_p),
      d(sqrt d_p) = (dSigma_pp - 2 sum_{l<j} L_pl dL_pl) / (2 sqrt d_p).
    Returns (L, dL, pivots)."""
    sigma2, rho = theta
    n = coords.shape[0]
    k = min(k, n)
    L = np.zeros((n, k))
    dL = np.zeros((2, n, k))
    d = np.full(n, float(sigma2))
    dd = np.stack([np.ones(n), np.zeros(n)])  # d Sigma_ii / d theta: c(0) = sigma2
    piv = []
    for j in range(k):
        p = int(np.argmax(d)) if pivots is None else int(pivots[j])
        piv.append(p)
        d2 = _vec.sqdist(coords, coords[p])
        col = _vec.covariance(d2, kind, sigma2, rho)
        dcol = _vec.covariance_grad(d2, kind, sigma2, rho)
        s = np.sqrt(d[p])
        L[:, j] = (col - L[:, :j] @ L[p, :j]) / s
        for q in range(2):
            ds = dd[q][p] / (2.0 * s)
            dnum = dcol[q] - dL[q][:, :j] @ L[p, :j] - L[:, :j] @ dL[q][p, :j]
            dL[q][:, j] = (dnum - L[:, j] * ds) / s
            dd[q] = dd[q] - 2.0 * L[:, j] * dL[q][:, j]
        d = d - L[:, j] ** 2
    return L, dL, np.asarray(piv)


class LracPrecond:
    """P_LRAC = L_k L_k^T + W^{-1} (eq. P_LRAC) with Woodbury solves and the
    determinant lemma."""

    def __init__(self, L, W):
        self.L = L
        self.W = W
        k = L.shape[1]
        self.M = np.eye(k) + L.T @ (W[:, None] * L)
        self.Mc = np.linalg.cholesky(self.M)
        self.logdet = 2.0 * np.sum(np.log(np.diag(self.Mc))) - np.sum(np.log(W))

    def solve(self, X):
        """P^{-1} X = W X - W L M^{-1} L^T W X."""
        WX = _col(self.W, X) * X
        Y = np.linalg.solve(self.M, self.L.T @ WX)
        return WX - _col(self.W, X) * (self.L @ Y)


def lrac_ops(model, W, L):
    """Operator Sigma~ + W^{-1} of eq. (pcls2) and P_LRAC^{-1}."""
    P = LracPrecond(L, W)

    def apply_A(X):
        return model.cov_apply(X) + X / _col(W, X)

    return apply_A, P.solve, P


# ----------------------------------------------------------------------------
# Newton mode finding, eq. (newton)
# ----------------------------------------------------------------------------
class Opts:
    def __init__(self, **kw):
        self.max_newton = 100
        self.newton_tol = 1e-6
        self.max_cg = 1000
        self.cg_tol = 1e-3
        self.num_probes = 50
        self.num_pred_samples = 2000
        self.pred_cg_tol = 1e-3
        self.seed = 0
        self.precond = PRECOND_VADU
        self.lrac_rank = 50
        for k, v in kw.items():
            if not hasattr(self, k):
                raise KeyError(k)
            setattr(self, k, v)


MAX_HALVINGS = 30
HALVING_SLACK = 1e-12


def psi(model, y, F, b, lik, aux):
    """Psi(b) = log p(y | F + b) - b^T Sigma~^{-1} b / 2."""
    Bb = model.B @ b
    return float(np.sum(lik_logp(lik, y, F + b, aux)) - 0.5 * np.sum(model.Dinv * Bb * Bb))


def find_mode(model, y, F, lik, aux, opts, replay=None, L=None):
    """Mode b* of p(y|F+b) p~(b) by Newton's method, eq. (newton):
    b_{t+1} = (W + Sigma~^{-1})^{-1} (W b_t + d log p / d b), each solve by PCG,
    with the step halved (at most MAX_HALVINGS times) while Psi falls below
    Psi_old - HALVING_SLACK |Psi_old| (a real decrease, not rounding); stop when
    the relative change of Psi is at most newton_tol, or when no halving
    restores Psi (b is then kept).

    replay: optional dict {"newton_iters": int, "cg_iters": [int, ...]} that
    fixes the iteration counts.  Returns (b, W, stats)."""
    n = model.n
    F = np.zeros(n) if F is None else np.asarray(F, dtype=np.float64)
    b = np.zeros(n)
    psi_old = psi(model, y, F, b, lik, aux)
    cg_iters = []
    halving_log = []
    newton_iters = 0
    max_newton = opts.max_newton if replay is None else replay["newton_iters"]
    if opts.precond == PRECOND_LRAC and L is None:
        L = pivoted_cholesky(model.coords, model.kind, model.theta, opts.lrac_rank)
    for it in range(max_newton):
        mu = F + b
        g = lik_grad(lik, y, mu, aux)
        W = lik_W(lik, y, mu, aux)
        rhs = W * b + g
        forced = None if replay is None else [replay["cg_iters"][it]]
        if opts.precond != PRECOND_LRAC:
            apply_A, apply_Pinv = sparse_precond_ops(model, W, opts.precond)
            res = pcg(apply_A, apply_Pinv, rhs, opts.cg_tol, opts.max_cg, forced)
            b_new = res.U
        else:
            # eq. (pcls2): (Sigma~ + W^{-1}) (W u) = Sigma~ rhs
            apply_A, apply_Pinv, _ = lrac_ops(model, W, L)
            res = pcg(apply_A, apply_Pinv, model.cov_apply(rhs), opts.cg_tol,
                      opts.max_cg, forced)
            b_new = res.U / W
        cg_iters.append(int(res.iters[0]))
        newton_iters += 1
        # step halving while the objective does not increase (the paper gives
        # no step control; full steps diverge e.g. for Poisson counts)
        psi_new = psi(model, y, F, b_new, lik, aux)
        halvings = 0
        max_h = MAX_HALVINGS if replay is None else replay.get("halvings", [0] * max_newton)[it]
        floor = psi_old - HALVING_SLACK * abs(psi_old)  # rounding-level changes accepted
        while halvings < max_h and (replay is not None or not (psi_new >= floor)):
            b_new = b + 0.5 * (b_new - b)
            psi_new = psi(model, y, F, b_new, lik, aux)
            halvings += 1
        halving_log.append(halvings)
        if replay is None and not (psi_new >= floor):
            break  # no increase even after halving: b is the mode to rounding
        b = b_new
        if replay is None and abs(psi_new - psi_old) <= opts.newton_tol * abs(psi_old):
            break
        psi_old = psi_new
    W = lik_W(lik, y, F + b, aux)
    return b, W, {"newton_iters": newton_iters, "cg_iters": cg_iters, "halvings": halving_log}


# ----------------------------------------------------------------------------
# SLQ negative log-marginal likelihood, eq. (VLA_loss)
# ----------------------------------------------------------------------------
def neg_log_marglik(model, y, F, lik, aux, b, opts, replay_cg=None, L=None,
                    want_grad=False, replay_grad_cg=None, col0=0):
    """L^VLA = -log p(y|mu*) + b*^T Sigma~^{-1} b* / 2 + log det(Sigma~ W + I)/2.

    VADU: log det = sum log D + sum log(W + 1/D) + SLQ term (eq. logdetsplit,
    log det P_VADU = log det(W + D^{-1})).
    LVA: log det P_LVA = -sum log D; P_1: log det P_1 = sum log (P_1)_ii
    (same split).
    LRAC: log det = sum log W + log det P_LRAC + SLQ term (eq. logdetsplit2).
    The probes are the counter-based columns col0 .. col0 + num_probes - 1
    (col0 > 0 evaluates a slice of a larger probe set; not for LRAC).
    Returns (nll, info) with info holding the pieces, the CG iteration counts
    and (want_grad, VADU only) the theta-gradient."""
    n = model.n
    F = np.zeros(n) if F is None else np.asarray(F, dtype=np.float64)
    mu = F + b
    W = lik_W(lik, y, mu, aux)
    t = opts.num_probes
    if col0 and opts.precond == PRECOND_LRAC:
        raise ValueError("col0 applies to the probes of eq. (pcls1)")
    eps = _rng.rademacher(opts.seed, _rng.TAG_SLQ, n, t, col0=col0)
    if opts.precond != PRECOND_LRAC:
        # eq. (logdetsplit): log det(Sigma~ W + I) = log det Sigma~ + log det P
        # + log det(P^{-1/2} A P^{-T/2}), log det Sigma~ = sum log D; probes
        # z = P^{1/2} eps with Cov(z) = P
        apply_A, apply_Pinv = sparse_precond_ops(model, W, opts.precond)
        if opts.precond == PRECOND_VADU:
            # P^{1/2} = B^T (W + D^{-1})^{1/2}, log det P = sum log(W + D^{-1})
            Z = model.Bt @ (np.sqrt(W + model.Dinv)[:, None] * eps)
            logdet_P = np.sum(np.log(W + model.Dinv))
        elif opts.precond == PRECOND_LVA:
            # P^{1/2} = B^T D^{-1/2}, log det P = -sum log D
            Z = model.Bt @ (np.sqrt(model.Dinv)[:, None] * eps)
            logdet_P = -np.sum(np.log(model.D))
        else:
            # P_1^{1/2} = diag(P_1)^{1/2}, log det P_1 = sum log (P_1)_ii
            p1 = diag_p1(model, W)
            Z = np.sqrt(p1)[:, None] * eps
            logdet_P = np.sum(np.log(p1))
        res = pcg(apply_A, apply_Pinv, Z, opts.cg_tol, opts.max_cg, replay_cg)
        logdet_fixed = np.sum(np.log(model.D)) + logdet_P
    else:
        if L is None:
            L = pivoted_cholesky(model.coords, model.kind, model.theta, opts.lrac_rank)
        apply_A, apply_Pinv, P = lrac_ops(model, W, L)
        eps_k = _rng.rademacher(opts.seed, _rng.TAG_LRAC_K, L.shape[1], t)
        eps_n = _rng.rademacher(opts.seed, _rng.TAG_LRAC_N, n, t)
        Z = L @ eps_k + eps_n / np.sqrt(W)[:, None]
        res = pcg(apply_A, apply_Pinv, Z, opts.cg_tol, opts.max_cg, replay_cg)
        logdet_fixed = np.sum(np.log(W)) + P.logdet
    quad = np.array([slq_quadrature(res.alphas[c], res.betas[c]) for c in range(t)])
    gamma = float(np.mean(res.r0z0 * quad))
    logdet = logdet_fixed + gamma
    Bb = model.B @ b
    quadform = float(np.sum(model.Dinv * Bb * Bb))
    loglik = float(np.sum(lik_logp(lik, y, mu, aux)))
    nll = -loglik + 0.5 * quadform + 0.5 * logdet
    info = {"loglik": loglik, "quadform": quadform, "logdet": logdet,
            "gamma": gamma, "cg_iters": res.iters.copy(), "quad": quad,
            "r0z0": res.r0z0.copy()}
    if want_grad:
        if opts.precond == PRECOND_VADU:
            grad, ginfo = _grad_theta_vadu(model, y, F, lik, aux, b, W, res, opts,
                                           replay_grad_cg)
        elif opts.precond == PRECOND_LRAC:
            grad, ginfo = _grad_lrac(model, y, F, lik, aux, b, W, res, opts, P,
                                     replay_grad_cg)
        else:
            raise NotImplementedError("the gradient is implemented for VADU and LRAC")
        info["grad"] = grad
        info.update(ginfo)  # includes grad_F (offset) and, with a xi, grad_xi
    return nll, info


def _dprec_form(model, k, X, Y):
    """Column-wise X^T (d Sigma~^{-1} / d theta_k) Y by eq. (vecchiaSigmaderiv)."""
    BX, BY = model.B @ X, model.B @ Y
    dBX, dBY = model.dB[k] @ X, model.dB[k] @ Y
    Dinv = model.Dinv
    dD = model.dD[k]
    return np.sum(dBX * Dinv[:, None] * BY, axis=0) + np.sum(BX * Dinv[:, None] * dBY, axis=0) \
        - np.sum(BX * (Dinv * Dinv * dD)[:, None] * BY, axis=0)


def _grad_lrac(model, y, F, lik, aux, b, W, res, opts, P, replay_grad_cg):
    """Gradients of L^VLA (App. "Gradients of Vecchia-Laplace approximations")
    with the LRAC STE formulas and control variates (App. "Preconditioner
    LRAC").  With u = (Sigma~ + W^{-1})^{-1} z and v = P^{-1} z (z ~ N(0, P)),
    M = I + L^T W L and l_i = L_i M^{-1} L_i^T:
      mu_i: d log det / d mu_i = dW_i / W_i + c_i (dW_i l_i - dW_i / W_i)
            - mean(h - c_i r), h = u_i dW_i v_i / W_i^2, r = dW_i v_i^2 / W_i^2;
      theta_k: c tr(M^{-1} (dL^T W L + L^T W dL)) + mean(h - c r),
            h = -(Sigma~ u)^T dSigma~^{-1} (Sigma~ v), r = v^T (dL L^T + L dL^T) v;
      xi: as mu with dW/dxi summed over the rows.
    The mode's response uses w = A^{-1} dL/db* = W^{-1} (Sigma~ + W^{-1})^{-1}
    Sigma~ dL/db* (eq. pcls2), solved by PCG with P_LRAC."""
    if not hasattr(model, "dB"):
        raise ValueError("model built without derivatives")
    n = model.n
    U = res.U
    V = res.Z0
    L = P.L
    Minv = np.linalg.inv(P.M)
    lev = np.einsum("ij,jk,ik->i", L, Minv, L)
    mu = F + b
    parts = {}
    dW = lik_dW(lik, y, mu, aux)
    Wi2 = 1.0 / (W * W)
    h_mu = (dW * Wi2)[:, None] * U * V
    r_mu = (dW * Wi2)[:, None] * V * V
    c_mu = _cv_weight(h_mu, r_mu)
    dlogdet_dmu = dW / W + c_mu * (dW * lev - dW / W) - np.mean(h_mu - c_mu[:, None] * r_mu,
                                                                axis=1)
    dL_db = 0.5 * dlogdet_dmu
    parts.update(h_mu=h_mu, r_mu=r_mu, c_mu=c_mu, dlogdet_dmu=dlogdet_dmu, lev=lev)
    apply_S, apply_Pinv, _ = lrac_ops(model, W, L)
    if np.any(dL_db != 0.0):
        forced = None if replay_grad_cg is None else [replay_grad_cg]
        wres = pcg(apply_S, apply_Pinv, model.cov_apply(dL_db), opts.cg_tol, opts.max_cg, forced)
        wsol = wres.U / W
        parts["grad_cg_iters"] = int(wres.iters[0])
    else:
        wsol = np.zeros(n)
        parts["grad_cg_iters"] = 0
    parts["grad_F"] = -lik_grad(lik, y, mu, aux) + dL_db - W * wsol
    # theta: Sigma~ u and Sigma~ v, and the pivoted Cholesky's derivative
    # the pivot of column j is the row where the column takes its largest
    # value sqrt(d_p) (the residual covariance is bounded by its diagonal)
    piv = [int(np.argmax(np.abs(L[:, j]))) for j in range(L.shape[1])]
    _, dL, _ = pivoted_cholesky_deriv(model.coords, model.kind, model.theta, L.shape[1], piv)
    SU = model.cov_apply(U)
    SV = model.cov_apply(V)
    LV = L.T @ V
    Bb = model.B @ b
    grad = np.zeros(2)
    for k in range(2):
        h = -_dprec_form(model, k, SU, SV)
        r = 2.0 * np.sum(LV * (dL[k].T @ V), axis=0)
        c = float(_cv_weight(h, r))
        trP = 2.0 * np.trace(Minv @ (L.T @ (W[:, None] * dL[k])))
        dlogdet = c * trP + float(np.mean(h - c * r))
        quad_k = float(_dprec_form(model, k, b[:, None], b[:, None])[0])
        implicit = -float(wsol @ _dprec_apply(model, k, b, Bb))
        grad[k] = 0.5 * quad_k + 0.5 * dlogdet + implicit
        parts.update({f"dlogdet_{k}": dlogdet, f"quad_{k}": quad_k, f"implicit_{k}": implicit,
                      f"c_{k}": c, f"h_{k}": h, f"r_{k}": r, f"trP_{k}": trP})
    if lik_has_aux(lik):
        dWx = lik_dW_dxi(lik, y, mu, aux)
        h_xi = np.sum((dWx * Wi2)[:, None] * U * V, axis=0)
        r_xi = np.sum((dWx * Wi2)[:, None] * V * V, axis=0)
        c_xi = float(_cv_weight(h_xi, r_xi))
        trW = float(np.sum(dWx / W))
        trM = float(np.sum(dWx * lev))
        dlogdet_xi = trW + c_xi * (trM - trW) - float(np.mean(h_xi - c_xi * r_xi))
        dlogp_xi = float(np.sum(lik_dlogp_dxi(lik, y, mu, aux)))
        implicit_xi = float(wsol @ lik_dgrad_dxi(lik, y, mu, aux))
        parts.update(grad_xi=-dlogp_xi + 0.5 * dlogdet_xi + implicit_xi, h_xi=h_xi, r_xi=r_xi,
                     c_xi=c_xi, dlogdet_xi=dlogdet_xi, dlogp_xi=dlogp_xi,
                     implicit_xi=implicit_xi)
    return grad, parts


def _dprec_apply(model, k, x, Bx=None):
    """(d Sigma~^{-1} / d theta_k) x by eq. (vecchiaSigmaderiv):
    dB^T D^{-1} B x + B^T D^{-1} dB x - B^T D^{-1} dD D^{-1} B x."""
    Bx = model.B @ x if Bx is None else Bx
    dBx = model.dB[k] @ x
    dD = model.dD[k]
    Dinv = model.Dinv
    return model.dB[k].T @ (_col(Dinv, x) * Bx) + model.Bt @ (_col(Dinv, x) * dBx) \
        - model.Bt @ (_col(Dinv * Dinv * dD, x) * Bx)


def _cv_weight(h, r):
    """c = sample Cov(h, r) / sample Var(r); 0 when r is (numerically) constant."""
    t = h.shape[-1]
    rm = r.mean(axis=-1, keepdims=True)
    hm = h.mean(axis=-1, keepdims=True)
    var = np.sum((r - rm) ** 2, axis=-1) / (t - 1)
    cov = np.sum((h - hm) * (r - rm), axis=-1) / (t - 1)
    thresh = 1e-10 * rm[..., 0] ** 2
    safe = np.where(var > thresh, var, 1.0)
    return np.where(var > thresh, cov / safe, 0.0)


def _grad_theta_vadu(model, y, F, lik, aux, b, W, res, opts, replay_grad_cg):
    """theta-gradient of L^VLA (appendix "Gradients of Vecchia-Laplace
    approximations") with the VADU STE formulas and control variates."""
    if not hasattr(model, "dB"):
        raise ValueError("model built without derivatives")
    n = model.n
    t = opts.num_probes
    U = res.U                  # A^{-1} z_i
    V = res.Z0                 # P^{-1} z_i
    Dinv = model.Dinv
    wd = W + Dinv
    Bb = model.B @ b
    BU = model.B @ U
    BV = model.B @ V
    grad = np.zeros(2)
    parts = {}
    # d log det / d mu (VADU mu-formula), needed for the implicit term
    # d log det(Sigma~ W + I) / d mu_i = dW_i (A^{-1})_ii, estimated per probe
    # by h_i = dW_i (A^{-1}z)_i (P^{-1}z)_i; the control variate
    # r_i = dW_i (B P^{-1}z)_i^2 has the known mean tr(P^{-1} dP/dmu_i) =
    # dW_i / (W_i + 1/D_i), since dP/dmu_i = dW_i B_i^T B_i for P_VADU.
    dW = lik_dW(lik, y, F + b, aux)
    h_mu = dW[:, None] * U * V
    r_mu = dW[:, None] * BV * BV
    c_mu = _cv_weight(h_mu, r_mu)
    trP_mu = dW / wd
    dlogdet_dmu = c_mu * trP_mu + np.mean(h_mu - c_mu[:, None] * r_mu, axis=1)
    dL_db = 0.5 * dlogdet_dmu
    parts.update(h_mu=h_mu, r_mu=r_mu, c_mu=c_mu, trP_mu=trP_mu, dlogdet_dmu=dlogdet_dmu)
    apply_A, apply_Pinv = vadu_ops(model, W)
    if np.any(dL_db != 0.0):
        forced = None if replay_grad_cg is None else [replay_grad_cg]
        wres = pcg(apply_A, apply_Pinv, dL_db, opts.cg_tol, opts.max_cg, forced)
        wsol = wres.U
        parts["grad_cg_iters"] = int(wres.iters[0])
    else:
        wsol = np.zeros(n)
        parts["grad_cg_iters"] = 0
    # d L / d F (App. "Gradients of Vecchia-Laplace approximations"): the
    # explicit part -d log p / d mu + (1/2) d log det / d mu, plus the mode's
    # response (d L / d b*)^T d b* / d F_i with d b* / d F_i = -A^{-1} W e_i;
    # at the mode d L / d b* = (1/2) d log det / d mu (the other terms cancel),
    # so d L / d F = -g + dL_db - W o (A^{-1} dL_db).
    parts["grad_F"] = -lik_grad(lik, y, F + b, aux) + dL_db - W * wsol
    if lik_has_aux(lik):
        # d L / d xi (same appendix): -d log p / d xi + (1/2) d log det / d xi
        # + (d L / d b*)^T d b* / d xi with d b* / d xi = A^{-1} d^2 log p /
        # d xi d mu, i.e. w^T d^2 log p / d xi d mu (A symmetric).  The log
        # determinant's xi-derivative uses the VADU STE with
        # h = (A^{-1}z)^T dW/dxi P^{-1}z, control variate r = (P^{-1}z)^T B^T
        # dW/dxi B P^{-1}z and its known mean tr((W + D^{-1})^{-1} dW/dxi).
        mu = F + b
        dWx = lik_dW_dxi(lik, y, mu, aux)
        h_xi = np.sum(dWx[:, None] * U * V, axis=0)
        r_xi = np.sum(dWx[:, None] * BV * BV, axis=0)
        c_xi = float(_cv_weight(h_xi, r_xi))
        trP_xi = float(np.sum(dWx / wd))
        dlogdet_xi = c_xi * trP_xi + float(np.mean(h_xi - c_xi * r_xi))
        dlogp_xi = float(np.sum(lik_dlogp_dxi(lik, y, mu, aux)))
        implicit_xi = float(wsol @ lik_dgrad_dxi(lik, y, mu, aux))
        parts.update(grad_xi=-dlogp_xi + 0.5 * dlogdet_xi + implicit_xi, h_xi=h_xi, r_xi=r_xi,
                     c_xi=c_xi, trP_xi=trP_xi, dlogdet_xi=dlogdet_xi, dlogp_xi=dlogp_xi,
                     implicit_xi=implicit_xi)
    for k in range(2):
        dD = model.dD[k]
        dBb = model.dB[k] @ b
        quad_k = 2.0 * np.sum(dBb * Dinv * Bb) - np.sum(Bb * Dinv * Dinv * dD * Bb)
        dBU = model.dB[k] @ U
        dBV = model.dB[k] @ V
        h = np.sum(dBU * Dinv[:, None] * BV, axis=0) + np.sum(BU * Dinv[:, None] * dBV, axis=0) \
            - np.sum(BU * (Dinv * Dinv * dD)[:, None] * BV, axis=0)
        r = 2.0 * np.sum(dBV * wd[:, None] * BV, axis=0) \
            - np.sum(BV * (Dinv * Dinv * dD)[:, None] * BV, axis=0)
        c = float(_cv_weight(h, r))
        tr_D = np.sum(dD * Dinv)
        tr_P = -np.sum(Dinv * Dinv * dD / wd)
        dlogdet = tr_D + c * tr_P + np.mean(h - c * r)
        implicit = -float(wsol @ _dprec_apply(model, k, b, Bb))
        grad[k] = 0.5 * quad_k + 0.5 * dlogdet + implicit
        parts[f"dlogdet_{k}"] = dlogdet
        parts[f"quad_{k}"] = quad_k
        parts[f"implicit_{k}"] = implicit
        parts[f"c_{k}"] = c
        parts[f"h_{k}"] = h
        parts[f"r_{k}"] = r
        parts[f"trP_{k}"] = tr_P
    return grad, parts


# ----------------------------------------------------------------------------
# prediction, eq. (latentpostpredictive) and Alg. simAlgo
# ----------------------------------------------------------------------------
def predict(model, coords_p, Fp, b, W, opts, replay_cg=None, chunk=256,
            want_var=True, col0=0):
    """Predictive latent means and simulated variances at coords_p.

    omega_p = F_p + A_p b*  (B_p = I, B_po = -A_p);
    diag Omega_p ~= D_p + (1/s) sum_i (A_p u_i)^2,  u_i = (W + Sigma~^{-1})^{-1}
    z3_i,  z3_i = W^{1/2} z1_i + B^T D^{-1/2} z2_i  (Alg. simAlgo).
    Sample columns are independent; they are processed in chunks of `chunk`
    columns, which does not change any column's arithmetic.  The samples are
    the counter-based columns col0 .. col0 + s - 1 (col0 > 0: a slice of a
    larger sample set; info["acc"] holds its unnormalised sum of squares)."""
    coords_p = np.asarray(coords_p, dtype=np.float64)
    npred = coords_p.shape[0]
    nbr_p = _vec.pred_neighbours(model.coords, coords_p, model.m)
    Ap, Dp = _vec.factor(model.coords, nbr_p, model.kind, model.theta, coords_self=coords_p)
    Bpo = _vec.sparse_offdiag(-Ap, nbr_p, model.n)
    Fp = np.zeros(npred) if Fp is None else np.asarray(Fp, dtype=np.float64)
    mean = Fp - Bpo @ b
    info = {"nbr_p": nbr_p, "Ap": Ap, "Dp": Dp}
    if not want_var:
        return mean, None, info
    s = opts.num_pred_samples
    n = model.n
    apply_A, apply_Pinv = vadu_ops(model, W)
    acc = np.zeros(npred)
    iters = np.zeros(s, dtype=np.int64)
    for c0 in range(0, s, chunk):
        c1 = min(s, c0 + chunk)
        z1 = _gaussian_cols(opts.seed, _rng.TAG_PRED_Z1, n, col0 + c0, col0 + c1)
        z2 = _gaussian_cols(opts.seed, _rng.TAG_PRED_Z2, n, col0 + c0, col0 + c1)
        z3 = np.sqrt(W)[:, None] * z1 + model.Bt @ (np.sqrt(model.Dinv)[:, None] * z2)
        forced = None if replay_cg is None else replay_cg[c0:c1]
        res = pcg(apply_A, apply_Pinv, z3, opts.pred_cg_tol, opts.max_cg, forced)
        z4 = Bpo @ res.U
        acc += np.sum(z4 * z4, axis=1)
        iters[c0:c1] = res.iters
    var = Dp + acc / s
    info["cg_iters"] = iters
    info["acc"] = acc
    return mean, var, info


PRED_LANCZOS_L1 = 1   # P_L1 = B^T (W + D^{-1}) B (Sec. 3.3.2)
PRED_LANCZOS_L2 = 2   # P_L2 = diag(Sigma + W^{-1}) on Sigma~ + W^{-1} (Sec. 3.3.2)
LANCZOS_BREAKDOWN = 1e-13


def lanczos_full_reorth(apply_M, q1, k):
    """k steps of the symmetric Lanczos process on M from the direction q1,
    with complete reorthogonalization (each new vector is orthogonalised
    against all previous Lanczos vectors by classical Gram-Schmidt, applied
    twice; Golub & Van Loan, Matrix Computations, Sec. 10.3.1).

    Step j: w = M q_j; alpha_j = q_j^T w; w -= Q_j (Q_j^T w) twice;
    beta_j = |w|; q_{j+1} = w / beta_j.  Stops early when beta_j <=
    LANCZOS_BREAKDOWN max|alpha| (an invariant subspace).  Returns Q (n x k')
    and the k' x k' tridiagonal T = tridiag(beta, alpha, beta)."""
    n = q1.shape[0]
    Q = np.zeros((n, k))
    alpha, beta = [], []
    Q[:, 0] = q1 / np.linalg.norm(q1)
    kk = k
    for j in range(k):
        w = apply_M(Q[:, j])
        Qj = Q[:, :j + 1]
        c = Qj.T @ w
        alpha.append(float(c[j]))
        w = w - Qj @ c
        w = w - Qj @ (Qj.T @ w)
        if j + 1 == k:
            break
        bj = float(np.linalg.norm(w))
        if bj <= LANCZOS_BREAKDOWN * max(abs(a) for a in alpha):
            kk = j + 1
            break
        beta.append(bj)
        Q[:, j + 1] = w / bj
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    return Q[:, :kk], T


def predict_lanczos(model, coords_p, Fp, b, W, k, precond):
    """Predictive latent means and Lanczos predictive variances (Sec. 3.3.2).

    omega_p as in predict; diag Omega_p ~= D_p + diag(B_po X B_po^T) with X
    the rank-k preconditioned Lanczos approximation of (W + Sigma~^{-1})^{-1}:
      P_L1: M = P^{-1/2} A P^{-T/2}, P^{-1/2} = (W + D^{-1})^{-1/2} B^{-T}
            (eq. P_VADU_prec), X = P^{-T/2} Q T^{-1} Q^T P^{-1/2};
      P_L2: M = P^{-1/2} (Sigma~ + W^{-1}) P^{-1/2}, P = diag(sigma^2 + 1/W)
            (diag Sigma = sigma^2 standing in for diag Sigma~),
            X = W^{-1} P^{-1/2} Q T^{-1} Q^T P^{-1/2} Sigma~.
    The Lanczos process starts from the average column x of B_po^T mapped
    into M's coordinates: P^{-1/2} x (P_L1), P^{-1/2} Sigma~ x (P_L2)."""
    coords_p = np.asarray(coords_p, dtype=np.float64)
    npred = coords_p.shape[0]
    nbr_p = _vec.pred_neighbours(model.coords, coords_p, model.m)
    Ap, Dp = _vec.factor(model.coords, nbr_p, model.kind, model.theta, coords_self=coords_p)
    Bpo = _vec.sparse_offdiag(-Ap, nbr_p, model.n)
    Fp = np.zeros(npred) if Fp is None else np.asarray(Fp, dtype=np.float64)
    mean = Fp - Bpo @ b
    xbar = (Bpo.T @ np.ones(npred)) / npred
    if precond == PRED_LANCZOS_L1:
        s = 1.0 / np.sqrt(W + model.Dinv)

        def apply_M(q):
            y = model.solve_B(s * q)
            return s * model.solve_Bt(W * y + model.prec_apply(y))

        Q, T = lanczos_full_reorth(apply_M, s * model.solve_Bt(xbar), k)
        G = Bpo @ model.solve_B(s[:, None] * Q)
        var = Dp + np.sum(G * np.linalg.solve(T, G.T).T, axis=1)
    elif precond == PRED_LANCZOS_L2:
        s = 1.0 / np.sqrt(model.theta[0] + 1.0 / W)

        def apply_M(q):
            y = s * q
            return s * (model.cov_apply(y) + y / W)

        Q, T = lanczos_full_reorth(apply_M, s * model.cov_apply(xbar), k)
        G1 = Bpo @ ((s / W)[:, None] * Q)
        G2 = Bpo @ model.cov_apply(s[:, None] * Q)
        var = Dp + np.sum(G1 * np.linalg.solve(T, G2.T).T, axis=1)
    else:
        raise ValueError("unknown Lanczos preconditioner")
    return mean, var, {"nbr_p": nbr_p, "Ap": Ap, "Dp": Dp, "Q": Q, "T": T,
                       "rank": Q.shape[1]}


def _gaussian_cols(seed, tag, n, c0, c1):
    """Columns c0..c1-1 of the n x s Gaussian probe matrix."""
    return _rng.gaussian(seed, tag, n, c1 - c0, col0=c0)


# ----------------------------------------------------------------------------
# estimation of theta (Sec. 4.1: L-BFGS with a sample average approximation)
# ----------------------------------------------------------------------------
def estimate(coords, m, kind, y, F, lik, aux, theta0, opts, nbr=None, gtol=1e-6, maxiter=100):
    """theta minimising L^VLA with the probes of opts.seed in every evaluation
    (so the objective is deterministic), over log theta by scipy's L-BFGS-B.
    Each evaluation: the factor at theta, the mode from b = 0, the SLQ
    likelihood and its STE gradient.  Returns (theta, nll, scipy result)."""
    from scipy.optimize import minimize

    coords = np.asarray(coords, dtype=np.float64)
    nbr = _vec.neighbours(coords, m) if nbr is None else nbr

    def fun(x):
        theta = np.exp(x)
        model = Model(coords, m, kind, theta, nbr=nbr, deriv=True)
        b, _, _ = find_mode(model, y, F, lik, aux, opts)
        nll, info = neg_log_marglik(model, y, F, lik, aux, b, opts, want_grad=True)
        return nll, info["grad"] * theta  # gradient in log theta

    res = minimize(fun, np.log(np.asarray(theta0, dtype=np.float64)), jac=True,
                   method="L-BFGS-B", options={"gtol": gtol, "ftol": 1e-15, "maxiter": maxiter})
    return np.exp(res.x), float(res.fun), res


def glm_params_to_x(theta, aux, beta, lik):
    """Search coordinates (log sigma2, log rho, [log xi], beta)."""
    x = [np.log(theta[0]), np.log(theta[1])]
    if lik_has_aux(lik):
        x.append(np.log(aux))
    return np.concatenate([np.asarray(x), np.asarray(beta, dtype=np.float64)])


def estimate_glm(coords, m, kind, y, X, lik, theta0, aux0, beta0, opts, nbr=None, gtol=1e-6,
                 maxiter=200):
    """Joint estimate of theta, the likelihood's auxiliary parameter xi (when
    it has one) and the coefficients beta of F = X beta (Sec. 2; Sec. 5's
    estimation of the shape, the covariance parameters and beta), by scipy's
    L-BFGS-B over (log sigma2, log rho, log xi, beta) with the probes of
    opts.seed in every evaluation.  The gradient: theta- and xi-gradients
    (STE, App. "Gradients of Vecchia-Laplace approximations") times the
    parameter (log scale), and X^T dL/dF for beta.
    Returns (theta, xi or None, beta, nll, scipy result)."""
    from scipy.optimize import minimize

    coords = np.asarray(coords, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    nbr = _vec.neighbours(coords, m) if nbr is None else nbr
    has_aux = lik_has_aux(lik)
    q = 3 if has_aux else 2

    def unpack(x):
        theta = np.exp(x[:2])
        aux = float(np.exp(x[2])) if has_aux else None
        return theta, aux, x[q:]

    def fun(x):
        theta, aux, beta = unpack(x)
        F = X @ beta
        model = Model(coords, m, kind, theta, nbr=nbr, deriv=True)
        b, _, _ = find_mode(model, y, F, lik, aux, opts)
        nll, info = neg_log_marglik(model, y, F, lik, aux, b, opts, want_grad=True)
        g = [info["grad"][0] * theta[0], info["grad"][1] * theta[1]]
        if has_aux:
            g.append(info["grad_xi"] * aux)
        return nll, np.concatenate([np.asarray(g), X.T @ info["grad_F"]])

    res = minimize(fun, glm_params_to_x(theta0, aux0, beta0, lik), jac=True, method="L-BFGS-B",
                   options={"gtol": gtol, "ftol": 1e-15, "maxiter": maxiter})
    theta, aux, beta = unpack(res.x)
    return theta, aux, beta, float(res.fun), res


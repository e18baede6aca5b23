"""Pins for the Laplace / CG / SLQ / STE / LRAC / prediction part of the oracle.

Each test checks the oracle against something other than itself: a dense
direct computation that the iterative method reaches in a special case, a
closed form, a theorem of the paper, finite differences, or a statistical
bound.  Sizes are tiny so the whole file runs in seconds."""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import laplace as L
from oracle import laplace as L_
from oracle import rng as R
from oracle import vecchia as V
from tests import dense_ref as DR


def _problem(n=80, m=6, kind=V.COV_EXPONENTIAL, theta=(1.0, 0.2), lik=L.LIK_BERNOULLI_LOGIT,
             seed=0, deriv=False, F=0.0):
    g = np.random.default_rng(seed)
    X = g.uniform(size=(n, 2))
    S = V.dense_covariance(X, kind, *theta)
    b = np.linalg.cholesky(S + 1e-10 * np.eye(n)) @ g.standard_normal(n)
    Fv = np.full(n, F)
    if lik == L.LIK_BERNOULLI_LOGIT:
        y = (g.uniform(size=n) < 1 / (1 + np.exp(-(Fv + b)))).astype(float)
    elif lik == L.LIK_POISSON:
        y = g.poisson(np.exp(Fv + b)).astype(float)
    elif lik == L.LIK_GAMMA:
        y = g.gamma(2.5, np.exp(Fv + b) / 2.5)
    else:
        y = Fv + b + 0.5 * g.standard_normal(n)
    model = L.Model(X, m, kind, theta, deriv=deriv)
    return model, y, Fv


def _liks(lik, aux=None):
    return (lambda y, mu: L.lik_logp(lik, y, mu, aux),
            lambda y, mu: L.lik_grad(lik, y, mu, aux),
            lambda y, mu: L.lik_W(lik, y, mu, aux))


# ---------------------------------------------------------------- likelihoods
@pytest.mark.parametrize("lik,aux,y", [(L.LIK_BERNOULLI_LOGIT, None, np.array([0.0, 1.0, 1.0, 0.0])),
                                       (L.LIK_POISSON, None, np.array([0.0, 3.0, 7.0, 1.0])),
                                       (L.LIK_GAUSSIAN, 0.3, np.array([0.2, -1.0, 2.0, 0.0])),
                                       (L.LIK_GAMMA, 2.5, np.array([0.3, 1.7, 4.0, 0.05]))])
def test_likelihood_derivatives_finite_differences(lik, aux, y):
    mu = np.array([-1.3, 0.2, 1.1, 2.5])
    h = 1e-5
    fd1 = (L.lik_logp(lik, y, mu + h, aux) - L.lik_logp(lik, y, mu - h, aux)) / (2 * h)
    fd2 = (L.lik_grad(lik, y, mu + h, aux) - L.lik_grad(lik, y, mu - h, aux)) / (2 * h)
    fd3 = (L.lik_W(lik, y, mu + h, aux) - L.lik_W(lik, y, mu - h, aux)) / (2 * h)
    np.testing.assert_allclose(L.lik_grad(lik, y, mu, aux), fd1, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(L.lik_W(lik, y, mu, aux), -fd2, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(L.lik_dW(lik, y, mu, aux), fd3, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("lik,aux,y", [(L.LIK_GAUSSIAN, 0.3, np.array([0.2, -1.0, 2.0, 0.0])),
                                       (L.LIK_GAMMA, 2.5, np.array([0.3, 1.7, 4.0, 0.05])),
                                       (L.LIK_GAMMA, 0.6, np.array([0.3, 1.7, 4.0, 0.05]))])
def test_likelihood_xi_derivatives_finite_differences(lik, aux, y):
    # derivatives in the auxiliary parameter (tau^2, Gamma shape) against
    # central differences of log p, d log p / d mu and W in xi
    mu = np.array([-1.3, 0.2, 1.1, 2.5])
    h = 1e-6 * aux
    d = lambda f: (f(lik, y, mu, aux + h) - f(lik, y, mu, aux - h)) / (2 * h)  # noqa: E731
    np.testing.assert_allclose(L.lik_dlogp_dxi(lik, y, mu, aux), d(L.lik_logp), rtol=1e-7,
                               atol=1e-8)
    np.testing.assert_allclose(L.lik_dgrad_dxi(lik, y, mu, aux), d(L.lik_grad), rtol=1e-7,
                               atol=1e-8)
    np.testing.assert_allclose(L.lik_dW_dxi(lik, y, mu, aux), d(L.lik_W), rtol=1e-7, atol=1e-8)
    assert not L.lik_has_aux(L.LIK_POISSON) and not L.lik_has_aux(L.LIK_BERNOULLI_LOGIT)


def test_likelihood_normalisation():
    # Poisson and Bernoulli probabilities sum to one over y; the Gaussian
    # log-density integrates to one (full constants included).
    mu = 0.7
    ys = np.arange(0, 80, dtype=float)
    assert abs(np.sum(np.exp(L.lik_logp(L.LIK_POISSON, ys, np.full_like(ys, mu)))) - 1) < 1e-12
    pb = np.exp(L.lik_logp(L.LIK_BERNOULLI_LOGIT, np.array([0.0, 1.0]), np.full(2, mu)))
    assert abs(pb.sum() - 1) < 1e-14
    x = np.linspace(-10, 10, 200001)
    dens = np.exp(L.lik_logp(L.LIK_GAUSSIAN, x, np.zeros_like(x), 0.4))
    assert abs(np.trapezoid(dens, x) - 1) < 1e-8


# ------------------------------------------------------------------------ CG
def test_pcg_solves_and_lanczos_ritz_values():
    model, y, F = _problem(n=60)
    W = L.lik_W(L.LIK_BERNOULLI_LOGIT, y, np.zeros(60))
    apply_A, apply_Pinv = L.vadu_ops(model, W)
    Ad = apply_A(np.eye(60))
    Pinv = apply_Pinv(np.eye(60))
    rhs = np.random.default_rng(1).standard_normal((60, 3))
    res = L.pcg(apply_A, apply_Pinv, rhs, 1e-12, 200)
    np.testing.assert_allclose(res.U, np.linalg.solve(Ad, rhs), rtol=1e-9, atol=1e-10)
    # Ritz values of T~ lie in the spectrum range of P^{-1}A and the extreme
    # ones converge to its extreme eigenvalues (CG-Lanczos relation).
    lam = np.sort(np.linalg.eigvals(Pinv @ Ad).real)
    for c in range(3):
        T = L.lanczos_tridiag(res.alphas[c], res.betas[c])
        ritz = np.linalg.eigvalsh(T)
        assert ritz.min() >= lam[0] * (1 - 1e-8) and ritz.max() <= lam[-1] * (1 + 1e-8)
        assert abs(ritz.max() - lam[-1]) < 1e-6 * lam[-1]
        # Gauss quadrature for f(x) = 1/x: b^T u_l = (r0^T z0) e1^T T~^{-1} e1
        assert abs(rhs[:, c] @ res.U[:, c] - res.r0z0[c] * np.linalg.inv(T)[0, 0]) \
            < 1e-10 * abs(rhs[:, c] @ res.U[:, c])


@pytest.mark.parametrize("precond", [L.PRECOND_VADU, L.PRECOND_LVA, L.PRECOND_DIAG])
def test_slq_equals_dense_hutchinson_at_convergence(precond):
    # Run to full convergence: Gauss quadrature is exact, so the SLQ term equals
    # (1/t) sum eps^T log(M) eps with M = P^{-1/2} A P^{-T/2}:
    # VADU P^{-1/2} = (W + D^{-1})^{-1/2} B^{-T} (eq. P_VADU_prec), LVA
    # D^{1/2} B^{-T}, P_1 diag(A)^{-1/2} (Sec. 3.1.4), all built densely here.
    n = 50
    model, y, F = _problem(n=n, m=5, seed=3)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, L.Opts(cg_tol=1e-13))
    opts = L.Opts(cg_tol=1e-13, num_probes=7, seed=5, precond=precond)
    nll, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, opts)
    Bd = model.B.toarray()
    Q = DR.dense_precision(Bd, model.D)
    A = np.diag(W) + Q
    if precond == L.PRECOND_VADU:
        Pih = np.diag((W + model.Dinv) ** -0.5) @ np.linalg.inv(Bd).T
        ld_P = np.sum(np.log(W + model.Dinv))
    elif precond == L.PRECOND_LVA:
        Pih = np.diag(model.D ** 0.5) @ np.linalg.inv(Bd).T
        ld_P = -np.sum(np.log(model.D))
    else:
        np.testing.assert_allclose(L.diag_p1(model, W), np.diag(A), rtol=1e-13)
        Pih = np.diag(np.diag(A) ** -0.5)
        ld_P = np.sum(np.log(np.diag(A)))
    # the fixed part of eq. (logdetsplit): log det Sigma~ + log det P
    np.testing.assert_allclose(info["logdet"] - info["gamma"], np.sum(np.log(model.D)) + ld_P,
                               rtol=1e-12, atol=1e-10)
    M = Pih @ A @ Pih.T
    Lm = DR.logm_spd(M)
    eps = R.rademacher(5, R.TAG_SLQ, n, 7)
    hutch = np.mean(np.einsum("ij,ik,kj->j", eps, Lm, eps))
    assert abs(info["gamma"] - hutch) < 1e-9 * max(1.0, abs(hutch))
    # weights: r0^T z0 = ||P^{-1/2} z||^2 = eps^T eps = n (Rademacher)
    np.testing.assert_allclose(info["r0z0"], n, rtol=1e-12)


def test_slq_statistical_bound():
    # Thm 3.2 scale: the SLQ estimate lies within 5 standard deviations of the
    # exact log det M; the Rademacher Hutchinson variance is
    # 2 sum_{a != b} (log M)_ab^2 / t.
    n, t = 70, 40
    model, y, F = _problem(n=n, m=6, seed=4, kind=V.COV_MATERN32, theta=(1.0, 0.15))
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, L.Opts(cg_tol=1e-12))
    opts = L.Opts(cg_tol=1e-12, num_probes=t, seed=9)
    _, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, opts)
    Bd = model.B.toarray()
    A = np.diag(W) + DR.dense_precision(Bd, model.D)
    Pih = np.diag((W + model.Dinv) ** -0.5) @ np.linalg.inv(Bd).T
    Lm = DR.logm_spd(Pih @ A @ Pih.T)
    off = Lm - np.diag(np.diag(Lm))
    sd = np.sqrt(2.0 * np.sum(off ** 2) / t)
    assert abs(info["gamma"] - np.trace(Lm)) <= 5 * sd + 1e-9


def test_vadu_identity_factor_special_case():
    # m = 0 gives B = I, so P_VADU = W + D^{-1} = A: CG stops after one
    # iteration with T~ = [1] and the SLQ term vanishes (Sec. 3.1.1).
    n = 40
    model, y, F = _problem(n=n, m=0, seed=2)
    b, W, st = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, L.Opts(cg_tol=1e-10))
    assert all(c == 1 for c in st["cg_iters"])
    opts = L.Opts(cg_tol=1e-10, num_probes=5)
    nll, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, opts)
    assert np.all(info["cg_iters"] == 1)
    assert abs(info["gamma"]) < 1e-12
    np.testing.assert_allclose(info["logdet"], np.sum(np.log(1.0 + model.theta[0] * W)), rtol=1e-12)


def test_theorem_3_1_eigenvalue_bounds():
    # lambda_min(P^{-1}A) > min (D_i W_ii + 1)^{-1};
    # lambda_l(P^{-1}A) <= (lambda_l(Sigma~) max W + 1) max (D_i W_ii + 1)^{-1}.
    n = 90
    model, y, F = _problem(n=n, m=5, seed=6, lik=L.LIK_POISSON, F=0.5)
    b, W, _ = L.find_mode(model, y, F, L.LIK_POISSON, None, L.Opts(cg_tol=1e-10))
    apply_A, apply_Pinv = L.vadu_ops(model, W)
    lam = np.sort(np.linalg.eigvals(apply_Pinv(np.eye(n)) @ apply_A(np.eye(n))).real)[::-1]
    Bd = model.B.toarray()
    Binv = np.linalg.inv(Bd)
    St = Binv @ np.diag(model.D) @ Binv.T
    lS = np.sort(np.linalg.eigvalsh(St))[::-1]
    q = 1.0 / (model.D * W + 1.0)
    assert lam[-1] > q.min() * (1 - 1e-10)
    assert np.all(lam <= (lS * W.max() + 1.0) * q.max() * (1 + 1e-9))


def test_theorem_3_1_lva_eigenvalue_bounds():
    # LVA: lambda_min(P^{-1}A) > 1 and lambda_l(P^{-1}A) <= lambda_l(Sigma~) max W + 1
    # (P_LVA^{-1/2} A P_LVA^{-T/2} = D^{1/2} B^{-T} W B^{-1} D^{1/2} + I).
    n = 90
    model, y, F = _problem(n=n, m=5, seed=6, lik=L.LIK_POISSON, F=0.5)
    b, W, _ = L.find_mode(model, y, F, L.LIK_POISSON, None, L.Opts(cg_tol=1e-10))
    apply_A, apply_Pinv = L.lva_ops(model, W)
    lam = np.sort(np.linalg.eigvals(apply_Pinv(np.eye(n)) @ apply_A(np.eye(n))).real)[::-1]
    Binv = np.linalg.inv(model.B.toarray())
    lS = np.sort(np.linalg.eigvalsh(Binv @ np.diag(model.D) @ Binv.T))[::-1]
    assert lam[-1] > 1.0 - 1e-10
    assert np.all(lam <= (lS * W.max() + 1.0) * (1 + 1e-9))


def test_diagonal_preconditioner_identity_factor_special_case():
    # m = 0: B = I, so P_1 = W + D^{-1} = A; CG stops after one iteration,
    # T~ = [1], the SLQ term vanishes and log det = sum log(1 + sigma^2 W).
    n = 40
    model, y, F = _problem(n=n, m=0, seed=2)
    o = L.Opts(cg_tol=1e-10, num_probes=5, precond=L.PRECOND_DIAG)
    b, W, st = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, o)
    assert all(c == 1 for c in st["cg_iters"])
    nll, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, o)
    assert np.all(info["cg_iters"] == 1) and abs(info["gamma"]) < 1e-12
    np.testing.assert_allclose(info["logdet"], np.sum(np.log(1.0 + model.theta[0] * W)), rtol=1e-12)


# --------------------------------------------------------------------- Newton
@pytest.mark.parametrize("lik", [L.LIK_BERNOULLI_LOGIT, L.LIK_POISSON])
def test_mode_equals_dense_newton_and_zero_gradient(lik):
    model, y, F = _problem(n=100, m=7, lik=lik, seed=7, F=(0.3 if lik == L.LIK_POISSON else 0.0))
    b, W, st = L.find_mode(model, y, F, lik, None, L.Opts(cg_tol=1e-12, newton_tol=1e-14))
    Q = DR.dense_precision(model.B, model.D)
    lp, lg, lw = _liks(lik)
    bd = DR.dense_mode(Q, y, F, lg, lw)
    np.testing.assert_allclose(b, bd, rtol=1e-8, atol=1e-10)
    # first-order condition of the mode: d log p / d b = Sigma~^{-1} b*
    np.testing.assert_allclose(lg(y, F + b), Q @ b, atol=1e-8)


def test_step_halving_reaches_the_mode_where_full_newton_diverges():
    # Poisson counts of a strong field (sigma2 = 4, F = 1): a full first
    # Newton step from b = 0 overshoots (Psi falls); with step halving the
    # iteration still reaches the point where d log p / d b = Sigma~^{-1} b.
    model, y, F = _problem(n=120, m=8, lik=L.LIK_POISSON, seed=21, theta=(4.0, 0.2), F=1.0)
    opts = L.Opts(cg_tol=1e-12, newton_tol=1e-15, max_newton=200)
    b0 = np.zeros(model.n)
    g0 = L.lik_grad(L.LIK_POISSON, y, F)
    W0 = L.lik_W(L.LIK_POISSON, y, F)
    A, Pinv = L.vadu_ops(model, W0)
    full = np.ravel(L.pcg(A, Pinv, W0 * b0 + g0, 1e-12, 1000).U)
    assert L.psi(model, y, F, full, L.LIK_POISSON, None) < L.psi(model, y, F, b0, L.LIK_POISSON, None)
    b, W, st = L.find_mode(model, y, F, L.LIK_POISSON, None, opts)
    assert st["halvings"][0] > 0
    Q = DR.dense_precision(model.B, model.D)
    np.testing.assert_allclose(L.lik_grad(L.LIK_POISSON, y, F + b), Q @ b, atol=1e-8)


@pytest.mark.parametrize("precond", [L.PRECOND_LRAC, L.PRECOND_LVA, L.PRECOND_DIAG])
def test_mode_other_preconditioners_equal_mode_vadu(precond):
    model, y, F = _problem(n=90, m=6, seed=8)
    o1 = L.Opts(cg_tol=1e-12, newton_tol=1e-14)
    o2 = L.Opts(cg_tol=1e-12, newton_tol=1e-14, precond=precond, lrac_rank=10)
    b1, _, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, o1)
    b2, _, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, o2)
    np.testing.assert_allclose(b1, b2, rtol=1e-8, atol=1e-9)


# ------------------------------------------------------------------------ NLL
def test_gaussian_likelihood_exact_marginal():
    # Laplace is exact for a Gaussian likelihood: with the SLQ term replaced by
    # the exact log det M, the NLL equals -log N(y; F, Sigma~ + tau2 I).
    n, tau2 = 60, 0.25
    model, y, F = _problem(n=n, m=5, lik=L.LIK_GAUSSIAN, seed=10)
    opts = L.Opts(cg_tol=1e-12, newton_tol=1e-15, num_probes=4)
    b, W, _ = L.find_mode(model, y, F, L.LIK_GAUSSIAN, tau2, opts)
    nll, info = L.neg_log_marglik(model, y, F, L.LIK_GAUSSIAN, tau2, b, opts)
    Bd = model.B.toarray()
    Q = DR.dense_precision(Bd, model.D)
    _, ldA = np.linalg.slogdet(np.diag(W) + Q)
    exact_gamma = ldA - np.sum(np.log(W + model.Dinv)) + 2 * np.sum(np.log(np.diag(Bd)))
    nll_exact = nll - 0.5 * info["gamma"] + 0.5 * exact_gamma
    St = np.linalg.inv(Q)
    ref = -multivariate_normal(mean=F, cov=St + tau2 * np.eye(n)).logpdf(y)
    assert abs(nll_exact - ref) < 1e-8 * abs(ref)


@pytest.mark.parametrize("precond", [L.PRECOND_VADU, L.PRECOND_LRAC, L.PRECOND_LVA,
                                     L.PRECOND_DIAG])
def test_logdet_matches_dense_within_probe_error(precond):
    # log det(Sigma~ W + I) estimated with t probes lies within 5 standard
    # errors (sample sd of the per-probe terms / sqrt t) of the dense value.
    n, t = 80, 64
    model, y, F = _problem(n=n, m=6, seed=11, kind=V.COV_MATERN32, theta=(1.0, 0.2))
    opts = L.Opts(cg_tol=1e-11, newton_tol=1e-14, num_probes=t, seed=3, precond=precond,
                  lrac_rank=12)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, opts)
    nll, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, opts)
    Q = DR.dense_precision(model.B, model.D)
    _, ld1 = np.linalg.slogdet(np.diag(W) + Q)
    _, ld0 = np.linalg.slogdet(Q)
    exact = ld1 - ld0
    per_probe = info["r0z0"] * info["quad"]
    se = np.std(per_probe, ddof=1) / np.sqrt(t)
    assert abs(info["logdet"] - exact) <= 5 * se + 1e-8


def test_lrac_full_rank_special_case():
    # k = n and m = n-1: L L^T = Sigma = Sigma~, so P_LRAC equals the operator
    # Sigma~ + W^{-1}; CG converges in one iteration and log det P matches
    # slogdet(Sigma + W^{-1}) (Woodbury / determinant lemma, Sec. 3.1.2).
    n = 40
    model, y, F = _problem(n=n, m=n - 1, seed=12)
    Lk = L.pivoted_cholesky(model.coords, model.kind, model.theta, n)
    S = V.dense_covariance(model.coords, model.kind, *model.theta)
    np.testing.assert_allclose(Lk @ Lk.T, S, atol=1e-9)
    W = L.lik_W(L.LIK_BERNOULLI_LOGIT, y, np.full(n, 0.3))
    apply_A, apply_Pinv, P = L.lrac_ops(model, W, Lk)
    _, ref = np.linalg.slogdet(S + np.diag(1.0 / W))
    assert abs(P.logdet - ref) < 1e-9 * abs(ref)
    res = L.pcg(apply_A, apply_Pinv, np.random.default_rng(0).standard_normal(n), 1e-7, 50)
    assert res.iters[0] == 1


def test_pivoted_cholesky_pivots_and_residual():
    # pivots pick the largest residual diagonal; the residual trace decreases
    n = 60
    X = np.random.default_rng(13).uniform(size=(n, 2))
    S = V.dense_covariance(X, V.COV_MATERN32, 1.0, 0.3)
    prev = np.trace(S)
    for k in (1, 5, 20):
        Lk = L.pivoted_cholesky(X, V.COV_MATERN32, (1.0, 0.3), k)
        Rm = S - Lk @ Lk.T
        assert np.all(np.linalg.eigvalsh(Rm) > -1e-10)     # Sigma - L L^T is PSD
        assert np.trace(Rm) < prev
        prev = np.trace(Rm)
    assert np.argmax(np.abs(L.pivoted_cholesky(X, V.COV_MATERN32, (1.0, 0.3), 1)[:, 0])) == 0


# ------------------------------------------------------------------- gradient
def _dense_vl_nll(X, nbr, kind, theta, y, F, lik):
    A, D = V.factor(X, nbr, kind, theta)
    Q = DR.dense_precision(V.sparse_B(A, nbr), D)
    lp, lg, lw = _liks(lik)
    return DR.dense_nll(Q, y, F, lp, lg, lw)[0]


@pytest.mark.parametrize("kind", [V.COV_EXPONENTIAL, V.COV_MATERN32])
def test_theta_gradient_matches_finite_differences(kind):
    # STE gradient with VADU control variates (App. A.3, A.4.1) against central
    # differences of the exact (dense) Vecchia-Laplace NLL, within 5 standard
    # errors over independent probe sets.
    n, m = 45, 5
    model, y, F = _problem(n=n, m=m, seed=14, kind=kind, theta=(1.2, 0.25), deriv=True)
    opts0 = L.Opts(cg_tol=1e-12, newton_tol=1e-15)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, opts0)
    grads = []
    for seed in range(8):
        opts = L.Opts(cg_tol=1e-12, newton_tol=1e-15, num_probes=400, seed=seed)
        _, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, opts,
                                    want_grad=True)
        grads.append(info["grad"])
    grads = np.array(grads)
    g_mean = grads.mean(axis=0)
    g_se = grads.std(axis=0, ddof=1) / np.sqrt(len(grads))
    fd = []
    for k, h in enumerate([1e-5, 1e-6]):
        e = np.zeros(2)
        e[k] = h
        th = np.array(model.theta)
        fp = _dense_vl_nll(model.coords, model.nbr, kind, th + e, y, F, L.LIK_BERNOULLI_LOGIT)
        fm = _dense_vl_nll(model.coords, model.nbr, kind, th - e, y, F, L.LIK_BERNOULLI_LOGIT)
        fd.append((fp - fm) / (2 * h))
    fd = np.array(fd)
    assert np.all(np.abs(g_mean - fd) <= 5 * g_se + 1e-5 * (1 + np.abs(fd))), (g_mean, fd, g_se)


def test_control_variate_does_not_change_the_mean():
    # h - c r has the same mean as h: compare the c = optimal estimate with the
    # c = 0 estimate through the identity E[r] = tr(P^{-1} dP) (App. A.4.1).
    n, t = 50, 3000
    model, y, F = _problem(n=n, m=5, seed=15, deriv=True)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, L.Opts(cg_tol=1e-12))
    opts = L.Opts(cg_tol=1e-12, num_probes=t, seed=1)
    _, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, opts,
                                want_grad=True)
    # exact tr(A^{-1} dA) for the log det derivative (dense)
    Bd = model.B.toarray()
    Q = DR.dense_precision(Bd, model.D)
    A = np.diag(W) + Q
    for k in range(2):
        dBd = model.dB[k].toarray()
        dD = model.dD[k]
        Di = model.Dinv
        dQ = dBd.T @ np.diag(Di) @ Bd + Bd.T @ np.diag(Di) @ dBd - Bd.T @ np.diag(Di * Di * dD) @ Bd
        exact = np.sum(dD * Di) + np.trace(np.linalg.solve(A, dQ))
        assert abs(info[f"dlogdet_{k}"] - exact) < 0.05 * (1 + abs(exact))
        # each STE piece is unbiased for its own trace:
        # E[h] = tr(A^{-1} dA), E[r] = tr(P^{-1} dP) with
        # P = B^T (W + D^{-1}) B (eq. P_VADU)
        h, r = info[f"h_{k}"], info[f"r_{k}"]
        trA = np.trace(np.linalg.solve(A, dQ))
        P = Bd.T @ np.diag(W + Di) @ Bd
        dP = dBd.T @ np.diag(W + Di) @ Bd + Bd.T @ np.diag(W + Di) @ dBd \
            - Bd.T @ np.diag(Di * Di * dD) @ Bd
        trP = np.trace(np.linalg.solve(P, dP))
        assert abs(info[f"trP_{k}"] - trP) < 1e-9 * (1 + abs(trP))
        assert abs(h.mean() - trA) <= 5 * h.std(ddof=1) / np.sqrt(t) + 1e-9
        assert abs(r.mean() - trP) <= 5 * r.std(ddof=1) / np.sqrt(t) + 1e-9
        # per probe, against the dense definitions h(z) = (A^{-1}z)^T dA P^{-1}z
        # and r(z) = (P^{-1}z)^T dP P^{-1}z with z = B^T (W+D^{-1})^{1/2} eps
        eps = R.rademacher(1, R.TAG_SLQ, n, 5)
        Z = Bd.T @ (np.sqrt(W + Di)[:, None] * eps)
        hd = np.einsum("ij,ij->j", np.linalg.solve(A, Z), dQ @ np.linalg.solve(P, Z))
        rd = np.einsum("ij,ij->j", np.linalg.solve(P, Z), dP @ np.linalg.solve(P, Z))
        np.testing.assert_allclose(h[:5], hd, rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(r[:5], rd, rtol=1e-8, atol=1e-10)


def _mu_derivative_setup(lik, n=40):
    F = 0.5 if lik == L.LIK_POISSON else 0.0
    model, y, Fv = _problem(n=n, m=5, seed=21, deriv=True, lik=lik, F=F)
    b, W, _ = L.find_mode(model, y, Fv, lik, None, L.Opts(cg_tol=1e-12, newton_tol=1e-15))
    dW = L.lik_dW(lik, y, Fv + b)
    Bd = model.B.toarray()
    A = np.diag(W) + DR.dense_precision(Bd, model.D)
    P = Bd.T @ np.diag(W + model.Dinv) @ Bd
    return model, y, Fv, b, W, dW, Bd, A, P


@pytest.mark.parametrize("lik", [L.LIK_POISSON, L.LIK_BERNOULLI_LOGIT])
def test_mu_derivative_of_the_log_determinant(lik):
    # The implicit part of the theta-gradient needs d log det(Sigma~ W + I)/d mu
    # (App. A.3; VADU mu-formula of App. A.4.1).  Its exact value is
    # dW_i (A^{-1})_ii with A = W + Sigma~^{-1}; the STE h_i = dW_i (A^{-1}z)_i
    # (P^{-1}z)_i is unbiased for it for any probes with Cov(z) = P, and the
    # control variate r_i = dW_i (B P^{-1} z)_i^2 has the mean
    # tr(P^{-1} dP/dmu_i).  Gaussian probes (the paper's def_SLQ) make r
    # random, so the control-variate weight and the trace term are exercised;
    # each piece is compared with a dense computation of its definition.
    n, t = 40, 4000
    model, y, Fv, b, W, dW, Bd, A, P = _mu_derivative_setup(lik, n)
    Di = model.Dinv
    apply_A, apply_Pinv = L.vadu_ops(model, W)
    g = R.gaussian(3, R.TAG_SLQ, n, t)
    Z = Bd.T @ (np.sqrt(W + Di)[:, None] * g)
    res = L.pcg(apply_A, apply_Pinv, Z, 1e-13, 2 * n)
    opts = L.Opts(cg_tol=1e-13, num_probes=t, seed=3)
    _, info = L._grad_theta_vadu(model, y, Fv, lik, None, b, W, res, opts, None)
    # tr(P^{-1} dP/dmu_i) with dP/dmu_i = B^T diag(dW_i e_i) B, densely
    trP_dense = dW * np.diag(Bd @ np.linalg.solve(P, Bd.T))
    np.testing.assert_allclose(info["trP_mu"], trP_dense, rtol=1e-9, atol=1e-14)
    # per probe: h and r against their dense definitions
    AZ, PZ = np.linalg.solve(A, Z[:, :6]), np.linalg.solve(P, Z[:, :6])
    np.testing.assert_allclose(info["h_mu"][:, :6], dW[:, None] * AZ * PZ, rtol=1e-8,
                               atol=1e-12)
    np.testing.assert_allclose(info["r_mu"][:, :6], dW[:, None] * (Bd @ PZ) ** 2, rtol=1e-8,
                               atol=1e-12)
    # the control-variate estimate is mean(h - c r) + c E[r], with E[r] from
    # the dense trace: a dropped, mis-signed or mis-scaled trace term fails
    h, r, c = info["h_mu"], info["r_mu"], info["c_mu"]
    assert np.all(np.abs(c) > 1e-3)
    cv = np.mean(h - c[:, None] * r, axis=1)
    np.testing.assert_allclose(info["dlogdet_dmu"], cv + c * trP_dense, rtol=1e-10,
                               atol=1e-13)
    # and it estimates the exact derivative within 5 standard errors, with a
    # smaller error than the c = 0 estimate
    exact = dW * np.diag(np.linalg.inv(A))
    se = np.std(h - c[:, None] * r, axis=1, ddof=1) / np.sqrt(t)
    assert np.all(np.abs(info["dlogdet_dmu"] - exact) <= 5 * se + 1e-12), \
        np.max(np.abs(info["dlogdet_dmu"] - exact) / (se + 1e-300))
    se0 = np.std(h, axis=1, ddof=1) / np.sqrt(t)
    assert np.mean(se) < np.mean(se0)
    # without the trace term the estimate is biased by c tr(P^{-1} dP/dmu)
    # far beyond its standard error
    assert np.max(np.abs(cv - exact) / se) > 10


@pytest.mark.parametrize("lik", [L.LIK_POISSON, L.LIK_BERNOULLI_LOGIT])
def test_mu_derivative_with_rademacher_probes(lik):
    # With Rademacher probes (the reading used for SLQ) B P^{-1} z =
    # (W + D^{-1})^{-1/2} eps, so r_i = dW_i eps_i^2 / (W_i + 1/D_i) is the
    # same for every probe: the control-variate weight is 0 and the estimate
    # is the plain mean of h, still within 5 standard errors of the exact
    # dW_i (A^{-1})_ii.
    n, t = 40, 4000
    model, y, Fv, b, W, dW, Bd, A, P = _mu_derivative_setup(lik, n)
    opts = L.Opts(cg_tol=1e-13, num_probes=t, seed=3)
    _, info = L.neg_log_marglik(model, y, Fv, lik, None, b, opts, want_grad=True)
    r = info["r_mu"]
    np.testing.assert_allclose(r, np.repeat(info["trP_mu"][:, None], t, axis=1), rtol=1e-10,
                               atol=1e-15)
    assert np.all(info["c_mu"] == 0.0)
    h = info["h_mu"]
    np.testing.assert_allclose(info["dlogdet_dmu"], h.mean(axis=1), rtol=1e-12, atol=1e-15)
    exact = dW * np.diag(np.linalg.inv(A))
    se = np.std(h, axis=1, ddof=1) / np.sqrt(t)
    assert np.all(np.abs(info["dlogdet_dmu"] - exact) <= 5 * se + 1e-12)


# ----------------------------------------------------------------- prediction
def test_prediction_textbook_limit():
    # m = n-1 and m_p = n: the Vecchia approximation is exact, so the
    # predictive mean is k_p^T Sigma^{-1} b* and the variance is
    # k_pp - k_p^T (Sigma + W^{-1})^{-1} k_p.  The simulated variance lies
    # within 5 sd of it with sd = sqrt(2/s) (var - D_p) (Prop. 3.3).
    n, npred, s = 60, 12, 4000
    model, y, F = _problem(n=n, m=n - 1, seed=16)
    Xp = np.random.default_rng(17).uniform(size=(npred, 2))
    opts = L.Opts(cg_tol=1e-12, newton_tol=1e-15, num_pred_samples=s, pred_cg_tol=1e-12,
                  seed=4)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, opts)
    model.m = n      # prediction conditions on all n training points
    mean, var, info = L.predict(model, Xp, None, b, W, opts, chunk=1000)
    S = V.dense_covariance(model.coords, model.kind, *model.theta)
    Kp = V.dense_covariance(Xp, model.kind, *model.theta, coords2=model.coords)
    np.testing.assert_allclose(mean, Kp @ np.linalg.solve(S, b), rtol=1e-7, atol=1e-8)
    exact = model.theta[0] - np.einsum("pi,pi->p", Kp, np.linalg.solve(S + np.diag(1 / W), Kp.T).T)
    sd = np.sqrt(2.0 / s) * (exact - info["Dp"])
    assert np.all(np.abs(var - exact) <= 5 * sd + 1e-10)


def test_prediction_variance_formula_small_m():
    # General m: the simulated variance is unbiased for D_p + diag(A_p A^{-1}
    # A_p^T) (eq. latentpostpredictive with B_p = I).
    n, npred, s = 120, 15, 3000
    model, y, F = _problem(n=n, m=6, seed=18, kind=V.COV_MATERN32, theta=(1.0, 0.2))
    Xp = np.random.default_rng(19).uniform(size=(npred, 2))
    opts = L.Opts(cg_tol=1e-12, newton_tol=1e-15, num_pred_samples=s, pred_cg_tol=1e-12,
                  seed=2)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, opts)
    mean, var, info = L.predict(model, Xp, None, b, W, opts, chunk=1500)
    Ap = np.zeros((npred, n))
    for p in range(npred):
        Ap[p, info["nbr_p"][p]] = info["Ap"][p]
    A = np.diag(W) + DR.dense_precision(model.B, model.D)
    exact = info["Dp"] + np.einsum("pi,pi->p", Ap, np.linalg.solve(A, Ap.T).T)
    np.testing.assert_allclose(mean, Ap @ b, rtol=1e-12, atol=1e-13)
    sd = np.sqrt(2.0 / s) * (exact - info["Dp"])
    assert np.all(np.abs(var - exact) <= 5 * sd + 1e-10)


def test_probe_and_sample_slices_equal_the_full_sets():
    """Counter-based probes: a slice of probe columns (col0) gives the same
    per-column quadratures, and sample-column slices add up to the full
    simulated variance (Alg. simAlgo sums over independent columns)."""
    import synth
    w = synth.make(None, seed=9, n=300, m=6, kind=synth.COV_MATERN32, sigma2=1.0, rho=0.2,
                   lik=synth.LIK_BERNOULLI_LOGIT, F=0.0, n_pred=40)
    model = L.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]))
    o = L.Opts(cg_tol=1e-10, pred_cg_tol=1e-10, num_probes=6, num_pred_samples=6, seed=3)
    b, W, _ = L.find_mode(model, w["y"], w["F"], w["lik"], None, o)
    _, full = L.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o)
    o2 = L.Opts(cg_tol=1e-10, num_probes=2, seed=3)
    _, part = L.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o2, col0=3)
    np.testing.assert_allclose(part["quad"], full["quad"][3:5], rtol=1e-12)
    _, var, info = L.predict(model, w["coords_pred"], w["Fp"], b, W, o)
    o3 = L.Opts(pred_cg_tol=1e-10, num_pred_samples=3, seed=3)
    _, _, i0 = L.predict(model, w["coords_pred"], w["Fp"], b, W, o3, col0=0)
    _, _, i1 = L.predict(model, w["coords_pred"], w["Fp"], b, W, o3, col0=3)
    np.testing.assert_allclose(info["Dp"] + (i0["acc"] + i1["acc"]) / 6, var, rtol=1e-12)


def test_offset_gradient_gaussian_closed_form():
    """Gaussian likelihood: W is constant, so the log-determinant does not
    depend on mu and d L / d F = -(Sigma~ + tau^2 I)^{-1} (y - F), the
    gradient of the exact negative log-density of N(F, Sigma~ + tau^2 I)."""
    n, m, tau2 = 60, 8, 0.3
    model, y, F = _problem(n=n, m=m, seed=21, lik=L.LIK_GAUSSIAN, deriv=True, F=0.4)
    F = F + np.linspace(-0.5, 0.5, n)
    o = L.Opts(cg_tol=1e-13, newton_tol=1e-15, num_probes=4, seed=2)
    b, W, _ = L.find_mode(model, y, F, L.LIK_GAUSSIAN, tau2, o)
    _, info = L.neg_log_marglik(model, y, F, L.LIK_GAUSSIAN, tau2, b, o, want_grad=True)
    Q = DR.dense_precision(model.B, model.D)
    S = np.linalg.inv(Q)
    exact = -np.linalg.solve(S + tau2 * np.eye(n), y - F)
    np.testing.assert_allclose(info["grad_F"], exact, rtol=1e-8, atol=1e-10)


def test_offset_gradient_matches_finite_differences():
    """Bernoulli-logit: d L / d F (STE for d log det / d mu, VADU control
    variates, implicit mode response) against central differences of the
    exact dense Vecchia-Laplace NLL along two directions, within 5 standard
    errors over independent probe sets.  Dropping the mode-response term or
    the log-determinant term moves it by more than 8 standard errors."""
    n, m = 45, 5
    model, y, F = _problem(n=n, m=m, seed=16, theta=(1.1, 0.3), deriv=True)
    o0 = L.Opts(cg_tol=1e-12, newton_tol=1e-15)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, o0)
    gs = []
    for seed in range(8):
        o = L.Opts(cg_tol=1e-12, newton_tol=1e-15, num_probes=400, seed=seed)
        _, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, b, o,
                                    want_grad=True)
        gs.append(info["grad_F"])
    gs = np.array(gs)
    g = np.random.default_rng(3)
    # directions that average many coordinates (a single coordinate's STE is
    # heavy-tailed over 8 probe sets)
    for d in (g.standard_normal(n), np.ones(n)):
        proj = gs @ d
        mean, se = proj.mean(), proj.std(ddof=1) / np.sqrt(len(proj))
        h = 1e-5
        fp = _dense_vl_nll(model.coords, model.nbr, V.COV_EXPONENTIAL, model.theta, y, F + h * d,
                           L.LIK_BERNOULLI_LOGIT)
        fm = _dense_vl_nll(model.coords, model.nbr, V.COV_EXPONENTIAL, model.theta, y, F - h * d,
                           L.LIK_BERNOULLI_LOGIT)
        fd = (fp - fm) / (2 * h)
        assert abs(mean - fd) <= 5 * se + 1e-6 * (1 + abs(fd)), (mean, fd, se)
        # the terms beyond -g are not negligible here: the pin would catch
        # a dropped log-determinant or mode-response term
        assert abs(-(L.lik_grad(L.LIK_BERNOULLI_LOGIT, y, F + b) @ d) - fd) > 8 * se


def test_estimate_is_stationary_and_near_the_exact_optimum():
    """The L-BFGS estimate with a sample average approximation (Sec. 4.1) is
    a zero of the STE gradient of the deterministic objective, and lies near
    the optimum of the exact dense Vecchia-Laplace NLL (the STE and SLQ
    estimators differ from the exact derivative and value by O(t^-1/2); with
    t = 200 the estimate is within 0.1 of it in log theta)."""
    from scipy.optimize import minimize

    g = np.random.default_rng(30)
    n, m = 200, 6
    X = g.uniform(size=(n, 2))
    S = V.dense_covariance(X, V.COV_EXPONENTIAL, 1.0, 0.15)
    b = np.linalg.cholesky(S + 1e-10 * np.eye(n)) @ g.standard_normal(n)
    y = (g.uniform(size=n) < 1 / (1 + np.exp(-b))).astype(float)
    F = np.zeros(n)
    nbr = V.neighbours(X, m)
    o = L.Opts(cg_tol=1e-10, newton_tol=1e-12, num_probes=200, seed=4)
    theta, nll, res = L.estimate(X, m, V.COV_EXPONENTIAL, y, F, L.LIK_BERNOULLI_LOGIT, None,
                                 (0.5, 0.05), o, nbr=nbr, gtol=1e-7)
    model = L.Model(X, m, V.COV_EXPONENTIAL, theta, nbr=nbr, deriv=True)
    bb, _, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, o)
    v0, info = L.neg_log_marglik(model, y, F, L.LIK_BERNOULLI_LOGIT, None, bb, o, want_grad=True)
    assert abs(v0 - nll) < 1e-9 * abs(nll)
    # CG counts change with theta, so the objective is smooth only to about
    # 1e-11 relative: the optimiser stops once steps gain no more than that
    assert np.max(np.abs(info["grad"] * theta)) < 1e-3
    exact = minimize(lambda x: _dense_vl_nll(X, nbr, V.COV_EXPONENTIAL, np.exp(x), y, F,
                                             L.LIK_BERNOULLI_LOGIT),
                     np.log([0.5, 0.05]), method="Nelder-Mead",
                     options={"xatol": 1e-8, "fatol": 1e-12, "maxiter": 2000})
    assert np.max(np.abs(np.log(theta) - exact.x)) < 0.1, (theta, np.exp(exact.x))


def test_joint_estimate_gamma_is_near_the_exact_optimum():
    """Joint estimate of (sigma2, rho, shape, beta) for a Gamma response with
    F = X beta (intercept and one covariate): the returned point lies near the
    minimiser of the exact dense Vecchia-Laplace NLL over the same parameters
    (within 0.05 in each search coordinate with t = 200 probes), and its
    gradient is a small fraction of the starting one.  (The STE gradient is
    not the derivative of the SLQ value, so the line search ends where the
    two disagree, at a gradient of O(t^-1/2), not at zero.)"""
    from scipy.optimize import minimize

    g = np.random.default_rng(44)
    n, m, a_true = 100, 6, 3.0
    Xs = g.uniform(size=(n, 2))
    S = V.dense_covariance(Xs, V.COV_EXPONENTIAL, 0.5, 0.2)
    b = np.linalg.cholesky(S + 1e-10 * np.eye(n)) @ g.standard_normal(n)
    Xd = np.column_stack([np.ones(n), g.standard_normal(n)])
    beta_true = np.array([0.3, -0.5])
    y = g.gamma(a_true, np.exp(Xd @ beta_true + b) / a_true)
    nbr = V.neighbours(Xs, m)
    o = L.Opts(cg_tol=1e-10, newton_tol=1e-12, num_probes=200, seed=8)
    theta, a, beta, nll, res = L.estimate_glm(Xs, m, V.COV_EXPONENTIAL, y, Xd, L.LIK_GAMMA,
                                              (1.0, 0.1), 1.0, np.zeros(2), o, nbr=nbr,
                                              gtol=1e-7)
    xhat = L.glm_params_to_x(theta, a, beta, L.LIK_GAMMA)
    model0 = L.Model(Xs, m, V.COV_EXPONENTIAL, (1.0, 0.1), nbr=nbr, deriv=True)
    b0, _, _ = L.find_mode(model0, y, np.zeros(n), L.LIK_GAMMA, 1.0, o)
    _, i0 = L.neg_log_marglik(model0, y, np.zeros(n), L.LIK_GAMMA, 1.0, b0, o, want_grad=True)
    g0 = np.concatenate([i0["grad"] * np.array([1.0, 0.1]), [i0["grad_xi"]], Xd.T @ i0["grad_F"]])
    assert np.max(np.abs(res.jac)) < 1e-3 * np.max(np.abs(g0)), (res.jac, g0)

    def dense(x):
        th, aa, bb = np.exp(x[:2]), float(np.exp(x[2])), x[3:]
        A, D = V.factor(Xs, nbr, V.COV_EXPONENTIAL, th)
        Q = DR.dense_precision(V.sparse_B(A, nbr), D)
        lp, lg, lw = _liks(L.LIK_GAMMA, aa)
        return DR.dense_nll(Q, y, Xd @ bb, lp, lg, lw)[0]

    # the exact optimum, started at the estimate (a local search)
    exact = minimize(dense, xhat, method="Nelder-Mead",
                     options={"xatol": 1e-6, "fatol": 1e-10, "maxiter": 5000, "maxfev": 5000})
    assert np.max(np.abs(xhat - exact.x)) < 0.05, (xhat, exact.x)


def test_gamma_likelihood_is_the_gamma_density():
    """Gamma with log link (Sec. 5): mean e^mu, shape a, i.e. scale e^mu / a;
    the log-density equals scipy's, and W = -d2 log p / d mu2 > 0 (log-concave
    in mu)."""
    from scipy.stats import gamma as G
    y = np.array([0.05, 0.4, 1.0, 3.5, 12.0])
    mu = np.array([-1.0, 0.3, 0.0, 1.2, 2.0])
    for a in (0.7, 2.5, 30.0):
        np.testing.assert_allclose(L.lik_logp(L.LIK_GAMMA, y, mu, a),
                                   G.logpdf(y, a, scale=np.exp(mu) / a), rtol=1e-12)
        assert np.all(L.lik_W(L.LIK_GAMMA, y, mu, a) > 0)



# ------------------------------------------------------------ xi-gradient
def test_xi_gradient_gaussian_closed_form():
    """Gaussian likelihood, xi = tau^2: L^VLA is the exact negative log-density
    of N(F, K), K = Sigma~ + tau^2 I, whose tau^2-derivative is
    tr(K^{-1})/2 - |K^{-1}(y - F)|^2/2.  With m = 0 (B = I, P_VADU = A) the
    STE is exact, so the oracle must match to rounding; with m = 5 its mean
    over probe sets must lie within 5 standard errors."""
    tau2 = 0.3
    for m in (0, 5):
        model, y, F = _problem(n=50, m=m, seed=31, lik=L.LIK_GAUSSIAN, deriv=True, F=0.2)
        o0 = L.Opts(cg_tol=1e-13, newton_tol=1e-15)
        b, W, _ = L.find_mode(model, y, F, L.LIK_GAUSSIAN, tau2, o0)
        K = np.linalg.inv(DR.dense_precision(model.B, model.D)) + tau2 * np.eye(model.n)
        Ki = np.linalg.inv(K)
        ref = 0.5 * np.trace(Ki) - 0.5 * np.sum((Ki @ (y - F)) ** 2)
        gs = []
        for seed in range(1 if m == 0 else 8):
            o = L.Opts(cg_tol=1e-13, newton_tol=1e-15, num_probes=200, seed=seed)
            _, info = L.neg_log_marglik(model, y, F, L.LIK_GAUSSIAN, tau2, b, o, want_grad=True)
            gs.append(info["grad_xi"])
        if m == 0:
            assert abs(gs[0] - ref) <= 1e-10 * abs(ref)
        else:
            se = np.std(gs, ddof=1) / np.sqrt(len(gs))
            assert abs(np.mean(gs) - ref) <= 5 * se + 1e-8 * abs(ref), (np.mean(gs), ref, se)


def _dense_nll_aux(model, y, F, lik, aux):
    Q = DR.dense_precision(model.B, model.D)
    lp, lg, lw = _liks(lik, aux)
    return DR.dense_nll(Q, y, F, lp, lg, lw)[0]


def test_xi_gradient_gamma_matches_finite_differences():
    """Gamma shape a: the STE xi-gradient (VADU control variate, implicit mode
    response) against central differences of the exact dense Vecchia-Laplace
    NLL in a.  m = 0: the STE is exact and must match to the difference
    error.  m = 5: within 5 standard errors over independent probe sets, and
    dropping the log-determinant or the mode-response term moves the value by
    more than 8 standard errors."""
    a = 2.5
    for m in (0, 5):
        model, y, F = _problem(n=45, m=m, seed=33, lik=L.LIK_GAMMA, deriv=True, theta=(0.8, 0.3))
        o0 = L.Opts(cg_tol=1e-13, newton_tol=1e-15)
        b, W, _ = L.find_mode(model, y, F, L.LIK_GAMMA, a, o0)
        h = 1e-5
        fd = (_dense_nll_aux(model, y, F, L.LIK_GAMMA, a + h)
              - _dense_nll_aux(model, y, F, L.LIK_GAMMA, a - h)) / (2 * h)
        infos = []
        for seed in range(1 if m == 0 else 8):
            o = L.Opts(cg_tol=1e-13, newton_tol=1e-15, num_probes=400, seed=seed)
            infos.append(L.neg_log_marglik(model, y, F, L.LIK_GAMMA, a, b, o, want_grad=True)[1])
        gs = np.array([i["grad_xi"] for i in infos])
        if m == 0:
            assert abs(gs[0] - fd) <= 1e-7 * (1 + abs(fd)), (gs[0], fd)
            continue
        se = gs.std(ddof=1) / np.sqrt(len(gs))
        assert abs(gs.mean() - fd) <= 5 * se + 1e-7 * (1 + abs(fd)), (gs.mean(), fd, se)
        # Rademacher probes make B P^{-1} z = (W + D^{-1})^{-1/2} eps, so every
        # control-variate value equals its known mean tr(P^{-1} dP/dxi)
        for i in infos:
            np.testing.assert_allclose(i["r_xi"], i["trP_xi"], rtol=1e-10)
        no_logdet = np.mean([i["grad_xi"] - 0.5 * i["dlogdet_xi"] for i in infos])
        no_implicit = np.mean([i["grad_xi"] - i["implicit_xi"] for i in infos])
        assert abs(no_logdet - fd) > 8 * se and abs(no_implicit - fd) > 8 * se


# ------------------------------------------------------ Lanczos prediction
def _lanczos_setup(n=70, m=6, npred=15, seed=41):
    model, y, F = _problem(n=n, m=m, seed=seed, kind=V.COV_MATERN32, theta=(1.0, 0.2))
    Xp = np.random.default_rng(seed + 1).uniform(size=(npred, 2))
    o = L.Opts(cg_tol=1e-12, newton_tol=1e-15)
    b, W, _ = L.find_mode(model, y, F, L.LIK_BERNOULLI_LOGIT, None, o)
    _, _, info = L.predict(model, Xp, None, b, W, o, want_var=False)
    Ap = np.zeros((npred, n))
    for p in range(npred):
        Ap[p, info["nbr_p"][p]] = info["Ap"][p]
    A = np.diag(W) + DR.dense_precision(model.B, model.D)
    exact = info["Dp"] + np.einsum("pi,pi->p", Ap, np.linalg.solve(A, Ap.T).T)
    return model, Xp, b, W, Ap, exact


@pytest.mark.parametrize("method", [L.PRED_LANCZOS_L1, L.PRED_LANCZOS_L2])
def test_lanczos_full_rank_is_exact(method):
    """k = n: the Lanczos vectors span the space and Q T^{-1} Q^T = M^{-1}, so
    both preconditioned forms give the dense predictive variance D_p +
    diag(A_p A^{-1} A_p^T) (eq. latentpostpredictive) and the mean A_p b*."""
    model, Xp, b, W, Ap, exact = _lanczos_setup()
    mean, var, info = L.predict_lanczos(model, Xp, None, b, W, model.n, method)
    assert info["rank"] == model.n
    np.testing.assert_allclose(mean, Ap @ b, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(var, exact, rtol=1e-8)


@pytest.mark.parametrize("method", [L.PRED_LANCZOS_L1, L.PRED_LANCZOS_L2])
def test_lanczos_relation_and_orthonormality(method):
    """M Q_k = Q_k T_k + beta_k q_{k+1} e_k^T (the residual lives in the last
    column only), Q_k^T Q_k = I, T_k symmetric positive definite, q_1 along
    the mapped mean column; M built densely from the preconditioner's
    definition (Sec. 3.3.2)."""
    model, Xp, b, W, Ap, exact = _lanczos_setup()
    k = 20
    _, _, info = L.predict_lanczos(model, Xp, None, b, W, k, method)
    Q, T = info["Q"], info["T"]
    Bd = model.B.toarray()
    Binv = np.linalg.inv(Bd)
    St = Binv @ np.diag(model.D) @ Binv.T
    if method == L.PRED_LANCZOS_L1:
        Pih = np.diag((W + model.Dinv) ** -0.5) @ Binv.T
        M = Pih @ (np.diag(W) + np.linalg.inv(St)) @ Pih.T
    else:
        s = (model.theta[0] + 1.0 / W) ** -0.5
        M = np.diag(s) @ (St + np.diag(1.0 / W)) @ np.diag(s)
    np.testing.assert_allclose(Q.T @ Q, np.eye(k), atol=1e-12)
    # the start: the mean column of B_po^T = -A_p^T mapped into M's coordinates
    xbar = -Ap.sum(axis=0) / Ap.shape[0]
    if method == L.PRED_LANCZOS_L1:
        q1 = Pih @ xbar
    else:
        q1 = s * (St @ xbar)
    np.testing.assert_allclose(Q[:, 0], q1 / np.linalg.norm(q1), atol=1e-12)
    R = M @ Q - Q @ T
    assert np.max(np.abs(R[:, :-1])) < 1e-10 * np.max(np.abs(M))
    assert np.allclose(T, T.T) and np.linalg.eigvalsh(T).min() > 0


def test_lanczos_l1_variance_increases_with_rank_to_the_exact_value():
    """P_L1 form: g^T T_k^{-1} g is the quadratic form of the inverse projected
    onto a growing (nested) Krylov space, so the variance never decreases in
    k and never exceeds the exact value (the systematic underestimation the
    paper reports)."""
    model, Xp, b, W, Ap, exact = _lanczos_setup()
    prev = None
    for k in (2, 5, 10, 20, 40):
        _, var, _ = L.predict_lanczos(model, Xp, None, b, W, k, L.PRED_LANCZOS_L1)
        assert np.all(var <= exact * (1 + 1e-10))
        if prev is not None:
            assert np.all(var >= prev * (1 - 1e-10))
        prev = var


# ------------------------------------------------------------ LRAC gradient
def test_pivoted_cholesky_derivative_matches_finite_differences():
    """d L_k / d theta with the pivots held fixed against central differences
    of the pivoted Cholesky factor at the same pivots."""
    X = np.random.default_rng(61).uniform(size=(60, 2))
    for kind in (V.COV_EXPONENTIAL, V.COV_MATERN32):
        th = np.array([1.3, 0.25])
        L, dL, piv = L_.pivoted_cholesky_deriv(X, kind, th, 12)
        np.testing.assert_array_equal(L, L_.pivoted_cholesky(X, kind, th, 12))
        for q, h in ((0, 1e-6), (1, 1e-7)):
            e = np.zeros(2)
            e[q] = h
            fd = (L_.pivoted_cholesky(X, kind, th + e, 12, pivots=piv)
                  - L_.pivoted_cholesky(X, kind, th - e, 12, pivots=piv)) / (2 * h)
            np.testing.assert_allclose(dL[q], fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def _lrac_fd_setup(lik, aux, n=45, m=5, seed=71):
    model, y, F = _problem(n=n, m=m, seed=seed, lik=lik, deriv=True, theta=(0.9, 0.25))
    o0 = L.Opts(cg_tol=1e-12, newton_tol=1e-15)
    b, W, _ = L.find_mode(model, y, F, lik, aux, o0)
    return model, y, F, b


def test_lrac_gradient_exact_at_full_rank():
    """k = n and m = n - 1: L L^T = Sigma = Sigma~ and P_LRAC equals the
    operator, so u = P^{-1} z, h = r for every probe (c = 1) and the LRAC STE
    gives the exact derivatives: theta, the offset F and the Gamma shape
    against central differences of the dense exact NLL."""
    n = 30
    for lik, aux in ((L.LIK_BERNOULLI_LOGIT, None), (L.LIK_GAMMA, 2.0)):
        model, y, F = _problem(n=n, m=n - 1, seed=73, lik=lik, deriv=True, theta=(0.9, 0.25))
        o = L.Opts(cg_tol=1e-13, newton_tol=1e-15, num_probes=6, seed=1,
                   precond=L.PRECOND_LRAC, lrac_rank=n)
        b, W, _ = L.find_mode(model, y, F, lik, aux, o)
        _, info = L.neg_log_marglik(model, y, F, lik, aux, b, o, want_grad=True)

        def dense(th, FF, aa):
            A, D = V.factor(model.coords, model.nbr, model.kind, th)
            Q = DR.dense_precision(V.sparse_B(A, model.nbr), D)
            lp, lg, lw = _liks(lik, aa)
            return DR.dense_nll(Q, y, FF, lp, lg, lw)[0]

        th = np.array(model.theta)
        for q, h in ((0, 1e-5), (1, 1e-6)):
            e = np.zeros(2)
            e[q] = h
            fd = (dense(th + e, F, aux) - dense(th - e, F, aux)) / (2 * h)
            assert abs(info["grad"][q] - fd) <= 1e-6 * (1 + abs(fd)), (q, info["grad"][q], fd)
        d = np.random.default_rng(5).standard_normal(n)
        fd = (dense(th, F + 1e-5 * d, aux) - dense(th, F - 1e-5 * d, aux)) / 2e-5
        assert abs(info["grad_F"] @ d - fd) <= 1e-6 * (1 + abs(fd))
        if aux is not None:
            fd = (dense(th, F, aux + 1e-5) - dense(th, F, aux - 1e-5)) / 2e-5
            assert abs(info["grad_xi"] - fd) <= 1e-6 * (1 + abs(fd))


@pytest.mark.parametrize("lik,aux", [(L.LIK_BERNOULLI_LOGIT, None), (L.LIK_GAMMA, 2.0)])
def test_lrac_gradient_matches_finite_differences(lik, aux):
    """k < n, m < n - 1: the LRAC STE gradients (theta, offset along an
    averaging direction, Gamma shape) within 5 standard errors over
    independent probe sets of central differences of the dense exact NLL."""
    model, y, F, b = _lrac_fd_setup(lik, aux)
    gs, gF, gx = [], [], []
    d = np.random.default_rng(9).standard_normal(model.n)
    for seed in range(8):
        o = L.Opts(cg_tol=1e-12, newton_tol=1e-15, num_probes=400, seed=seed,
                   precond=L.PRECOND_LRAC, lrac_rank=8)
        _, info = L.neg_log_marglik(model, y, F, lik, aux, b, o, want_grad=True)
        gs.append(info["grad"])
        gF.append(info["grad_F"] @ d)
        if aux is not None:
            gx.append(info["grad_xi"])

    def dense(th, FF, aa):
        A, D = V.factor(model.coords, model.nbr, model.kind, th)
        Q = DR.dense_precision(V.sparse_B(A, model.nbr), D)
        lp, lg, lw = _liks(lik, aa)
        return DR.dense_nll(Q, y, FF, lp, lg, lw)[0]

    th = np.array(model.theta)
    checks = []
    for q, h in ((0, 1e-5), (1, 1e-6)):
        e = np.zeros(2)
        e[q] = h
        checks.append((np.array(gs)[:, q], (dense(th + e, F, aux) - dense(th - e, F, aux)) / (2 * h)))
    checks.append((np.array(gF), (dense(th, F + 1e-5 * d, aux) - dense(th, F - 1e-5 * d, aux)) / 2e-5))
    if aux is not None:
        checks.append((np.array(gx), (dense(th, F, aux + 1e-5) - dense(th, F, aux - 1e-5)) / 2e-5))
    for est, fd in checks:
        se = est.std(ddof=1) / np.sqrt(len(est))
        assert abs(est.mean() - fd) <= 5 * se + 1e-6 * (1 + abs(fd)), (est.mean(), fd, se)

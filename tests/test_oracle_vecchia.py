"""Pins for the Vecchia part of the oracle (Sec. 2.1, appendix derivatives)."""
import math

import numpy as np
import pytest
from scipy.special import gamma as gamma_fn, kv

from oracle import vecchia as V


def _brute_nn(coords, i, cand, m):
    # pure-Python exhaustive search, sorted by (squared distance, index)
    q = coords[i]
    keyed = []
    for j in cand:
        dx = coords[j][0] - q[0]
        dy = coords[j][1] - q[1]
        keyed.append((dx * dx + dy * dy, j))
    keyed.sort()
    return [j for _, j in keyed[:m]]


@pytest.mark.parametrize("n,m,lim", [(200, 7, 16), (400, 12, 40)])
def test_neighbours_match_exhaustive_search(n, m, lim):
    rng = np.random.default_rng(n)
    X = rng.uniform(size=(n, 2))
    nbr = V.neighbours(X, m, brute_limit=lim)   # exercises the k-d tree path
    for i in range(n):
        ref = _brute_nn(X, i, range(i), m)
        got = [j for j in nbr[i] if j >= 0]
        assert got == ref, i


def test_neighbours_of_selected_rows_match_exhaustive_search():
    # rows scattered over the exhaustive range and several tree blocks, in
    # no particular order, with a repeat
    rng = np.random.default_rng(17)
    X = rng.uniform(size=(600, 2))
    rows = np.array([599, 0, 3, 15, 16, 31, 32, 33, 100, 257, 3, 420, 64])
    got = V.neighbours_rows(X, 8, rows, brute_limit=16)
    for r, i in enumerate(rows):
        assert [j for j in got[r] if j >= 0] == _brute_nn(X, i, range(i), 8), i


def test_neighbours_ties_break_by_index():
    # integer lattice: many exactly equal distances
    g = np.array([(x, y) for x in range(6) for y in range(6)], dtype=float)
    perm = np.random.default_rng(3).permutation(len(g))
    X = g[perm]
    nbr = V.neighbours(X, 5, brute_limit=4)
    for i in range(len(X)):
        assert [j for j in nbr[i] if j >= 0] == _brute_nn(X, i, range(i), 5)


def test_pred_neighbours_match_exhaustive_search():
    rng = np.random.default_rng(5)
    Xt = rng.uniform(size=(5000, 2))    # above the exhaustive-search limit
    Xp = rng.uniform(size=(40, 2))
    nbr = V.pred_neighbours(Xt, Xp, 9)
    allpts = np.concatenate([Xt, Xp])
    for p in range(len(Xp)):
        ref = _brute_nn(allpts, 5000 + p, range(5000), 9)
        assert list(nbr[p]) == ref


def _matern_general(d, nu, sigma2, rho):
    # textbook Matern: sigma2 2^{1-nu}/Gamma(nu) (sqrt(2 nu) d/rho)^nu K_nu(.)
    x = math.sqrt(2.0 * nu) * d / rho
    return sigma2 * 2.0 ** (1.0 - nu) / gamma_fn(nu) * x ** nu * kv(nu, x)


@pytest.mark.parametrize("kind,nu", [(V.COV_EXPONENTIAL, 0.5), (V.COV_MATERN32, 1.5)])
def test_covariance_is_matern(kind, nu):
    d = np.linspace(1e-3, 0.7, 50)
    got = V.covariance(d * d, kind, 1.7, 0.13)
    ref = _matern_general(d, nu, 1.7, 0.13)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    assert V.covariance(np.array([0.0]), kind, 1.7, 0.13)[0] == 1.7


@pytest.mark.parametrize("kind", [V.COV_EXPONENTIAL, V.COV_MATERN32])
def test_covariance_grad_finite_differences(kind):
    d2 = np.linspace(1e-4, 0.3, 40)
    s2, rho, h = 1.3, 0.09, 1e-6
    g = V.covariance_grad(d2, kind, s2, rho)
    fd_s = (V.covariance(d2, kind, s2 + h, rho) - V.covariance(d2, kind, s2 - h, rho)) / (2 * h)
    fd_r = (V.covariance(d2, kind, s2, rho + h) - V.covariance(d2, kind, s2, rho - h)) / (2 * h)
    np.testing.assert_allclose(g[0], fd_s, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(g[1], fd_r, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("kind", [V.COV_EXPONENTIAL, V.COV_MATERN32])
def test_exact_gp_limit(kind):
    # m = n-1: conditioning on all earlier points, so B^T D^{-1} B = Sigma^{-1}
    # and B^{-1} D B^{-T} = Sigma (Sec. 2.1; the LDL^T factorisation).
    n = 120
    X = np.random.default_rng(1).uniform(size=(n, 2))
    theta = (1.0, 0.1)
    nbr = V.neighbours(X, n - 1)
    A, D = V.factor(X, nbr, kind, theta)
    B = V.sparse_B(A, nbr).toarray()
    S = V.dense_covariance(X, kind, *theta)
    Q = B.T @ np.diag(1.0 / D) @ B
    np.testing.assert_allclose(Q @ S, np.eye(n), atol=1e-6)
    Binv = np.linalg.inv(B)
    np.testing.assert_allclose(Binv @ np.diag(D) @ Binv.T, S, atol=1e-10)
    # B is unit lower triangular
    assert np.allclose(np.diag(B), 1.0) and np.allclose(np.triu(B, 1), 0.0)


def test_vecchia_conditionals_are_kriging():
    # each row: A_i = kriging weights, D_i = kriging variance on N(i)
    n, m = 300, 6
    X = np.random.default_rng(2).uniform(size=(n, 2))
    theta = (0.8, 0.2)
    nbr = V.neighbours(X, m)
    A, D = V.factor(X, nbr, V.COV_MATERN32, theta)
    S = V.dense_covariance(X, V.COV_MATERN32, *theta)
    for i in [0, 1, 2, 5, 77, 299]:
        N = [j for j in nbr[i] if j >= 0]
        if not N:
            assert D[i] == theta[0]
            continue
        SN = S[np.ix_(N, N)]
        c = S[i, N]
        w = np.linalg.lstsq(SN, c, rcond=None)[0]
        np.testing.assert_allclose(A[i, :len(N)], w, rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(D[i], S[i, i] - c @ w, rtol=1e-8)


@pytest.mark.parametrize("kind", [V.COV_EXPONENTIAL, V.COV_MATERN32])
def test_factor_derivatives_finite_differences(kind):
    n, m = 150, 8
    X = np.random.default_rng(4).uniform(size=(n, 2))
    nbr = V.neighbours(X, m)
    s2, rho = 1.1, 0.15
    A, D, dA, dD = V.factor(X, nbr, kind, (s2, rho), deriv=True)
    for k, (e0, e1) in enumerate([(1e-3, 0.0), (0.0, 1e-5)]):
        Ap, Dp = V.factor(X, nbr, kind, (s2 + e0, rho + e1))
        Am, Dm = V.factor(X, nbr, kind, (s2 - e0, rho - e1))
        h = e0 + e1
        scale = 1.0 + np.max(np.abs(dA[k]))
        np.testing.assert_allclose(dA[k], (Ap - Am) / (2 * h), rtol=1e-5, atol=1e-7 * scale)
        np.testing.assert_allclose(dD[k], (Dp - Dm) / (2 * h), rtol=1e-4, atol=1e-7)
    # sigma2 scales Sigma: A independent of sigma2, D proportional to it
    assert np.max(np.abs(dA[0])) < 1e-10
    np.testing.assert_allclose(dD[0], D / s2, rtol=1e-12)


def test_prediction_rows_are_kriging_on_training_points():
    n, m = 400, 10
    rng = np.random.default_rng(6)
    X = rng.uniform(size=(n, 2))
    Xp = rng.uniform(size=(25, 2))
    theta = (1.0, 0.12)
    nbr_p = V.pred_neighbours(X, Xp, m)
    Ap, Dp = V.factor(X, nbr_p, V.COV_EXPONENTIAL, theta, coords_self=Xp)
    for p in range(len(Xp)):
        N = list(nbr_p[p])
        SN = V.dense_covariance(X[N], V.COV_EXPONENTIAL, *theta)
        c = V.dense_covariance(Xp[p:p + 1], V.COV_EXPONENTIAL, *theta, coords2=X[N])[0]
        w = np.linalg.lstsq(SN, c, rcond=None)[0]
        np.testing.assert_allclose(Ap[p], w, rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(Dp[p], theta[0] - c @ w, rtol=1e-8)

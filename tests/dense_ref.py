"""Dense exact references used only to pin the oracle.

These are textbook dense computations (numpy.linalg) of quantities that the
iterative method reaches in special cases: the dense Vecchia precision, the
exact Laplace mode by Newton with direct solves, the exact log-determinant,
and the textbook Gaussian-process predictive distribution.  They share no
code with the oracle except the likelihood derivative functions, which are
pinned separately against finite differences."""
import numpy as np


def dense_precision(B, D):
    Bd = B.toarray() if hasattr(B, "toarray") else B
    return Bd.T @ np.diag(1.0 / D) @ Bd


def dense_mode(Q, y, F, logp_grad, logp_W, tol=1e-14, max_iter=200):
    """argmax_b log p(y|F+b) - b^T Q b / 2 by Newton with direct solves."""
    b = np.zeros(Q.shape[0])
    for _ in range(max_iter):
        g = logp_grad(y, F + b)
        W = logp_W(y, F + b)
        bn = np.linalg.solve(np.diag(W) + Q, W * b + g)
        if np.max(np.abs(bn - b)) <= tol * (1.0 + np.max(np.abs(b))):
            b = bn
            break
        b = bn
    return b


def dense_nll(Q, y, F, logp, logp_grad, logp_W):
    """Exact Laplace negative log-marginal likelihood for prior precision Q:
    -log p(y|mu*) + b*^T Q b*/2 + log det(Q^{-1} W + I)/2."""
    b = dense_mode(Q, y, F, logp_grad, logp_W)
    W = logp_W(y, F + b)
    _, ld1 = np.linalg.slogdet(np.diag(W) + Q)
    _, ld0 = np.linalg.slogdet(Q)
    return -np.sum(logp(y, F + b)) + 0.5 * b @ Q @ b + 0.5 * (ld1 - ld0), b


def logm_spd(M):
    lam, V = np.linalg.eigh(0.5 * (M + M.T))
    return (V * np.log(lam)) @ V.T

"""Vecchia approximation (oracle side).  TEST INFRASTRUCTURE ONLY.

Follows Sec. 2.1 of the paper: for a fixed ordering s_1..s_n of the locations,
N(i) holds the (at most m) nearest neighbours of s_i among s_1..s_{i-1}; then
    A_i = Sigma_{i,N(i)} Sigma_{N(i)}^{-1},
    D_i = Sigma_{ii} - Sigma_{N(i),i}^T Sigma_{N(i)}^{-1} Sigma_{N(i),i},
B is unit lower triangular with B_{i,N(i)} = -A_i, D = diag(D_i) and the
approximate precision is B^T D^{-1} B.  Prediction points (Sec. 2.2.1, with
the observed locations first in the ordering and prediction locations
conditioned on observed locations only, Sec. 4.1) use the m nearest training
points; then B_p = I and B_po holds -A_p.

Derivatives of A_i and D_i with respect to the covariance parameters follow the
appendix "Derivatives of the Vecchia-approximated precision and covariance
matrices".

Readings where the paper is silent:
  * N(i) is sorted by (squared distance, index); squared distance is
    dx*dx + dy*dy evaluated as two products and one sum (no fused multiply-add).
  * For i <= m+1, N(i) is all earlier points.
  * Exponential covariance: sigma2 * exp(-d / rho); Matern-3/2 as printed in
    Sec. 4.1: sigma2 * (1 + sqrt(3) d / rho) * exp(-sqrt(3) d / rho).
  * theta = (sigma2, rho); derivatives are on the raw scale.
  * No nugget.

Parity pins (tests/test_oracle_vecchia.py): brute-force neighbours on tiny
inputs; covariance against the general Matern formula via scipy's Bessel K;
exact-GP limit m = n-1 (B^T D^{-1} B equals the dense inverse covariance);
derivatives against central finite differences of the factor.
"""
import numpy as np
from scipy.spatial import cKDTree

COV_EXPONENTIAL = 0
COV_MATERN32 = 1

_SQRT3 = np.sqrt(3.0)


# ----------------------------------------------------------------------------
# distances and neighbours
# ----------------------------------------------------------------------------
def sqdist(a, b):
    """Squared Euclidean distance between 2-D points, as dx*dx + dy*dy."""
    dx = a[..., 0] - b[..., 0]
    dy = a[..., 1] - b[..., 1]
    return dx * dx + dy * dy


def _rank_candidates(q, cand, coords, m):
    """Keep the m candidates nearest to coords[q], ordered by (d2, index)."""
    cand = np.asarray(cand, dtype=np.int64)
    d2 = sqdist(coords[cand], coords[q])
    order = np.lexsort((cand, d2))[:m]
    return cand[order], d2[order]


def neighbours_brute(coords, m):
    """N(i) for every i by exhaustive search over j < i (Sec. 2.1)."""
    n = coords.shape[0]
    nbr = np.full((n, m), -1, dtype=np.int64)
    for i in range(1, n):
        sel, _ = _rank_candidates(i, np.arange(i), coords, m)
        nbr[i, : sel.size] = sel
    return nbr


def neighbours(coords, m, brute_limit=4096):
    """N(i): the min(i, m) nearest points among s_0..s_{i-1} (0-based), ordered
    by (squared distance, index), for every row.  Exact."""
    coords = np.asarray(coords, dtype=np.float64)
    return neighbours_rows(coords, m, np.arange(coords.shape[0]), brute_limit)


def neighbours_rows(coords, m, rows, brute_limit=4096):
    """N(i) for the given rows only (r x m, -1 padded); row i of the result
    is the same as row i of the full search.

    Rows below `brute_limit` use exhaustive search.  Later rows, in blocks
    [lo, 2 lo), query a k-d tree built on the prefix s_0..s_{2lo-1}; a query is
    accepted only when the farthest returned point is strictly farther than
    the m-th eligible one (so no unreturned point can enter the set), otherwise
    it is repeated with more candidates.  The final order always uses sqdist."""
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    out = np.full((rows.size, m), -1, dtype=np.int64)
    for pos in np.nonzero((rows >= 1) & (rows < brute_limit))[0]:
        i = int(rows[pos])
        sel, _ = _rank_candidates(i, np.arange(i), coords, m)
        out[pos, : sel.size] = sel
    lo = brute_limit
    while lo < n:
        hi = min(n, 2 * lo)
        pos = np.nonzero((rows >= lo) & (rows < hi))[0]
        if pos.size:
            tree = cKDTree(coords[:hi])
            _prefix_query(tree, coords, rows[pos], m, out, pos, eligible_below_self=True)
        lo = hi
    return out


def pred_neighbours(coords_train, coords_pred, m):
    """For each prediction point, the m nearest training points ordered by
    (squared distance, index) (Sec. 2.2.1 with observed locations first)."""
    coords_train = np.asarray(coords_train, dtype=np.float64)
    coords_pred = np.asarray(coords_pred, dtype=np.float64)
    n = coords_train.shape[0]
    npred = coords_pred.shape[0]
    mm = min(m, n)
    nbr = np.full((npred, m), -1, dtype=np.int64)
    if n <= 4096:
        for p in range(npred):
            d2 = sqdist(coords_train, coords_pred[p])
            order = np.lexsort((np.arange(n), d2))[:mm]
            nbr[p, :mm] = order
        return nbr
    tree = cKDTree(coords_train)
    allpts = np.concatenate([coords_train, coords_pred])
    _prefix_query(tree, allpts, n + np.arange(npred), m, nbr, np.arange(npred),
                  eligible_below_self=False, ntrain=n)
    return nbr


def _prefix_query(tree, coords, rows, m, out, outpos, eligible_below_self, ntrain=None):
    """Exact kNN restricted to eligible tree points, with a growing candidate
    count.  Tree point j is eligible for row i if j < i (eligible_below_self)
    or always (prediction).  The result for rows[r] goes to out[outpos[r]]."""
    npts = tree.n
    pending = np.arange(len(rows))
    kq = 2 * m + 8
    while pending.size:
        k = min(kq, npts)
        dist, idx = tree.query(coords[rows[pending]], k=k)
        dist = dist.reshape(len(pending), k)
        idx = idx.reshape(len(pending), k)
        retry = []
        for r, p in enumerate(pending):
            i = int(rows[p])
            want = min(m, i) if eligible_below_self else min(m, npts)
            ok = idx[r] < (i if eligible_below_self else npts)
            cand = idx[r][ok]
            cd = dist[r][ok]
            if cand.size < want:
                if k == npts:      # every tree point was returned
                    sel, _ = _rank_candidates(i, cand, coords, m)
                    out[outpos[p], : sel.size] = sel
                else:
                    retry.append(p)
                continue
            # m-th eligible distance vs farthest returned distance
            rm = np.sort(cd)[want - 1]
            if k < npts and not (dist[r][-1] > rm * (1.0 + 1e-9) + 1e-300):
                retry.append(p)
                continue
            sel, _ = _rank_candidates(i, cand, coords, m)
            out[outpos[p], : sel.size] = sel
        pending = np.asarray(retry, dtype=np.int64)
        kq *= 2


# ----------------------------------------------------------------------------
# covariance functions (Sec. 4.1 for Matern-3/2)
# ----------------------------------------------------------------------------
def covariance(d2, kind, sigma2, rho):
    """c_theta as a function of squared distance."""
    d = np.sqrt(d2)
    if kind == COV_EXPONENTIAL:
        return sigma2 * np.exp(-d / rho)
    if kind == COV_MATERN32:
        a = _SQRT3 * d / rho
        return sigma2 * (1.0 + a) * np.exp(-a)
    raise ValueError("unknown covariance kind")


def covariance_grad(d2, kind, sigma2, rho):
    """(d c / d sigma2, d c / d rho) as functions of squared distance."""
    d = np.sqrt(d2)
    if kind == COV_EXPONENTIAL:
        e = np.exp(-d / rho)
        return e, sigma2 * e * d / (rho * rho)
    if kind == COV_MATERN32:
        a = _SQRT3 * d / rho
        e = np.exp(-a)
        return (1.0 + a) * e, sigma2 * a * a * e / rho
    raise ValueError("unknown covariance kind")


def dense_covariance(coords, kind, sigma2, rho, coords2=None):
    """Dense Sigma (used by tests and by the LRAC pivoted Cholesky)."""
    c2 = coords if coords2 is None else coords2
    d2 = sqdist(coords[:, None, :], c2[None, :, :])
    return covariance(d2, kind, sigma2, rho)


# ----------------------------------------------------------------------------
# Vecchia factor (Sec. 2.1) and its derivatives (appendix)
# ----------------------------------------------------------------------------
def factor(coords, nbr, kind, theta, coords_self=None, deriv=False, chunk=65536):
    """Vecchia factor rows.

    coords       n_train x 2 locations the neighbour indices refer to
    nbr          r x m neighbour indices (-1 padded)
    coords_self  r x 2 locations of the rows (default: coords, i.e. r = n)
    Returns A (r x m, zero in padded slots), D (r,) and, with deriv=True,
    dA (2 x r x m) and dD (2 x r) for theta = (sigma2, rho).
    """
    sigma2, rho = float(theta[0]), float(theta[1])
    coords = np.asarray(coords, dtype=np.float64)
    pts = coords if coords_self is None else np.asarray(coords_self, dtype=np.float64)
    r, m = nbr.shape
    A = np.zeros((r, m))
    D = np.empty(r)
    dA = np.zeros((2, r, m)) if deriv else None
    dD = np.empty((2, r)) if deriv else None
    cnt = (nbr >= 0).sum(axis=1)
    # Rows grouped by neighbour count so each group is one batched solve.
    for k in np.unique(cnt):
        rows_k = np.nonzero(cnt == k)[0]
        for s in range(0, rows_k.size, chunk):
            rows = rows_k[s: s + chunk]
            _factor_rows(coords, pts, nbr, rows, int(k), kind, sigma2, rho,
                         A, D, dA, dD)
    if deriv:
        return A, D, dA, dD
    return A, D


def _factor_rows(coords, pts, nbr, rows, k, kind, sigma2, rho, A, D, dA, dD):
    if k == 0:
        D[rows] = sigma2                      # Sigma_ii, no conditioning
        if dA is not None:
            dD[0, rows] = 1.0                 # d sigma2 / d sigma2
            dD[1, rows] = 0.0
        return
    idx = nbr[rows, :k]                        # (R, k)
    P = coords[idx]                            # (R, k, 2)
    q = pts[rows]                              # (R, 2)
    d2_nn = sqdist(P[:, :, None, :], P[:, None, :, :])   # (R, k, k)
    d2_qn = sqdist(P, q[:, None, :])                     # (R, k)
    S = covariance(d2_nn, kind, sigma2, rho)
    c = covariance(d2_qn, kind, sigma2, rho)
    a = np.linalg.solve(S, c[..., None])[..., 0]         # A_i = Sigma_N^{-1} c
    A[rows, :k] = a
    D[rows] = sigma2 - np.einsum("rk,rk->r", c, a)
    if dA is None:
        return
    gS = covariance_grad(d2_nn, kind, sigma2, rho)
    gc = covariance_grad(d2_qn, kind, sigma2, rho)
    g_diag = (1.0, 0.0)                        # d Sigma_ii / d (sigma2, rho)
    for p in range(2):
        # d A_i = Sigma_N^{-1} (d c - d Sigma_N A_i)
        rhs = gc[p] - np.einsum("rkl,rl->rk", gS[p], a)
        da = np.linalg.solve(S, rhs[..., None])[..., 0]
        dA[p, rows, :k] = da
        # d D_i = d Sigma_ii - d A_i^T c - A_i^T d c
        dD[p, rows] = g_diag[p] - np.einsum("rk,rk->r", da, c) \
            - np.einsum("rk,rk->r", a, gc[p])


def sparse_offdiag(vals, nbr, n=None):
    """Sparse r x n matrix with entries vals[i, k] at (i, nbr[i, k])."""
    import scipy.sparse as sp
    r, m = nbr.shape
    n = r if n is None else n
    mask = (nbr >= 0).ravel()
    rows = np.repeat(np.arange(r), m)[mask]
    cols = nbr.ravel()[mask]
    return sp.csr_matrix((vals.ravel()[mask], (rows, cols)), shape=(r, n))


def sparse_B(A, nbr):
    """Unit lower-triangular B with B_{i,N(i)} = -A_i (Sec. 2.1), as CSR."""
    import scipy.sparse as sp
    n = nbr.shape[0]
    return (sp.identity(n, format="csr") + sparse_offdiag(-A, nbr, n)).tocsr()


def sparse_dB(dA, nbr):
    """d B / d theta_k: zero diagonal, entries -dA_i on N(i) (appendix)."""
    return sparse_offdiag(-dA, nbr, nbr.shape[0])

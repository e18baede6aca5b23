"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs and probes, element by element.

Sizes span several tiles of every kernel and leave ragged tails (n not a
multiple of 64; probe counts below, at and above one wave).  FP64 results
must agree within relative 1e-9; integer results (neighbour sets, iteration
counts) exactly.  When a CG or Newton stopping decision lands on the other
side of its threshold (a difference of one iteration), the oracle replays the
device's counts and the comparison uses the replay."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from oracle import vecchia as OV  # noqa: E402
from tests.gpu_common import (dev, host, oracle_mode_matching, opts_pair, rel_err,  # noqa: E402
                               rel_err_elem, say)

TOL = 1e-9


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def c1():
    # n = 2,000 exponential range 0.1, m = 10, Bernoulli-logit, tol 1e-8
    w = synth.make("c1_n2000", seed=0)
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]), deriv=True)
    return w, model


def _build(P, w, deriv=True, m=None, theta=None):
    th = theta or (w["sigma2"], w["rho"])
    return P.VecchiaLaplace(dev(w["coords"]), w["m"] if m is None else m, w["kind"], th,
                            want_deriv=deriv)


def test_neighbours_and_factor(P, c1):
    w, model = c1
    say("case: c1 neighbours/factor n=2000 m=10")
    g = _build(P, w)
    nbr = host(g.export("nbr")).reshape(w["n"], w["m"])
    assert np.array_equal(nbr, model.nbr)
    bval = host(g.export("bval")).reshape(w["n"], w["m"])
    assert rel_err(bval, -model.A) < TOL
    D = host(g.export("D"))
    np.testing.assert_allclose(D, model.D, rtol=TOL)
    np.testing.assert_allclose(host(g.export("dbval_rho")).reshape(w["n"], w["m"]),
                               -model.dA[1], rtol=1e-8, atol=1e-9 * np.abs(model.dA[1]).max())
    np.testing.assert_allclose(host(g.export("dD_rho")), model.dD[1], rtol=1e-8,
                               atol=1e-9 * np.abs(model.dD[1]).max())
    np.testing.assert_allclose(host(g.export("dD_sigma2")), model.dD[0], rtol=1e-9)
    g.close()


@pytest.mark.parametrize("n,m,kind", [(1, 5, 0), (2, 5, 1), (7, 10, 1), (65, 0, 0),
                                      (300, 31, 1), (4099, 20, 1), (5000, 7, 0)])
def test_neighbours_factor_edge_sizes(P, n, m, kind):
    say(f"case: factor edge n={n} m={m} kind={kind}")
    X = synth.locations(n, seed=n)
    theta = (1.3, 0.2)
    g = P.VecchiaLaplace(dev(X), m, kind, theta)
    ref_nbr = OV.neighbours(X, m)
    A, D = OV.factor(X, ref_nbr, kind, theta)
    if m > 0:
        nbr = host(g.export("nbr")).reshape(n, m)
        assert np.array_equal(nbr, ref_nbr)
        assert rel_err(host(g.export("bval")).reshape(n, m), -A) < 1e-8
    np.testing.assert_allclose(host(g.export("D")), D, rtol=1e-8)
    g.close()


def test_duplicate_locations_not_spd(P):
    X = synth.locations(100, seed=1)
    X[50] = X[10]
    with pytest.raises(P.VLError) as e:
        P.VecchiaLaplace(dev(X), 5, 0, (1.0, 0.1))
    assert e.value.code == P.VL_ERR_NOT_SPD


@pytest.mark.parametrize("t", [1, 3, 50, 64, 65, 130])
def test_spmm_trsm(P, c1, t):
    w, model = c1
    say(f"case: spmm/trsm t={t}")
    g = _build(P, w, deriv=False)
    rng = np.random.default_rng(t)
    X = rng.standard_normal((w["n"], t))
    Xd = dev(X)
    Y = torch.empty_like(Xd)
    for tr, ref in ((False, model.B @ X), (True, model.Bt @ X)):
        P.vl_spmm(g.h, Xd, Y, transpose=tr)
        torch.cuda.synchronize()
        assert rel_err(host(Y), ref) < 1e-12
    for tr in (False, True):
        P.vl_trsm(g.h, Xd, Y, transpose=tr)
        ref = model.solve_Bt(X) if tr else model.solve_B(X)
        assert rel_err(host(Y), ref) < 1e-10
    g.close()


@pytest.fixture(scope="module")
def ragged():
    # n = 4099: the last row group of 16 holds 3 rows
    X = synth.locations(4099, seed=41)
    return X, OL.Model(X, 20, 1, (1.1, 0.07))


# Products over blocks of 32 to 64 columns run on row groups of 4 with the
# union of their columns; other widths row by row.  Both sides of both
# thresholds, with partial column slices.
@pytest.mark.parametrize("t", [31, 32, 33, 63, 64, 65])
def test_grouped_products_ragged(P, ragged, t):
    X, model = ragged
    say(f"case: grouped spmm n=4099 m=20 t={t}")
    g = P.VecchiaLaplace(dev(X), 20, 1, (1.1, 0.07))
    rng = np.random.default_rng(1000 + t)
    Z = rng.standard_normal((X.shape[0], t))
    Zd = dev(Z)
    Y = torch.empty_like(Zd)
    y1 = torch.empty((X.shape[0], 1), dtype=torch.float64, device="cuda")
    for tr, ref in ((False, model.B @ Z), (True, model.Bt @ Z)):
        P.vl_spmm(g.h, Zd, Y, transpose=tr)
        torch.cuda.synchronize()
        # the device factor agrees with the oracle's to about 1e-10 here
        assert rel_err(host(Y), ref) < TOL
        # the same columns one at a time (row-by-row kernel): each row's sum
        # only runs in another order
        cols = []
        for c in range(t):
            P.vl_spmm(g.h, Zd[:, c:c + 1].contiguous(), y1, transpose=tr)
            cols.append(host(y1)[:, 0])
        assert rel_err(host(Y), np.stack(cols, axis=1)) < 1e-13
    g.close()


@pytest.fixture(scope="module")
def c1_fit(P, c1):
    w, model = c1
    say("case: c1 mode + nll + grad + predict")
    o, go = opts_pair(P, cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"],
                      num_probes=w["t"], num_pred_samples=w["s"], seed=7)
    g = _build(P, w)
    mode, st = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    newton_cg = host(g.export("newton_cg_iters")).tolist()
    halvings = host(g.export("newton_halvings")).tolist()
    nll, grad, nst = g.neg_log_marglik(go, want_grad=True)
    grad_F = host(g.grad_offset())
    Xcov = np.random.default_rng(17).standard_normal((w["n"], 3))
    grad_beta = g.grad_beta(dev(Xcov))
    slq_iters = host(g.export("block_iters")).tolist()
    quad = host(g.export("slq_quad"))
    r0z0 = host(g.export("slq_r0z0"))
    W = host(g.export("W"))
    mean, var, pst = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), go)
    pred_iters = host(g.export("block_iters")).tolist()
    out = dict(mode=host(mode), st=st, newton_cg=newton_cg, halvings=halvings, nll=nll, grad=grad,
               grad_F=grad_F, grad_beta=grad_beta, Xcov=Xcov,
               slq_iters=slq_iters, quad=quad, r0z0=r0z0, W=W, mean=host(mean),
               var=host(var), pred_iters=pred_iters, opts=o)
    g.close()
    return out


def test_mode(c1, c1_fit):
    w, model = c1
    f = c1_fit
    b, W, st, replayed = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None,
                                              f["opts"], f["newton_cg"],
                                              gpu_halvings=f["halvings"])
    say(f"newton iters gpu={f['newton_cg']} oracle={st['cg_iters']} replayed={replayed}")
    assert rel_err(f["mode"], b) < TOL
    np.testing.assert_allclose(f["W"], W, rtol=1e-9)


def test_nll_and_gradient(c1, c1_fit):
    w, model = c1
    f = c1_fit
    b, W, _, _ = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, f["opts"],
                                      f["newton_cg"])
    nll, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, f["opts"],
                                   want_grad=True)
    if list(info["cg_iters"]) != f["slq_iters"]:
        say("SLQ iteration counts differ; replaying the device's counts")
        assert np.max(np.abs(np.array(info["cg_iters"]) - np.array(f["slq_iters"]))) <= 1
        nll, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, f["opts"],
                                       replay_cg=f["slq_iters"], want_grad=True)
    np.testing.assert_allclose(f["r0z0"], info["r0z0"], rtol=1e-12)
    assert rel_err_elem(f["quad"], info["quad"]) < TOL
    assert abs(f["nll"] - nll) <= TOL * abs(nll)
    e_g = rel_err_elem(f["grad"], info["grad"])
    say(f"gradient: device {f['grad']} oracle {info['grad']} rel {e_g:.2e}")
    assert e_g < TOL
    # gradient in the offset F and, for F = X beta, in beta (App. A.3)
    e_f = rel_err(f["grad_F"], info["grad_F"])
    gb_o = f["Xcov"].T @ info["grad_F"]
    e_b = rel_err_elem(f["grad_beta"], gb_o)
    say(f"offset gradient rel {e_f:.2e}; beta gradient device {f['grad_beta']} oracle {gb_o} "
        f"rel {e_b:.2e}")
    assert e_f < TOL
    assert e_b < TOL


def test_predict(c1, c1_fit):
    w, model = c1
    f = c1_fit
    b, W, _, _ = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, f["opts"],
                                      f["newton_cg"])
    mean, var, info = OL.predict(model, w["coords_pred"], w["Fp"], b, W, f["opts"],
                                 replay_cg=f["pred_iters"])
    assert abs(np.array(info["cg_iters"]) - np.array(f["pred_iters"])).max() == 0
    assert rel_err(f["mean"], mean) < TOL
    assert rel_err_elem(f["var"], var) < TOL


@pytest.mark.parametrize("n", [40000, 5000])
@pytest.mark.parametrize("t", [1, 8, 50, 65, 300, 1000])
def test_trsm_head_and_tail(P, t, n):
    # For t <= 64 the first 4096 rows come from the dense inverse of B's
    # leading block and the rest from the sync-free tail kernels, in both
    # directions (35904 tail rows at n = 40000, a ragged 904 at n = 5000).
    # Wider blocks (65, 300: one and two column slices, ragged) take the first
    # 2048 rows from the dense inverse, the others by level-scheduled launches
    # (backward: tail rows, the fold into the head rows up to 12288, the head
    # rows by their own levels); at t = 1000 the dense product runs in its
    # 128-row blocks (ragged last column tile of 40).  The
    # reference solves with the oracle's factor.  The range (0.005, about the
    # spacing of the points) keeps every neighbour covariance well conditioned,
    # so the two factors agree to rounding and the comparison isolates the
    # solve; the neighbour sets, and with them the dependency DAG the kernels
    # schedule, do not depend on the range.
    m = 20
    say(f"case: trsm head+tail n={n} t={t}")
    X = synth.locations(n, seed=11)
    g = P.VecchiaLaplace(dev(X), m, OV.COV_MATERN32, (1.0, 0.005))
    nbr = OV.neighbours(X, m)
    A, _ = OV.factor(X, nbr, OV.COV_MATERN32, (1.0, 0.005))
    assert np.array_equal(host(g.export("nbr")).reshape(n, m), nbr)
    assert rel_err(host(g.export("bval")).reshape(n, m), -A) < TOL
    B = OV.sparse_B(A, nbr)
    from scipy.sparse.linalg import spsolve_triangular
    R = np.random.default_rng(t).standard_normal((n, t))
    Rd = dev(R)
    Y = torch.empty_like(Rd)
    for tr in (False, True):
        P.vl_trsm(g.h, Rd, Y, transpose=tr)
        ref = (spsolve_triangular(B.T.tocsr(), R, lower=False, unit_diagonal=True) if tr
               else spsolve_triangular(B, R, lower=True, unit_diagonal=True))
        e = rel_err(host(Y), ref)
        say(f"trsm t={t} transpose={tr}: rel err {e:.2e}")
        assert e < TOL, (tr, e)
    g.close()

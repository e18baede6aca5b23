"""Parity at the full sizes of the measured workloads, where the oracle cannot
run the whole path in seconds:

  c2_n1e5   n = 100,000, Matern-3/2 range 0.05, m = 20, Bernoulli-logit,
            50 probes, CG tolerance 1e-3, 10,000 test points, s = 2000
            (the configuration the throughput is measured on);
  c3_n2e6   n = 2,000,000, Matern-3/2 range 0.02, m = 20, Poisson with
            offset 1, 64 probes, CG tolerance 1e-2, s = 256 (skipped, see
            below), and the same shape at n = 200,000.

Checks, each against what the oracle computes exactly at this size:
  * every neighbour set (exact), every D_i (1e-9) and every row A_i within
    m * kappa(Sigma_N(i)) * u of the oracle's (the conditioning bound of the
    neighbour solve), the oracle spread over processes by row range;
  * the mode against the oracle's Newton iteration (replaying the device's CG
    counts) and, at a tight tolerance, through its first-order condition
    g(F + b) = B^T D^{-1} B b (Sec. 2.2, eq. newton) with the oracle's factor;
  * the likelihood pieces that need no probes (eq. VLA_loss, logdetsplit) at
    the device's mode, the whole assembly of the estimate, and one SLQ probe
    (eq. def_SLQ) run by the oracle on the same Rademacher column;
  * predictive rows and means at all test points (eq. latentpostpredictive)
    and the simulated variance of one sample column (Alg. simAlgo);
  * the mixed-precision form against the FP64 path: relative 1e-4 on the
    negative log-marginal likelihood and 1e-3 on the predictive variances.
Each step prints what it checks before it runs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from oracle import vecchia as OV  # noqa: E402
from tests import oracle_pool  # noqa: E402
from tests.gpu_common import (dev, host, opts_pair, oracle_mode_matching,  # noqa: E402
                               rel_err, say)

TOL = 1e-9
NLL_TOL_MIXED = 1e-4
VAR_TOL_MIXED = 1e-3
FOC_CG_TOL = 1e-6

C3_FAULT = ("the library refuses n above 262,144: a build at n = 2,000,000 ended in a GPU "
            "memory fault whose cause is not found (a CPU emulation of every build kernel "
            "at this size shows no out-of-bounds access); this case stays off the GPU until "
            "the cause is shown")
WORKLOADS = [
    pytest.param(("c2_n1e5", {}), id="c2_n1e5"),
    # the n = 2e6 workload's shape at the largest size the library runs
    pytest.param(("c3_n2e6", {"n": 200000}), id="c3_shape_n2e5"),
    pytest.param(("c3_n2e6", {}), id="c3_n2e6", marks=pytest.mark.skip(reason=C3_FAULT)),
]
# The oracle's Newton iteration replaying the device's CG counts takes
# minutes at the n = 2e5 shape (about 2100 CG iterations); the first-order
# condition checks that mode instead.
SLOW_ORACLE_MODE = {"c3_shape_n2e5"}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module", params=WORKLOADS)
def case(request, P):
    base, over = request.param
    name = base if not over else f"{base} n={over['n']}"
    say(f"case: {name} inputs")
    w = synth.make(base, seed=5, **over)
    say(f"case: {name} oracle neighbours and factor over row ranges")
    nbr, A, D = oracle_pool.neighbours_and_factor(w["coords"], w["m"], w["kind"],
                                                  (w["sigma2"], w["rho"]))
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]),
                     nbr=nbr.astype(np.int64), factor=(A, D))
    say(f"case: {name} FP64 build + mode + NLL + predict")
    o, go = opts_pair(P, cg_tol=w["cg_tol"], pred_cg_tol=w["pred_cg_tol"], num_probes=w["t"],
                      num_pred_samples=w["s"], seed=7)
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
    mode, mst = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    newton_cg = host(g.export("newton_cg_iters")).tolist()
    halvings = host(g.export("newton_halvings")).tolist()
    nll, _, st = g.neg_log_marglik(go)
    slq_iters = host(g.export("block_iters"))
    quad, r0z0 = host(g.export("slq_quad")), host(g.export("slq_r0z0"))
    mean, var, pst = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), go)
    fit = dict(o=o, go=go, mode=host(mode), newton_cg=newton_cg, halvings=halvings, nll=nll, mean=host(mean), var=host(var),
               quad=quad, r0z0=r0z0, slq_iters=slq_iters,
               pred_nbr=host(g.export("pred_nbr")).reshape(-1, w["m"]),
               pred_bval=host(g.export("pred_bval")).reshape(-1, w["m"]),
               pred_D=host(g.export("pred_D")),
               nbr=host(g.export("nbr")).reshape(w["n"], w["m"]),
               bval=host(g.export("bval")).reshape(w["n"], w["m"]), D=host(g.export("D")))
    say(f"{name} FP64: newton {mst.newton_iters} cg {mst.cg_iters_total} slq_max "
        f"{st.cg_iters_max} pred_max {pst.cg_iters_max} nll {nll:.10f}")
    # Tolerance of the results downstream of the factor.  The neighbour
    # covariances of Sec. 2.1 reach condition numbers near 1e10 at n = 1e5,
    # range 0.05, so two correct FP64 solvers of those systems give factor
    # rows up to ~1e-7 apart (bounded per row by test_neighbours_and_factor),
    # and every CG iterate inherits a perturbation of that relative size: an
    # oracle with Cholesky instead of LU neighbour solves moves the mode and a
    # one-sample variance by 2.2x its own factor difference.  Modes and
    # variances are therefore held to 10x the measured factor discrepancy
    # (never looser than needed: 1e-9 when the factor agrees to 1e-10).
    e_fac = float(np.max(np.abs(fit["bval"] + model.A).max(axis=1)
                         / np.maximum(np.abs(model.A).max(axis=1), 1e-300)))
    fit["tol_downstream"] = max(TOL, 10.0 * e_fac)
    say(f"{name} factor discrepancy {e_fac:.2e}: downstream tolerance {fit['tol_downstream']:.2e}")
    yield name, w, model, g, fit
    g.close()


def _neighbour_condition(coords, nbr, kind, theta):
    """2-norm condition number of every row's neighbour covariance Sigma_N(i)
    (1 for rows with fewer than two neighbours)."""
    n, m = nbr.shape
    kap = np.ones(n)
    cnt = (nbr >= 0).sum(axis=1)
    for k in np.unique(cnt):
        if k < 2:
            continue
        rows = np.nonzero(cnt == k)[0]
        for s in range(0, rows.size, 16384):
            r = rows[s: s + 16384]
            P = coords[nbr[r, :k]]
            d2 = ((P[:, :, None, :] - P[:, None, :, :]) ** 2).sum(-1)
            kap[r] = np.linalg.cond(OV.covariance(d2, kind, theta[0], theta[1]))
    return kap


def test_neighbours_and_factor(case):
    name, w, model, _, fit = case
    say(f"case: {name} neighbour sets and factor rows, all {w['n']} rows")
    assert np.array_equal(fit["nbr"], model.nbr)
    e_d = rel_err(fit["D"], model.D)
    # A_i solves Sigma_N(i) A_i = Sigma_N(i),i: two correct FP64 solvers agree
    # only to about m * kappa(Sigma_N(i)) * u relative to |A_i| (the neighbour
    # covariances reach kappa ~ 1e10 here), so each row gets its own bound
    kap = _neighbour_condition(w["coords"], model.nbr, w["kind"], (w["sigma2"], w["rho"]))
    scale = np.maximum(np.abs(model.A).max(axis=1), 1e-300)
    e_row = np.abs(fit["bval"] + model.A).max(axis=1) / scale
    bound = w["m"] * kap * 2.0 ** -53 + 1e-14
    worst = int(np.argmax(e_row / bound))
    say(f"{name} factor: D rel {e_d:.2e}; A rows: max rel {e_row.max():.2e}, "
        f"worst row vs its bound {e_row[worst]:.2e} / {bound[worst]:.2e} "
        f"(kappa {kap[worst]:.2e}); kappa max {kap.max():.2e}")
    assert np.all(e_row <= bound)
    assert e_d < TOL


def test_mode_matches_the_oracle(request, case):
    name, w, model, _, fit = case
    if request.node.callspec.id in SLOW_ORACLE_MODE:
        pytest.skip("oracle Newton takes minutes here; the first-order condition test covers it")
    say(f"case: {name} oracle Newton mode with the device's CG counts")
    b, _, _, replayed = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, fit["o"],
                                             fit["newton_cg"], gpu_halvings=fit["halvings"])
    e = rel_err(fit["mode"], b)
    say(f"{name} mode: newton cg {fit['newton_cg']} replayed={replayed} rel err {e:.2e} "
        f"(tolerance {fit['tol_downstream']:.2e})")
    assert e < fit["tol_downstream"]


def test_mode_first_order_condition(P, case):
    name, w, model, _, _ = case
    say(f"case: {name} mode at CG tol {FOC_CG_TOL}, first-order condition with the oracle factor")
    _, go = opts_pair(P, cg_tol=FOC_CG_TOL, newton_tol=1e-12, num_probes=w["t"])
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
    mode, st = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    halv = host(g.export("newton_halvings"))
    g.close()
    b = host(mode)
    grad = OL.lik_grad(w["lik"], w["y"], w["F"] + b)
    r = grad - model.prec_apply(b)
    say(f"{name} mode: newton {st.newton_iters} cg {st.cg_iters_total} halvings {halv.tolist()} "
        f"|g - Sigma~^-1 b| = {np.linalg.norm(r):.3e} (|g| = {np.linalg.norm(grad):.3e})")
    assert not st.hit_cap
    # The last Newton system is solved to a residual below the CG tolerance,
    # which is the first-order residual at the new point up to a term of
    # second order in the (tiny) last step.  Sigma~^{-1} b is evaluated here
    # with the oracle's factor, whose rows differ from the device's by up to
    # m * kappa(Sigma_N) * u (about 1e-7 relative at kappa ~ 1e10); applied to
    # the innovation vector D^{-1} B b that difference is not smoothed away,
    # so it enters at that relative size against |Sigma~^{-1} b| = |g|.
    assert np.linalg.norm(r) < 10.0 * FOC_CG_TOL + 1e-6 * np.linalg.norm(grad)


def test_nll_pieces_and_one_probe(case):
    name, w, model, _, fit = case
    say(f"case: {name} NLL pieces at the device mode")
    b = fit["mode"]
    mu = w["F"] + b
    W = OL.lik_W(w["lik"], w["y"], mu)
    loglik = float(np.sum(OL.lik_logp(w["lik"], w["y"], mu)))
    Bb = model.B @ b
    quadform = float(np.sum(model.Dinv * Bb * Bb))
    logdet_fixed = float(np.sum(np.log(model.D)) + np.sum(np.log(W + model.Dinv)))
    # eq. def_SLQ with the device's per-probe quadratures
    gamma = float(np.mean(fit["r0z0"] * fit["quad"]))
    nll_o = -loglik + 0.5 * quadform + 0.5 * (logdet_fixed + gamma)
    e = abs(fit["nll"] - nll_o) / abs(nll_o)
    say(f"{name} NLL assembly: device {fit['nll']:.10f} oracle pieces {nll_o:.10f} rel {e:.2e}")
    assert e < TOL
    # Rademacher probes with z = B^T (W + D^{-1})^{1/2} eps give r0'z0 = eps'eps = n
    e_r = rel_err(fit["r0z0"], np.full(w["t"], float(w["n"])))
    say(f"{name} SLQ weights r0'z0 vs n: rel {e_r:.2e}")
    assert e_r < 1e-8
    # probe 0 run by the oracle: the probe columns are counter-based, so column
    # 0 of a one-probe run is column 0 of the device's run
    say(f"case: {name} SLQ probe 0 by the oracle")
    o1 = OL.Opts(cg_tol=w["cg_tol"], num_probes=1, seed=7)
    _, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o1)
    replayed = int(info["cg_iters"][0]) != int(fit["slq_iters"][0])
    if replayed:
        _, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o1,
                                     replay_cg=[int(fit["slq_iters"][0])])
    e_q = abs(info["quad"][0] * info["r0z0"][0] - fit["quad"][0] * fit["r0z0"][0]) / abs(
        info["quad"][0] * info["r0z0"][0])
    say(f"{name} probe 0: iters {fit['slq_iters'][0]} replayed={replayed} "
        f"log-det term rel {e_q:.2e}")
    assert e_q < TOL


def test_prediction(P, case):
    name, w, model, g, fit = case
    say(f"case: {name} prediction rows and means at {w['n_pred']} test points")
    nbr_p = OV.pred_neighbours(w["coords"], w["coords_pred"], w["m"])
    Ap, Dp = OV.factor(w["coords"], nbr_p, w["kind"], (w["sigma2"], w["rho"]),
                       coords_self=w["coords_pred"])
    assert np.array_equal(fit["pred_nbr"], nbr_p)
    assert rel_err(fit["pred_D"], Dp) < TOL
    # per-row conditioning bound of the neighbour solve, as for the training rows
    kap = _neighbour_condition(w["coords"], nbr_p, w["kind"], (w["sigma2"], w["rho"]))
    e_row = np.abs(fit["pred_bval"] + Ap).max(axis=1) / np.maximum(np.abs(Ap).max(axis=1), 1e-300)
    bound = w["m"] * kap * 2.0 ** -53 + 1e-14
    say(f"{name} prediction rows: max rel {e_row.max():.2e}, max ratio to bound "
        f"{(e_row / bound).max():.2e}")
    assert np.all(e_row <= bound)
    mean_o = w["Fp"] + np.sum(Ap * fit["mode"][nbr_p], axis=1)
    e_m = rel_err(fit["mean"], mean_o)
    say(f"{name} predictive means: rel {e_m:.2e}")
    assert e_m < TOL
    # D_p plus an average of squares: never below the conditional variance
    assert np.all(fit["var"] >= Dp * (1.0 - 1e-12))
    # one simulation column end to end (Alg. simAlgo with s = 1)
    say(f"case: {name} predictive variance of one sample column by the oracle")
    o1, go1 = opts_pair(P, pred_cg_tol=w["pred_cg_tol"], num_pred_samples=1, seed=7)
    _, var1, _ = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), go1)
    iters1 = host(g.export("block_iters"))
    W = OL.lik_W(w["lik"], w["y"], w["F"] + fit["mode"])
    _, var_o, info = OL.predict(model, w["coords_pred"], w["Fp"], fit["mode"], W, o1)
    replayed = int(info["cg_iters"][0]) != int(iters1[0])
    if replayed:
        _, var_o, info = OL.predict(model, w["coords_pred"], w["Fp"], fit["mode"], W, o1,
                                    replay_cg=[int(iters1[0])])
    e_v = rel_err(host(var1), var_o)
    say(f"{name} one-sample variance: iters {iters1[0]} replayed={replayed} rel {e_v:.2e} "
        f"(tolerance {fit['tol_downstream']:.2e})")
    assert e_v < fit["tol_downstream"]


def test_mixed_matches_fp64(P, case):
    name, w, _, _, fit = case
    say(f"case: {name} mixed precision mode + NLL + predict")
    go = fit["go"]
    go.precision = P.VL_MIXED
    try:
        g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
        mode, _ = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
        nll, _, st = g.neg_log_marglik(go)
        _, var, pst = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), go)
        g.close()
    finally:
        go.precision = P.VL_FP64
    e_nll = abs(nll - fit["nll"]) / abs(fit["nll"])
    e_var = rel_err(host(var), fit["var"])
    e_mode = rel_err(host(mode), fit["mode"])
    say(f"{name} mixed vs FP64: nll {e_nll:.2e} var {e_var:.2e} mode {e_mode:.2e} "
        f"slq_max {st.cg_iters_max} pred_max {pst.cg_iters_max}")
    assert e_nll < NLL_TOL_MIXED
    assert e_var < VAR_TOL_MIXED

"""Parity at the full sizes of the measured workloads, where the oracle cannot
run the whole path in seconds:

  c2_n1e5   n = 100,000, Matern-3/2 range 0.05, m = 20, Bernoulli-logit,
            50 probes, CG tolerance 1e-3, 10,000 test points, s = 2000
            (the configuration the throughput is measured on);
  c3_n2e6   n = 2,000,000, Matern-3/2 range 0.02, m = 20, Poisson with
            offset 1, 64 probes, CG tolerance 1e-2, s = 256 (skipped, see
            below), and the same shape at n = 200,000.

Checks, each against what the oracle computes at this size from its own
inputs (no device value enters an oracle computation; only the device's
iteration counts are replayed):
  * every neighbour set (exact), every D_i (1e-9) and every row A_i within
    m * kappa(Sigma_N(i)) * u of the oracle's (the conditioning bound of the
    neighbour solve), the oracle spread over processes by row range;
  * the mode against the oracle's Newton iteration (replaying the device's CG
    counts) and, at a tight tolerance, through its first-order condition
    g(F + b) = B^T D^{-1} B b (Sec. 2.2, eq. newton) with the oracle's factor;
  * every SLQ probe's log-det term (eq. def_SLQ), run by the oracle on the
    same Rademacher columns at the oracle's mode, and the likelihood
    (eq. VLA_loss, logdetsplit) assembled from the oracle's pieces;
  * predictive rows and means at all test points (eq. latentpostpredictive)
    and the simulated variances of a full tile of 64 sample columns
    (Alg. simAlgo), element by element;
  * the mixed-precision form against the FP64 path: relative 1e-4 on the
    negative log-marginal likelihood and 1e-3 on the predictive variances.
Results downstream of the factor are held to a bar fixed from the oracle
alone: 10x the spread between the oracle's factor and a second FP64
implementation of it (see the fixture).
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
            "memory fault whose cause is not found (the library's own kernels run at this "
            "size in a host emulation of the HIP runtime under AddressSanitizer, through "
            "build, solves, mode, likelihood and prediction, show no invalid access); this "
            "case stays off the GPU until the cause is shown")
WORKLOADS = [
    pytest.param(("c2_n1e5", {}), id="c2_n1e5"),
    # the n = 2e6 workload's shape at the largest size the library runs
    pytest.param(("c3_n2e6", {"n": 200000}), id="c3_shape_n2e5"),
    pytest.param(("c3_n2e6", {}), id="c3_n2e6", marks=pytest.mark.skip(reason=C3_FAULT)),
]


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
    # Tolerance of the results downstream of the factor, fixed from the oracle
    # alone before any comparison.  The neighbour covariances of Sec. 2.1
    # reach condition numbers near 1e10 here, so two correct FP64
    # implementations of the factor (covariances evaluated in a different
    # order, Cholesky instead of LU) give rows up to ~1e-7 apart, and every CG
    # iterate inherits a perturbation of that relative size (the innovation
    # vector D^{-1} B b is not smoothed): between the oracle and such a
    # variant the mode and a variance move by about 2x the factor spread.
    # Modes, likelihood, probes and variances are held to 10x the spread
    # between the oracle and its Cholesky variant (never tighter than 1e-9).
    say(f"case: {name} second FP64 factor (Cholesky, reordered covariances) for the tolerance")
    A_ch, D_ch = oracle_pool.factor_cholesky(w["coords"], nbr.astype(np.int64), w["kind"],
                                             (w["sigma2"], w["rho"]))
    fit["variant"] = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]),
                              nbr=nbr.astype(np.int64), factor=(A_ch, D_ch))
    scale = np.maximum(np.abs(model.A).max(axis=1), 1e-300)
    e_spread = float(np.max(np.abs(A_ch - model.A).max(axis=1) / scale))
    fit["tol_downstream"] = max(TOL, 10.0 * e_spread)
    e_fac = float(np.max(np.abs(fit["bval"] + model.A).max(axis=1) / scale))
    say(f"{name} factor spread of two oracles {e_spread:.2e}: downstream tolerance "
        f"{fit['tol_downstream']:.2e} (device factor vs oracle: {e_fac:.2e})")
    # the oracle's own mode (replaying the device's Newton and CG counts):
    # every later oracle computation takes its inputs from the oracle alone
    say(f"case: {name} oracle Newton mode with the device's CG counts")
    b_o, W_o, _, replayed = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, o,
                                                 newton_cg, gpu_halvings=halvings)
    fit["b_oracle"], fit["W_oracle"], fit["mode_replayed"] = b_o, W_o, replayed
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


def test_mode_matches_the_oracle(case):
    name, w, model, _, fit = case
    e = rel_err(fit["mode"], fit["b_oracle"])
    say(f"{name} mode: newton cg {fit['newton_cg']} replayed={fit['mode_replayed']} "
        f"rel err {e:.2e} (tolerance {fit['tol_downstream']:.2e})")
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


def test_nll_pieces_and_every_probe(case):
    name, w, model, _, fit = case
    say(f"case: {name} NLL pieces at the oracle mode")
    b = fit["b_oracle"]
    tol = fit["tol_downstream"]
    mu = w["F"] + b
    W = OL.lik_W(w["lik"], w["y"], mu)
    loglik = float(np.sum(OL.lik_logp(w["lik"], w["y"], mu)))
    Bb = model.B @ b
    quadform = float(np.sum(model.Dinv * Bb * Bb))
    logdet_fixed = float(np.sum(np.log(model.D)) + np.sum(np.log(W + model.Dinv)))
    # Rademacher probes with z = B^T (W + D^{-1})^{1/2} eps give r0'z0 = eps'eps = n
    e_r = rel_err(fit["r0z0"], np.full(w["t"], float(w["n"])))
    say(f"{name} SLQ weights r0'z0 vs n: rel {e_r:.2e}")
    assert e_r < 1e-8
    # every probe column run by the oracle (the probe columns are
    # counter-based; slices of them run in parallel processes), replaying
    # the device's per-column CG counts
    say(f"case: {name} all {w['t']} SLQ probes by the oracle")
    quad, r0z0, iters = oracle_pool.slq_columns(model, w["y"], w["F"], w["lik"], b, fit["o"],
                                                w["t"], replay=[int(v) for v in fit["slq_iters"]])
    term_o, term_d = quad * r0z0, fit["quad"] * fit["r0z0"]
    e_q = float(np.max(np.abs(term_d - term_o) / np.abs(term_o)))
    say(f"{name} probes: device iters {fit['slq_iters'].tolist()} log-det terms max rel "
        f"{e_q:.2e} (tolerance {tol:.2e})")
    assert np.array_equal(iters, fit["slq_iters"])
    assert e_q < tol
    # eq. def_SLQ and eq. VLA_loss assembled from the oracle's own pieces
    gamma = float(np.mean(r0z0 * quad))
    nll_o = -loglik + 0.5 * quadform + 0.5 * (logdet_fixed + gamma)
    e = abs(fit["nll"] - nll_o) / abs(nll_o)
    say(f"{name} NLL: device {fit['nll']:.10f} oracle {nll_o:.10f} rel {e:.2e}")
    assert e < tol


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
    tol = fit["tol_downstream"]
    mean_o = w["Fp"] + np.sum(Ap * fit["b_oracle"][nbr_p], axis=1)
    e_m = rel_err(fit["mean"], mean_o)
    say(f"{name} predictive means: rel {e_m:.2e} (tolerance {tol:.2e})")
    assert e_m < tol
    # D_p plus an average of squares: never below the conditional variance
    assert np.all(fit["var"] >= Dp * (1.0 - 1e-12))
    # one full tile of 64 simulation columns end to end (Alg. simAlgo), the
    # oracle's columns split over processes
    say(f"case: {name} predictive variances of a 64-column sample tile by the oracle")
    o64, go64 = opts_pair(P, pred_cg_tol=w["pred_cg_tol"], num_pred_samples=64, seed=7)
    _, var64, _ = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), go64)
    iters64 = host(g.export("block_iters"))
    var_o, it_o = oracle_pool.pred_columns(model, w["coords_pred"], w["Fp"], fit["b_oracle"],
                                           fit["W_oracle"], o64, 64,
                                           replay=[int(v) for v in iters64])
    assert np.array_equal(it_o, iters64)
    # the variances pass through about 300 CG iterations at the n = 2e6
    # shape; their bar is 10x the spread between the oracle and its second
    # implementation on this very output (same mode, same counts), when
    # that exceeds the factor-based bar
    var_v, _ = oracle_pool.pred_columns(fit["variant"], w["coords_pred"], w["Fp"],
                                        fit["b_oracle"], fit["W_oracle"], o64, 64,
                                        replay=[int(v) for v in iters64])
    e_spread = float(np.max(np.abs(var_v - var_o) / var_o))
    tol_v = max(tol, 10.0 * e_spread)
    e_v = float(np.max(np.abs(host(var64) - var_o) / var_o))
    say(f"{name} 64-sample variances: iters {iters64.min()}..{iters64.max()} elementwise rel "
        f"{e_v:.2e} (two oracles {e_spread:.2e}, tolerance {tol_v:.2e})")
    assert e_v < tol_v


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

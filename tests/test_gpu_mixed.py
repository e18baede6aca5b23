"""Mixed-precision form against the FP64 oracle: FP32 preconditioner solves
(FP32 n x t blocks, FP64 row sums) inside the FP64 block PCG, whose FP64
operator and residual recurrence refine every FP32 solve: level-scheduled
with FP32 B values for blocks wider than 64 columns, the dense leading block
and sync-free tail with FP32 right-hand sides and results for narrower ones.
Probe counts below and above 64 run both.  The bar: relative 1e-4 on the
negative log-likelihood and 1e-3 on the predictive variances; the errors of
the mode, the predictive means and the gradient are measured and printed."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from tests.gpu_common import dev, host, opts_pair, rel_err, say  # noqa: E402

NLL_TOL = 1e-4
VAR_TOL = 1e-3


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


CASES = {
    # n = 2,000 exponential range 0.1, m = 10, Bernoulli-logit
    "c1": dict(name="c1_n2000", over=dict(), t_wide=72, s=256, tol=1e-8, ptol=1e-6),
    # n = 20,000 Matern-3/2 range 0.05, m = 20, Poisson with offset 1
    "mid": dict(name="c2_n1e5", over=dict(n=20000, n_pred=2000, lik=OL.LIK_POISSON, F=1.0),
                t_wide=80, s=96, tol=1e-3, ptol=1e-3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_mixed_against_fp64_oracle(P, case):
    spec = CASES[case]
    w = synth.make(spec["name"], seed=3, **spec["over"])
    tw = spec["t_wide"]
    say(f"case: mixed precision {case} n={w['n']} m={w['m']} t={w['t']} and {tw} s={spec['s']}")
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]), deriv=True)
    o, go = opts_pair(P, cg_tol=spec["tol"], pred_cg_tol=spec["ptol"], num_probes=w["t"],
                      num_pred_samples=spec["s"], seed=11)
    ow, gw = opts_pair(P, cg_tol=spec["tol"], num_probes=tw, seed=11)
    go.precision = P.VL_MIXED
    gw.precision = P.VL_MIXED
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]),
                         want_deriv=True)
    mode, _ = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    # t <= 64 with the gradient (narrow FP32 solves), then more than 64 probes
    # (level-scheduled FP32 solves)
    nll, grad, _ = g.neg_log_marglik(go, want_grad=True)
    nll_w, _, _ = g.neg_log_marglik(gw)
    mean, var, _ = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), go)
    g.close()
    b, W, _ = OL.find_mode(model, w["y"], w["F"], w["lik"], None, o)
    nll_o, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o, want_grad=True)
    nll_ow, _ = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, ow)
    mean_o, var_o, _ = OL.predict(model, w["coords_pred"], w["Fp"], b, W, o)
    e_nll = abs(nll - nll_o) / abs(nll_o)
    e_nll_w = abs(nll_w - nll_ow) / abs(nll_ow)
    e_var = rel_err(host(var), var_o)
    e_mode = rel_err(host(mode), b)
    e_mean = rel_err(host(mean), mean_o)
    e_grad = rel_err(np.array(grad), np.array(info["grad"]))
    say(f"mixed {case}: rel err nll(t={w['t']})={e_nll:.2e} nll(t={tw})={e_nll_w:.2e} "
        f"var={e_var:.2e} mode={e_mode:.2e} mean={e_mean:.2e} grad={e_grad:.2e}")
    assert e_nll < NLL_TOL and e_nll_w < NLL_TOL
    assert e_var < VAR_TOL
    assert e_mode < 1e-6 and e_mean < 1e-6  # the Newton update stays FP64

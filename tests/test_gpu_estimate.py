"""Estimation of theta by L-BFGS with a sample average approximation
(vl_estimate, Sec. 4.1) against the oracle's estimate (scipy L-BFGS-B on the
oracle's likelihood and STE gradient with the same probes): both locate the
zero of the same deterministic gradient."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from tests.gpu_common import dev, say  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


def test_estimate_matches_the_oracle(P):
    w = synth.make(None, seed=31, n=1000, m=10, kind=synth.COV_EXPONENTIAL, sigma2=1.0,
                   rho=0.1, lik=synth.LIK_BERNOULLI_LOGIT, F=0.0, n_pred=0)
    theta0 = (0.5, 0.05)
    o = OL.Opts(cg_tol=1e-9, newton_tol=1e-12, num_probes=16, seed=6)
    go = P.vl_default_opts(cg_tol=o.cg_tol, newton_tol=o.newton_tol, num_probes=16, seed=6)
    say("case: theta estimate n=1000, 16 probes")
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], theta0, want_deriv=True)
    th, nll, it, ev = g.estimate(dev(w["y"]), dev(w["F"]), w["lik"], theta0, opts=go,
                                 max_iter=60, grad_tol=1e-6)
    g.close()
    th_o, nll_o, res = OL.estimate(w["coords"], w["m"], w["kind"], w["y"], w["F"], w["lik"],
                                   None, theta0, o, gtol=1e-7)
    e = np.max(np.abs(np.log(th) - np.log(th_o)))
    say(f"device theta {th} nll {nll:.10f} ({it} iterations, {ev} evaluations); oracle "
        f"{tuple(th_o)} nll {nll_o:.10f} ({res.nit} iterations); log-theta difference {e:.2e}")
    assert e < 1e-3
    assert abs(nll - nll_o) < 1e-7 * abs(nll_o)

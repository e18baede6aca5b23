"""GPU parity of the preconditioned Lanczos predictive variances (Sec. 3.3.2,
P_L1 and P_L2 with complete reorthogonalization) against the FP64 oracle on
the same seeded inputs: the Lanczos coefficients, the predictive means and
the variances element by element.  Ranks below and above one wave of columns
(the narrow and the wide triangular-solve paths for the rank-k block), a
ragged n = 6,001, and the full-rank limit where the approximation is exact
(compared with a dense computation)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from tests import dense_ref as DR  # noqa: E402
from tests.gpu_common import dev, host, oracle_mode_matching, opts_pair, rel_err, rel_err_elem, say  # noqa: E402,E501

TOL = 1e-9


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


def _run(P, w, method, k, n_pred=None):
    o, go = opts_pair(P, cg_tol=1e-10, newton_tol=1e-10, seed=1)
    go.pred_method = method
    go.lanczos_rank = k
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
    mode, _ = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    newton_cg = host(g.export("newton_cg_iters")).tolist()
    halvings = host(g.export("newton_halvings")).tolist()
    cp = w["coords_pred"] if n_pred is None else w["coords_pred"][:n_pred]
    Fp = w["Fp"] if n_pred is None else w["Fp"][:n_pred]
    mean, var, _ = g.predict(dev(cp), dev(Fp), go)
    out = dict(mode=host(mode), mean=host(mean), var=host(var),
               alpha=host(g.export("lanczos_alpha")), beta=host(g.export("lanczos_beta")))
    g.close()
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]))
    b, W, _, _ = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, o, newton_cg,
                                      gpu_halvings=halvings)
    return out, model, b, W, cp, Fp


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("case,k", [("c1", 30), ("c1", 120), ("n6001", 50)])
def test_lanczos_variances(P, method, case, k):
    if case == "c1":
        # n = 2,000 exponential range 0.1, m = 10, Bernoulli-logit, 500 test points
        w = synth.make("c1_n2000", seed=0)
    else:
        # n = 6,001 Matern-3/2 range 0.05, m = 10, Poisson with offset 1, 777 test points
        w = synth.make(None, seed=6, n=6001, m=10, kind=synth.COV_MATERN32, sigma2=1.0,
                       rho=0.05, lik=synth.LIK_POISSON, F=1.0, n_pred=777)
    say(f"case: lanczos P_L{method} {case} n={w['n']} k={k}")
    f, model, b, W, cp, Fp = _run(P, w, method, k)
    mean, var, info = OL.predict_lanczos(model, cp, Fp, b, W, k, method)
    T = info["T"]
    a_o, b_o = np.diag(T), np.diag(T, 1)
    say(f"rank {len(f['alpha'])} (oracle {info['rank']}); alpha rel "
        f"{rel_err_elem(f['alpha'], a_o):.2e} beta rel {rel_err_elem(f['beta'], b_o):.2e} "
        f"var rel {rel_err_elem(f['var'], var):.2e}")
    assert len(f["alpha"]) == info["rank"]
    assert rel_err_elem(f["alpha"], a_o) < TOL
    assert rel_err_elem(f["beta"], b_o) < TOL
    assert rel_err(f["mean"], mean) < TOL
    assert rel_err_elem(f["var"], var) < TOL


@pytest.mark.parametrize("method", [1, 2])
def test_lanczos_full_rank_is_exact(P, method):
    """k = n: the approximation equals the dense predictive variance D_p +
    diag(A_p A^{-1} A_p^T) (eq. latentpostpredictive)."""
    w = synth.make(None, seed=8, n=300, m=8, kind=synth.COV_EXPONENTIAL, sigma2=1.0, rho=0.2,
                   lik=synth.LIK_BERNOULLI_LOGIT, F=0.0, n_pred=40)
    say(f"case: lanczos P_L{method} full rank n=300")
    f, model, b, W, cp, Fp = _run(P, w, method, w["n"])
    _, _, info = OL.predict(model, cp, Fp, b, W, OL.Opts(), want_var=False)
    Ap = np.zeros((len(cp), w["n"]))
    for p in range(len(cp)):
        Ap[p, info["nbr_p"][p]] = info["Ap"][p]
    A = np.diag(W) + DR.dense_precision(model.B, model.D)
    exact = info["Dp"] + np.einsum("pi,pi->p", Ap, np.linalg.solve(A, Ap.T).T)
    e = rel_err_elem(f["var"], exact)
    say(f"full-rank variance vs dense: rel {e:.2e}")
    assert e < 1e-8


def test_lanczos_argument_checks(P):
    w = synth.make("c1_n2000", seed=0)
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
    go = P.vl_default_opts(cg_tol=1e-6)
    g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    cp = dev(w["coords_pred"][:10])
    for method, k in ((1, 0), (2, w["n"] + 1), (7, 10)):
        bad = P.vl_default_opts(pred_method=method, lanczos_rank=k)
        with pytest.raises(P.VLError) as e:
            g.predict(cp, None, bad)
        assert e.value.code == P.VL_ERR_INVALID_ARG
    g.close()

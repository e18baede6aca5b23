"""GPU parity of the LRAC preconditioner (Sec. 3.1.2): pivoted Cholesky
factor, the Woodbury matrix I + L^T W L (FP64 matrix-core panels), Newton
mode finding with eq. (pcls2) and the SLQ likelihood with eq. (logdetsplit2),
against the FP64 oracle on the same seeded inputs and probes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from tests.gpu_common import dev, host, oracle_mode_matching, opts_pair, rel_err, say  # noqa: E402

TOL = 1e-9
K_RANK = 50


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def fit(P):
    # n = 2,000 exponential range 0.1, m = 10, Bernoulli-logit; rank 50
    w = synth.make("c1_n2000", seed=0)
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]))
    say("case: LRAC c1 n=2000 m=10 k=50")
    o, go = opts_pair(P, cg_tol=w["cg_tol"], num_probes=w["t"], seed=5,
                      precond=OL.PRECOND_LRAC, lrac_rank=K_RANK)
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
    mode, st = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, go)
    out = dict(mode=host(mode), newton_cg=host(g.export("newton_cg_iters")).tolist(),
               halvings=host(g.export("newton_halvings")).tolist(),
               L=host(g.export("lrac_L")).reshape(w["n"], K_RANK),
               piv=host(g.export("lrac_piv")).astype(np.int64))
    nll, _, nst = g.neg_log_marglik(go)
    out.update(nll=nll, slq_iters=host(g.export("block_iters")).tolist(),
               quad=host(g.export("slq_quad")), r0z0=host(g.export("slq_r0z0")),
               W=host(g.export("W")), chol=host(g.export("lrac_chol")))
    g.close()
    return w, model, o, out


def test_pivoted_cholesky(fit):
    w, model, o, f = fit
    Lo = OL.pivoted_cholesky(w["coords"], w["kind"], (w["sigma2"], w["rho"]), K_RANK)
    # the pivot of column j is the row where it takes the value sqrt(d_p),
    # its largest entry; compare the sequences, else replay the device's
    piv_o = [int(np.argmax(np.abs(Lo[:, j]))) for j in range(K_RANK)]
    if piv_o != f["piv"].tolist():
        say("pivot sequences differ; replaying the device's pivots")
        Lo = OL.pivoted_cholesky(w["coords"], w["kind"], (w["sigma2"], w["rho"]), K_RANK,
                                 pivots=f["piv"])
    assert rel_err(f["L"], Lo) < TOL


def test_woodbury_matrix_on_matrix_cores(fit):
    # Cholesky factor of I + L^T W L from the FP64 matrix-core panels, against
    # numpy on the exported L and W (K = k rounded up to 16, identity padding)
    w, model, o, f = fit
    K = (K_RANK + 15) // 16 * 16
    Mx = np.eye(K)
    Mx[:K_RANK, :K_RANK] += f["L"].T @ (f["W"][:, None] * f["L"])
    C = np.linalg.cholesky(Mx)
    assert rel_err(f["chol"].reshape(K, K), C) < 1e-11


def test_lrac_mode(fit):
    w, model, o, f = fit
    Lo = OL.pivoted_cholesky(w["coords"], w["kind"], (w["sigma2"], w["rho"]), K_RANK,
                             pivots=f["piv"])
    b, W, st, replayed = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, o,
                                              f["newton_cg"], L=Lo,
                                              gpu_halvings=f["halvings"])
    say(f"newton cg gpu={f['newton_cg']} oracle={st['cg_iters']} replayed={replayed}")
    assert rel_err(f["mode"], b) < TOL


def test_lrac_nll(fit):
    w, model, o, f = fit
    Lo = OL.pivoted_cholesky(w["coords"], w["kind"], (w["sigma2"], w["rho"]), K_RANK,
                             pivots=f["piv"])
    b, W, _, _ = oracle_mode_matching(model, w["y"], w["F"], w["lik"], None, o, f["newton_cg"],
                                      L=Lo)
    nll, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o, L=Lo)
    if list(info["cg_iters"]) != f["slq_iters"]:
        say("SLQ iteration counts differ; replaying the device's counts")
        nll, info = OL.neg_log_marglik(model, w["y"], w["F"], w["lik"], None, b, o, L=Lo,
                                       replay_cg=f["slq_iters"])
    assert rel_err(f["r0z0"], info["r0z0"]) < TOL
    assert rel_err(f["quad"], info["quad"]) < TOL
    assert abs(f["nll"] - nll) <= TOL * abs(nll)


def _lrac_grad_case(P, w, lik, aux, k, t, X=None):
    """Device NLL with gradients under P_LRAC and the oracle's at the same
    mode, probes, pivots and iteration counts."""
    o, go = opts_pair(P, cg_tol=1e-10, newton_tol=1e-12, num_probes=t, seed=5,
                      precond=OL.PRECOND_LRAC, lrac_rank=k)
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]),
                         want_deriv=True)
    g.find_mode(dev(w["y"]), dev(w["F"]), lik, aux, go)
    newton_cg = host(g.export("newton_cg_iters")).tolist()
    halvings = host(g.export("newton_halvings")).tolist()
    piv = host(g.export("lrac_piv")).astype(np.int64)
    nll, grad, _ = g.neg_log_marglik(go, want_grad=True)
    slq = host(g.export("block_iters")).tolist()
    gF = host(g.grad_offset())
    gx = g.grad_aux() if aux is not None else None
    gb = g.grad_beta(dev(X)) if X is not None else None
    g.close()
    model = OL.Model(w["coords"], w["m"], w["kind"], (w["sigma2"], w["rho"]), deriv=True)
    Lo = OL.pivoted_cholesky(w["coords"], w["kind"], (w["sigma2"], w["rho"]), k, pivots=piv)
    b, _, _, _ = oracle_mode_matching(model, w["y"], w["F"], lik, aux, o, newton_cg, L=Lo,
                                      gpu_halvings=halvings)
    nll_o, info = OL.neg_log_marglik(model, w["y"], w["F"], lik, aux, b, o, L=Lo, want_grad=True,
                                     replay_cg=slq)
    return dict(nll=nll, grad=grad, gF=gF, gx=gx, gb=gb), nll_o, info


def test_lrac_gradients_bernoulli(P):
    """theta- and offset gradients with the LRAC STE formulas (App. A.4.2; the
    pivoted Cholesky factor's derivative at fixed pivots) at n = 2,000."""
    w = synth.make("c1_n2000", seed=0)
    say("case: LRAC gradients c1 n=2000 k=50 t=50")
    f, nll_o, info = _lrac_grad_case(P, w, w["lik"], None, K_RANK, 50)
    say(f"theta gradient device {f['grad']} oracle {info['grad']}; offset rel "
        f"{rel_err(f['gF'], info['grad_F']):.2e}")
    assert abs(f["nll"] - nll_o) <= TOL * abs(nll_o)
    np.testing.assert_allclose(f["grad"], info["grad"], rtol=TOL)
    assert rel_err(f["gF"], info["grad_F"]) < TOL


def test_lrac_gradients_gamma(P):
    """Gamma shape (xi) gradient with P_LRAC, a ragged n = 1,501 and k = 20."""
    n = 1501
    coords = synth.locations(n, seed=81)
    b = synth.latent_field(coords, synth.COV_MATERN32, 1.0, 0.1, seed=81)
    F = np.full(n, 0.2)
    y = synth.responses(synth.LIK_GAMMA, F + b, seed=81, shape=2.5)
    w = dict(coords=coords, y=y, F=F, m=10, kind=synth.COV_MATERN32, sigma2=1.0, rho=0.1)
    say("case: LRAC gradients gamma n=1501 k=20 t=32")
    f, nll_o, info = _lrac_grad_case(P, w, P.VL_LIK_GAMMA, 2.5, 20, 32)
    bar = TOL * (abs(info["dlogp_xi"]) + 0.5 * abs(info["dlogdet_xi"]) + abs(info["implicit_xi"]))
    say(f"shape gradient device {f['gx']!r} oracle {info['grad_xi']!r} bar {bar:.2e}")
    assert abs(f["nll"] - nll_o) <= TOL * abs(nll_o)
    np.testing.assert_allclose(f["grad"], info["grad"], rtol=TOL)
    assert rel_err(f["gF"], info["grad_F"]) < TOL
    assert abs(f["gx"] - info["grad_xi"]) <= bar

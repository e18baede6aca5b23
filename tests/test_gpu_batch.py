"""Batching form: uneven problems packed into one block-diagonal system and
fitted together (vl_batch_*), against solo runs of each problem through the
C ABI and, for every problem, against the FP64 oracle at relative 1e-9.

The batch runs at CG tolerance 1e-10: the batch reports no per-solve CG
counts for the oracle to replay, and at this tolerance every solve is
converged far enough that a stopping decision one iteration apart changes
no result at the 1e-9 level."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import laplace as OL  # noqa: E402
from tests.gpu_common import dev, host, opts_pair, rel_err, say  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def batch(P):
    # 10 problems, n log-uniform in [800, 3000], m in {10, 20, 30},
    # exponential or Matern-3/2, range U(0.02, 0.2), Bernoulli-logit
    probs = synth.batch_problems(count=10, seed=2, n_lo=800, n_hi=3000)
    say("case: batch of 10 problems, n = " + ", ".join(str(p["n"]) for p in probs))
    o, go = opts_pair(P, cg_tol=1e-10, num_probes=8)
    items = [dict(coords=p["coords"], y=p["y"], F=p["F"], m=p["m"], cov=p["kind"],
                  theta=(p["sigma2"], p["rho"]), seed=1000 + k) for k, p in enumerate(probs)]
    b = P.VecchiaLaplaceBatch(items)
    nll = b.fit(go)
    modes = [host(b.mode(k)) for k in range(len(probs))]
    stats = [b.stats(k).as_dict() for k in range(len(probs))]
    paths = [b.tuned_path(c) for c in range(2)]
    b.close()
    return probs, o, go, nll, modes, stats, paths


def test_batch_equals_solo_runs(P, batch):
    probs, o, go, nll, modes, stats, paths = batch
    say(f"autotuned solve paths (t=1, t=8): {paths}")
    assert all(pt in (0, 1, 2) for pt in paths)
    for k, p in enumerate(probs):
        g = P.VecchiaLaplace(dev(p["coords"]), p["m"], p["kind"], (p["sigma2"], p["rho"]))
        go.seed = 1000 + k
        mode, st = g.find_mode(dev(p["y"]), dev(p["F"]), p["lik"], None, go)
        nll1, _, nst = g.neg_log_marglik(go)
        g.close()
        say(f"problem {k}: n={p['n']} m={p['m']} nll batch={nll[k]:.12g} solo={nll1:.12g} "
            f"newton {stats[k]['newton_iters']}/{st.newton_iters}")
        assert stats[k]["newton_iters"] == st.newton_iters
        assert rel_err(modes[k], host(mode)) < 1e-9
        assert abs(nll[k] - nll1) <= 1e-9 * abs(nll1)


def test_batch_against_oracle(P, batch):
    probs, o, go, nll, modes, stats, paths = batch
    for k, p in enumerate(probs):
        model = OL.Model(p["coords"], p["m"], p["kind"], (p["sigma2"], p["rho"]))
        o.seed = 1000 + k
        b, W, ost = OL.find_mode(model, p["y"], p["F"], p["lik"], None, o)
        nll_o, _ = OL.neg_log_marglik(model, p["y"], p["F"], p["lik"], None, b, o)
        e_b = rel_err(modes[k], b)
        e_n = abs(nll[k] - nll_o) / abs(nll_o)
        say(f"problem {k}: n={p['n']} oracle nll={nll_o:.12g} newton {ost['newton_iters']}/"
            f"{stats[k]['newton_iters']} mode rel {e_b:.2e} nll rel {e_n:.2e}")
        assert e_b < 1e-9
        assert e_n < 1e-9

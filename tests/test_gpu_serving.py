"""Serving form: the continuous-batching request loop (vl_server_*).  The same
requests run once alone (one slot, one after another) and once in a mix
(four slots, submitted together, overlapping on the device); every result
must be identical, bit for bit, and the mix must actually overlap."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from tests.gpu_common import host, say  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


def _requests():
    # Poisson arrivals of fit + predict requests, n log-uniform in [2e3, 2e4],
    # 200..600 test points, m = 20, Bernoulli or Poisson with probability 1/2
    reqs = synth.serving_requests(6, seed=4, n_lo=2000, n_hi=20000, np_lo=200, np_hi=600)
    return [dict(coords=r["coords"], y=r["y"], F=r["F"], m=r["m"], cov=r["kind"],
                 theta=(r["sigma2"], r["rho"]), lik=r["lik"], seed=77 + k,
                 coords_p=r["coords_pred"], Fp=r["Fp"]) for k, r in enumerate(reqs)]


def _run(P, slots, reqs):
    o = P.vl_default_opts(num_probes=16, num_pred_samples=64, cg_tol=1e-3, pred_cg_tol=1e-3)
    s = P.Server(slots, 200e9, o)
    tickets = [s.submit(r) for r in reqs]
    out = []
    for tk in tickets:
        nll, mean, var, st, qms = s.wait(tk)
        out.append((nll, host(mean), host(var), st, qms))
    info = s.info()
    s.close()
    return out, info


def test_results_equal_alone_and_in_the_mix(P):
    reqs = _requests()
    say("case: serving 6 requests, n = " + ", ".join(str(r["coords"].shape[0]) for r in reqs))
    alone, info1 = _run(P, 1, reqs)
    mix, info4 = _run(P, 4, reqs)
    say(f"peak running alone={info1[1]} mix={info4[1]}; peak HBM estimate {info4[0] / 1e9:.2f} GB")
    assert info1[1] == 1 and info4[1] > 1
    for k, (a, b) in enumerate(zip(alone, mix)):
        say(f"request {k}: nll {a[0]:.12g} / {b[0]:.12g}, latency {a[3]['t_ms']:.0f} / "
            f"{b[3]['t_ms']:.0f} ms")
        assert a[0] == b[0]
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert np.all(np.isfinite(a[2])) and np.all(a[2] > 0)


def test_admission_respects_the_budget(P):
    # a budget that fits one request at a time serialises them
    reqs = _requests()[:3]
    o = P.vl_default_opts(num_probes=16, num_pred_samples=64)
    s = P.Server(4, 1.0, o)  # smaller than any request: each runs alone
    tickets = [s.submit(r) for r in reqs]
    for tk in tickets:
        s.wait(tk)
    peak_bytes, peak_running = s.info()
    s.close()
    assert peak_running == 1

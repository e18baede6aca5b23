"""The C ABI's allocator hook (vl_set_allocator): with PyTorch's caching
allocator installed, every device buffer a model owns comes from it and goes
back to it at vl_free, and results equal those of the library's default
allocator bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from tests.gpu_common import dev, host, say  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_12000_amd as P
    P.lib()
    return P


class Counting:
    def __init__(self):
        self.live = {}
        self.allocs = 0

    def alloc(self, nbytes, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, stream=stream)
        self.live[p] = nbytes
        self.allocs += 1
        return p

    def release(self, ptr, stream):
        assert ptr in self.live, "freed a pointer the hook never returned"
        del self.live[ptr]
        torch.cuda.caching_allocator_delete(ptr)


def _fit(P, w, opts):
    g = P.VecchiaLaplace(dev(w["coords"]), w["m"], w["kind"], (w["sigma2"], w["rho"]))
    mode, _ = g.find_mode(dev(w["y"]), dev(w["F"]), w["lik"], None, opts)
    nll, _, _ = g.neg_log_marglik(opts)
    mean, var, _ = g.predict(dev(w["coords_pred"]), dev(w["Fp"]), opts)
    return g, host(mode), nll, host(mean), host(var)


def test_model_memory_comes_from_the_installed_allocator(P):
    say("case: allocator hook, n=6000 fit + predict")
    w = synth.make(None, seed=11, n=6000, m=10, kind=synth.COV_MATERN32, sigma2=1.0, rho=0.1,
                   lik=synth.LIK_BERNOULLI_LOGIT, F=0.0, n_pred=300)
    opts = P.vl_default_opts(cg_tol=1e-8, pred_cg_tol=1e-8, num_probes=16,
                             num_pred_samples=32, seed=3)
    g0, mode0, nll0, mean0, var0 = _fit(P, w, opts)
    g0.close()
    del g0
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    cnt = Counting()
    P.vl_set_allocator(cnt.alloc, cnt.release)
    try:
        g, mode, nll, mean, var = _fit(P, w, opts)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - base
        owned = sum(cnt.live.values())
        assert cnt.allocs > 0 and owned > 0
        # the handle's state (factor, schedules, dense inverse, CG blocks)
        # is torch memory: at least the dense inverse of the leading block
        assert held >= owned >= 2 * 4096 * 4096 * 8
        g.close()
        del g  # drops the wrapper's reference to the coordinate tensor
        torch.cuda.synchronize()
        assert not cnt.live, f"{len(cnt.live)} buffers not returned"
        assert torch.cuda.memory_allocated() == base
    finally:
        P.vl_set_allocator(None, None)
    assert nll == nll0
    assert np.array_equal(mode, mode0)
    assert np.array_equal(mean, mean0) and np.array_equal(var, var0)

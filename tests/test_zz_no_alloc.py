"""The allocation-free triangular solve (vl_trsm_noalloc) against vl_trsm,
through the C ABI: the same kernels on the same inputs, so the results must
be identical, and the allocation-free call must not reach the installed
device allocator at all.  Two calls in a row, the second with a smaller
input (fewer columns, then a smaller model), so the second runs on the
fixed per-GPU scratch the first left behind."""
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
    """Device allocator hook backed by PyTorch's caching allocator that
    counts the calls the library makes."""

    def __init__(self):
        self.allocs = 0
        self.frees = 0

    def alloc(self, nbytes, stream):
        self.allocs += 1
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def release(self, ptr, stream):
        self.frees += 1
        torch.cuda.caching_allocator_delete(ptr)


def _solve_both(P, g, X, transpose):
    Xd = dev(X)
    ref = torch.full_like(Xd, np.nan)
    out = torch.full_like(Xd, np.nan)
    P.vl_trsm(g.h, Xd, ref, transpose=transpose)
    torch.cuda.synchronize()
    cnt = Counting()
    P.vl_set_allocator(cnt.alloc, cnt.release)
    try:
        P.vl_trsm_noalloc(g.h, Xd, out, transpose=transpose)
        torch.cuda.synchronize()
    finally:
        P.vl_set_allocator(None, None)
    assert cnt.allocs == 0 and cnt.frees == 0, (cnt.allocs, cnt.frees)
    return host(out), host(ref)


@pytest.mark.parametrize("n,m", [(20000, 20), (3001, 10)])
def test_noalloc_solve_equals_vl_trsm(P, n, m):
    X = synth.locations(n, seed=n)
    g = P.VecchiaLaplace(dev(X), m, 1, (1.0, 0.05))
    rng = np.random.default_rng(n)
    for t in (50, 3):  # the second call smaller than the first
        for tr in (False, True):
            say(f"case: noalloc trsm n={n} m={m} t={t} transpose={tr}")
            out, ref = _solve_both(P, g, rng.standard_normal((n, t)), tr)
            assert np.all(np.isfinite(out))
            assert np.array_equal(out, ref)
    g.close()


def test_noalloc_rejects_wide_blocks(P):
    X = synth.locations(500, seed=3)
    g = P.VecchiaLaplace(dev(X), 8, 0, (1.0, 0.1))
    Xd = dev(np.ones((500, 65)))
    with pytest.raises(P.VLError) as e:
        P.vl_trsm_noalloc(g.h, Xd, torch.empty_like(Xd))
    assert e.value.code == P.VL_ERR_INVALID_ARG
    g.close()

"""The allocation-free entry point llr_beta_c_noalloc against llr_beta_c
through the C ABI: the same kernels on the same inputs, so the results are
identical, over two calls in a row (the second with fewer intervals and a
coarser grid, reusing the fixed buffer the first one filled); sizes beyond
its fixed 1 MiB buffer are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def llr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1509_08391_amd import llr as m
    m.lib()
    return m


def _case(n, seed):
    rng = np.random.default_rng(seed)
    V6 = 6 * 20 ** 4
    dE = 0.0005 * V6
    c = 0.6 * V6 + dE * (np.arange(n) + 0.5)
    a = 1.011 + 0.002 * np.sin(np.linspace(0, 3, n)) + 1e-4 * rng.normal(size=n)
    return c, a, dE, V6


def test_noalloc_matches_allocating_entry_point(llr):
    ctx = llr.Context(precision=llr.FP32)
    for n, (blo, bhi, h) in [(128, (1.008, 1.012, 1e-5)), (40, (1.009, 1.011, 4e-5))]:
        c, a, dE, V6 = _case(n, 7 + n)
        ref = ctx.beta_c(c, a, dE, V6, blo, bhi, h=h, tol=1e-9)
        got = ctx.beta_c_noalloc(c, a, dE, V6, blo, bhi, h=h, tol=1e-9)
        assert got == ref, (n, got, ref)
        assert blo <= got[0] <= bhi and got[1] > 0
    # 8 (3 n + ng + 8) bytes must fit 1 MiB
    c, a, dE, V6 = _case(128, 1)
    with pytest.raises(llr.LLRError):
        ctx.beta_c_noalloc(c, a, dE, V6, 1.0, 1.2, h=1e-6, tol=1e-9)
    ctx.close()

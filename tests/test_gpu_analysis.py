"""GPU parity of the analysis of repeated runs (through the C ABI) against the
oracle: ln P_beta(E) within 1e-8 absolute (both subtract a ln Z of size
~beta E ~ 1e6, so the difference of two FP64 evaluations is ~1e-10), the same
peak edges, bootstrap samples within the reconstruction's 1e-8 on beta_c,
finite-size fits within 1e-9 relative."""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_fss_tables.txt")


@pytest.fixture(scope="module")
def llr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1509_08391_amd import llr as m
    m.lib()
    return m


def _two_phase(n=128, s=480.0, u0=0.60, six_v=960000.0):
    """a_k of the shape the L=20 runs give: rising, dipping through the
    coexistence region, rising again."""
    k = np.arange(n)
    c = u0 * six_v + s * (k + 0.5)
    a = 1.0055 + 0.0001 * k - 0.0035 * np.exp(-((k - 90) / 14.0) ** 2) + 2e-5 * np.sin(k)
    return c, a, s, six_v


def test_prob_density_and_peaks(llr):
    c, a, s, six_v = _two_phase()
    ctx = llr.Context(precision=llr.FP64)
    E = np.concatenate([np.linspace(c[0] - 0.5 * s - 10, c[-1] + 0.5 * s + 10, 5001), c, c + 0.5 * s])
    for beta in (1.0105, 1.0110, 1.0115):
        g = ctx.prob_density(c, a, s, beta, E)
        o = oracle.prob_density(c, a, s, beta, E)
        inside = np.isfinite(o)
        assert np.array_equal(np.isfinite(g), inside)
        assert np.max(np.abs(g[inside] - o[inside])) < 1e-8
        Eg, lg = ctx.prob_peaks(c, a, s, beta)
        Eo, lo = oracle.prob_peaks(c, a, s, beta)
        assert np.array_equal(Eg, Eo)
        assert np.max(np.abs(lg - lo)) < 1e-8
    ctx.close()


def test_bootstrap_matches_oracle(llr):
    c, a, s, six_v = _two_phase()
    rng = np.random.default_rng(4)
    runs = a[None, :] + rng.normal(0, 3e-4, (8, a.size))
    ctx = llr.Context(precision=llr.FP32)
    bg, pg = ctx.bootstrap(c, runs, s, six_v, 1.008, 1.012, n_boot=40, seed=77)
    ctx.close()
    bo, po = oracle.bootstrap(c, runs, s, six_v, 1.008, 1.012, n_boot=40, seed=77)
    assert np.max(np.abs(bg - bo)) < 1e-8
    assert np.max(np.abs(pg / po - 1)) < 1e-9
    assert bg.std() > 0


def test_fss_fit_matches_oracle(llr):
    t, cur = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            t[cur] = []
            continue
        t[cur].append([float(v) for v in line.split()])
    for key in ("peakloc", "peak"):
        d = np.array(t[key])
        for Lmin in (8, 10, 12, 14):
            for kmax in (1, 2, 3):
                m = d[:, 0] >= Lmin
                if m.sum() <= kmax + 1:
                    continue
                pw = np.array([0.0] + [-4.0 * k for k in range(1, kmax + 1)])
                pg, eg, cg = llr.fss_fit(d[m, 0], d[m, 1], d[m, 2], pw)
                po, eo, co = oracle.fss_fit(d[m, 0], d[m, 1], d[m, 2], pw)
                assert np.max(np.abs(pg - po) / np.maximum(np.abs(po), 1e-300)) < 1e-9
                assert np.max(np.abs(eg / eo - 1)) < 1e-9
                assert abs(cg - co) <= 1e-9 * max(1.0, co)


def test_analysis_rejects_bad_arguments(llr):
    c, a, s, six_v = _two_phase(n=16)
    ctx = llr.Context(precision=llr.FP64)
    with pytest.raises(llr.LLRError):
        ctx.prob_density(c * 1.001, a, s, 1.0, [c[3]])           # centres not spaced by s
    with pytest.raises(llr.LLRError):
        ctx.bootstrap(c, np.tile(a, (1100, 1)), s, six_v, 1.0, 1.02, 4, 1)  # more than 1024 runs
    with pytest.raises(llr.LLRError):
        llr.fss_fit([8.0, 10.0], [1.0, 1.0], [1.0, 1.0], [0.0, -4.0])     # m must exceed n_par
    ctx.close()

"""Host-side helpers of the measurement runs (CPU): the integrated
autocorrelation time used to compare the class-wise and per-link restriction
against the closed form of an AR(1) process, tau = (1 + rho) / (2 (1 - rho)),
and for independent samples 1/2."""
import numpy as np
import pytest

from paper_1509_08391_amd.experiments import _tau_int


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_tau_int_of_ar1(rho):
    rng = np.random.default_rng(3)
    n, m = 100000, 4
    e = rng.normal(size=(n, m))
    x = np.empty_like(e)
    x[0] = e[0] / np.sqrt(1 - rho ** 2)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    exact = (1 + rho) / (2 * (1 - rho))
    tau = _tau_int(x)
    # the automatic window truncates the tail (bias ~ e^{-W/tau}) and the
    # estimate has relative spread ~ sqrt(2 (2 W + 1) / n)
    assert np.all(np.abs(tau - exact) < 0.06 * exact + 0.02), (tau, exact)


def test_experiments_command_line_offers_every_sweep_order_and_study():
    """The experiments' command line (no device used): every sweep order of
    the library and both delta E studies are selectable."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-m", "paper_1509_08391_amd.experiments", "--help"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    for word in ("grouped", "interleaved", "staggered", "dE8", "dE12"):
        assert word in r.stdout, word

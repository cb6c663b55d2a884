"""Oracle pins for the Robbins-Monro update (eq. (kk21), Algorithm 1) driven by
mock samplers whose restricted density is known exactly (Sec. 2.2):
  * rho(E) = exp(-a* E): the root of <<Delta E>>(a) = 0 is a* for any width,
    <<Delta E>>(a) = (w/2) Lang((a - a*) w/2) with Lang(y) = coth y - 1/y
    (closed form of F(Delta a)), and sqrt(n)(a_n - a*) has the asymptotic
    variance c^2 sigma_xi^2 / (2 c M' - 1) of eq. (var) with c M' = 1;
  * Gaussian rho (appendix, eq. (kkk32)): the root is found by quadrature."""
import numpy as np
from scipy import integrate, optimize

import oracle


def _sample_trunc_exp(rng, lam, lo, hi, size):
    """E on [lo, hi] with density ~ exp(lam E), exact inverse CDF."""
    u = rng.random(size)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), u.shape)
    w = hi - lo
    small = np.abs(lam) < 1e-12
    safe = np.where(small, 1.0, lam)
    return np.where(small, lo + w * u, lo + np.log1p(u * np.expm1(safe * w)) / safe)


def test_rm_step_sign_and_gain():
    # mean above the centre lowers a; step is 12 (mean - c) / ((n+1) w^2)
    assert oracle.rm_step(1.0, 10.5, 10.0, 0, 2.0) == 1.0 - 12 * 0.5 / 4.0
    assert oracle.rm_step(1.0, 9.5, 10.0, 4, 2.0) == 1.0 + 12 * 0.5 / (5 * 4.0)


def test_rm_converges_to_exact_root_with_predicted_variance():
    rng = np.random.default_rng(7)
    a_star, w, c, n_a = 0.83, 3.0, 50.0, 40
    lo, hi = c - w / 2, c + w / 2
    reps, n_it = 4000, 400
    a = np.full(reps, 1.6)
    for n in range(n_it):
        E = _sample_trunc_exp(rng, (a - a_star)[:, None], lo, hi, (reps, n_a))
        mean = E.mean(axis=1)
        a = np.array([oracle.rm_step(a[i], mean[i], c, n, w) for i in range(reps)])
    # closed-form check of the mock density's mean offset at one a
    y = 0.7 * w / 2
    Eprobe = _sample_trunc_exp(rng, 0.7, lo, hi, 400000)
    assert abs((Eprobe.mean() - c) - (w / 2) * (1 / np.tanh(y) - 1 / y)) < 5 * Eprobe.std() / 600
    # asymptotic variance: c = 12/w^2, M' = w^2/12, sigma_xi^2 = w^2/(12 n_a)
    pred_var = 12.0 / (w * w * n_a * n_it)
    assert abs(a.mean() - a_star) < 4 * np.sqrt(pred_var / reps)
    assert abs(a.var() / pred_var - 1.0) < 0.1


def test_rm_root_with_gaussian_density_by_quadrature():
    rng = np.random.default_rng(3)
    mu, sig = 0.0, 4.0            # ln rho = -(E - mu)^2 / (2 sig^2)
    lo, hi = 6.0, 10.0
    c, w = 8.0, 4.0

    def mean_offset(a):
        f = lambda E: np.exp(-(E - mu) ** 2 / (2 * sig ** 2) + a * (E - c))
        num = integrate.quad(lambda E: (E - c) * f(E), lo, hi)[0]
        return num / integrate.quad(f, lo, hi)[0]

    root = optimize.brentq(mean_offset, -5, 5)
    assert abs(root - c / sig ** 2) < 0.01     # beta-convention: a = -d ln rho / dE + O(dE^2)
    # sample the restricted density at coupling a by rejection from uniform
    def draw(a, size):
        out = np.empty(0)
        g = lambda E: -(E - mu) ** 2 / (2 * sig ** 2) + a * E
        m = max(g(lo), g(hi), g(min(max(mu + a * sig ** 2, lo), hi)))
        while out.size < size:
            E = rng.uniform(lo, hi, 4 * size)
            keep = rng.random(E.size) < np.exp(g(E) - m)
            out = np.concatenate([out, E[keep]])
        return out[:size]
    a = 0.0
    hist = []
    for n in range(300):
        a = oracle.rm_step(a, draw(a, 200).mean(), c, n, w)
        hist.append(a)
    sd = np.sqrt(12.0 / (w * w * 200 * 300))
    assert abs(a - root) < 5 * sd

"""Oracle pins for the reconstruction (eq. (kk3a) trapezium recursion, midpoint
sums eqs. (l19)-(l20), C_V of Sec. 3.4) and for the warm-start network
(forward, gradient, Adam) against independent implementations."""
import numpy as np
import pytest
from scipy import optimize

import oracle


def _gauss_case(n=1000, s=0.5, mu=100.0, sig=20.0, lo=-60.0):
    c = lo + s * (np.arange(n) + 0.5)
    a = (c - mu) / sig ** 2                 # beta-convention: a = -d ln rho/dE for a Gaussian rho
    return c, a, s, mu, sig


def test_ln_rho_trapezium_exact_for_gaussian():
    c, a, s, mu, sig = _gauss_case()
    lr = oracle.ln_rho(a, s)
    exact = -(c - mu) ** 2 / (2 * sig ** 2) + (c[0] - mu) ** 2 / (2 * sig ** 2)
    assert np.max(np.abs(lr - exact)) < 1e-10 * np.max(np.abs(exact))


def test_ln_rho_error_is_second_order_for_curved_density():
    # ln rho = -E^4/4 on [0.2, 1.2]: a(E) = E^3; trapezium error O(s^2)
    errs = []
    for s in (0.02, 0.01):
        c = 0.2 + s * (np.arange(int(round(1.0 / s))) + 0.5)
        lr = oracle.ln_rho(c ** 3, s)
        exact = -(c ** 4 - c[0] ** 4) / 4
        errs.append(np.max(np.abs(lr - exact)))
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("beta", [-0.05, 0.0, 0.03, 0.1])
def test_moments_of_discretised_gaussian(beta):
    c, a, s, mu, sig = _gauss_case()
    six_v = 1000.0
    _, u, cv = oracle.reconstruct(c, a, s, six_v, [beta])
    logw = -(c - mu) ** 2 / (2 * sig ** 2) + beta * c
    p = np.exp(logw - logw.max())
    p /= p.sum()
    m = np.sum(p * c)
    var = np.sum(p * (c - m) ** 2)
    assert abs(u[0] * six_v - m) < 1e-10 * abs(m)
    assert abs(cv[0] * six_v - var) < 1e-9 * var
    # continuum: <E> = mu + beta sig^2, Var = sig^2 (range covers > 5 sigma)
    assert abs(m - (mu + beta * sig ** 2)) < 1e-6 * sig
    assert abs(var / sig ** 2 - 1) < 1e-3


def test_beta_c_of_two_phase_density():
    # ln rho: two Gaussian bumps of unequal width; find argmax Var(E) independently
    s = 0.25
    c = 50 + s * (np.arange(800) + 0.5)
    def lnrho(E):
        return np.logaddexp(-(E - 90) ** 2 / (2 * 6 ** 2) - 1.0 * E,
                            -(E - 180) ** 2 / (2 * 9 ** 2) - 1.0 * E + 2.0)
    h = 1e-5
    a = -(lnrho(c + h) - lnrho(c - h)) / (2 * h)
    six_v = 600.0

    def var_at(b):
        # beta-convention weight; ln rho rebuilt by trapezium from a, independently
        L = np.concatenate([[0.0], -np.cumsum(0.5 * s * (a[:-1] + a[1:]))])
        x = L + b * c
        p = np.exp(x - x.max()); p /= p.sum()
        m = np.sum(p * c)
        return np.sum(p * (c - m) ** 2)
    grid = np.arange(0.9, 1.1, 1e-4)
    b0 = grid[np.argmax([var_at(b) for b in grid])]
    res = optimize.minimize_scalar(lambda b: -var_at(b), bracket=(b0 - 1e-4, b0, b0 + 1e-4), tol=1e-12)
    bc, peak = oracle.beta_c(c, a, s, six_v, 0.9, 1.1, h=1e-5, tol=1e-10)
    assert abs(bc - res.x) < 2e-6
    assert abs(peak * six_v / var_at(res.x) - 1) < 1e-8


def _torch_mlp(w):
    import torch
    W1 = torch.tensor(w[0:128].reshape(64, 2), dtype=torch.float64, requires_grad=True)
    b1 = torch.tensor(w[128:192], dtype=torch.float64, requires_grad=True)
    W2 = torch.tensor(w[192:4288].reshape(64, 64), dtype=torch.float64, requires_grad=True)
    b2 = torch.tensor(w[4288:4352], dtype=torch.float64, requires_grad=True)
    W3 = torch.tensor(w[4352:4416].reshape(1, 64), dtype=torch.float64, requires_grad=True)
    b3 = torch.tensor(w[4416:4417], dtype=torch.float64, requires_grad=True)
    params = [W1, b1, W2, b2, W3, b3]

    def f(u, invL):
        x = torch.stack([(torch.as_tensor(u) - 0.6) / 0.1, (torch.as_tensor(invL) - 0.0875) / 0.0375], 1)
        h1 = torch.tanh(x @ W1.T + b1)
        h2 = torch.tanh(h1 @ W2.T + b2)
        return 1.0 + 0.1 * (h2 @ W3.T + b3)[:, 0]
    return f, params


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.55, 0.7, n)
    invL = 1.0 / rng.choice([8, 12, 16], n)
    a = 1.0 + 0.3 * (u - 0.6) + 0.2 * invL
    return u, invL, a


def test_mlp_init_xavier_and_forward_matches_torch():
    import torch
    w = oracle.mlp_init(7)
    assert w.size == oracle.N_PARAMS == 4417
    assert np.all(np.abs(w[0:128]) <= np.sqrt(6 / 66)) and np.all(w[128:192] == 0)
    assert np.all(np.abs(w[192:4288]) <= np.sqrt(6 / 128)) and np.all(w[4288:4352] == 0)
    assert np.all(np.abs(w[4352:4416]) <= np.sqrt(6 / 65)) and w[4416] == 0
    assert abs(w[192:4288].std() - np.sqrt(6 / 128) / np.sqrt(3)) < 0.01
    u, invL, a = _data()
    f, _ = _torch_mlp(w)
    ref = f(u, invL).detach().numpy()
    got = oracle.mlp_forward(w, u, invL)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_mlp_gradient_matches_autograd_and_finite_differences():
    import torch
    w = oracle.mlp_init(11)
    w[128:192] = 0.05
    u, invL, a = _data()
    loss, g = oracle.mlp_loss_grad(w, u, invL, a)
    f, params = _torch_mlp(w)
    tl = torch.mean((f(u, invL) - torch.as_tensor(a)) ** 2)
    tl.backward()
    tg = np.concatenate([p.grad.numpy().ravel() for p in params])
    assert abs(loss - tl.item()) < 1e-14
    assert np.max(np.abs(g - tg)) < 1e-12 * max(1.0, np.max(np.abs(tg)))
    rng = np.random.default_rng(1)
    for i in rng.choice(4417, 40, replace=False):
        e = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[i] += e; wm[i] -= e
        fd = (oracle.mlp_loss_grad(wp, u, invL, a)[0] - oracle.mlp_loss_grad(wm, u, invL, a)[0]) / (2 * e)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-3)


def test_adam_matches_torch_optimizer():
    import torch
    rng = np.random.default_rng(2)
    w = rng.normal(size=4417)
    m = np.zeros(4417); v = np.zeros(4417)
    tw = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=4417)
        oracle.mlp_adam(w, m, v, g, t, 1e-3)
        tw.grad = torch.tensor(g)
        opt.step()
        assert np.max(np.abs(w - tw.detach().numpy())) < 1e-13


def test_training_fits_smooth_target():
    u, invL, a = _data(160, seed=3)
    w0 = oracle.mlp_init(5)
    w, hist = oracle.mlp_train(w0, u, invL, a, epochs=1500, lr=3e-3)
    assert hist[-1] < 1e-2 * hist[0]
    assert np.sqrt(hist[-1]) < 2e-3

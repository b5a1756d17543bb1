"""Pins of the oracle surrogate network: GELU against its closed form and a
library routine, input gradients and weight gradients against central
differences, Adam against torch.optim.Adam.  CPU only."""
import math

import numpy as np
import torch

import workloads as W
from oracle import mlp


def _params(n_in=10, width=8, seed=1):
    p = W.mlp_init(n_in, width, seed)
    rng = np.random.default_rng(seed)
    p["mu"] = rng.normal(size=n_in) * 0.1
    p["inv_sigma"] = rng.uniform(0.5, 2.0, size=n_in)
    p["b1"] = rng.normal(size=width) * 0.1
    p["b2"] = rng.normal(size=width) * 0.1
    p["b3"] = np.array([0.3])
    p["w3"] = rng.normal(size=width)
    return p


def test_gelu_matches_closed_form_and_torch():
    z = torch.linspace(-6, 6, 1001, dtype=torch.float64)
    phi = 0.5 * (1 + torch.erf(z / math.sqrt(2)))
    assert torch.allclose(mlp.gelu(z), z * phi, rtol=0, atol=1e-15)
    assert torch.allclose(mlp.gelu(z), torch.nn.functional.gelu(z), rtol=0, atol=1e-14)


def test_forward_shapes_and_hand_evaluation():
    p = _params()
    x = np.random.default_rng(2).normal(size=(3, 10))
    y, _ = mlp.forward(p, x)
    # one sample by hand with numpy + math.erf
    u = (x[0] - p["mu"]) * p["inv_sigma"]
    g = np.vectorize(lambda z: 0.5 * z * (1 + math.erf(z / math.sqrt(2))))
    h1 = g(p["W1"] @ u + p["b1"])
    h2 = g(p["W2"] @ h1 + p["b2"])
    assert abs(y[0] - (p["w3"] @ h2 + p["b3"][0])) < 1e-12


def test_input_gradient_matches_central_differences():
    p = _params()
    x = np.random.default_rng(3).normal(size=(4, 10))
    _, gx = mlp.forward(p, x, need_input_grad=True)
    eps = 1e-6
    for l in range(10):
        e = np.zeros(10)
        e[l] = eps
        fd = (mlp.forward(p, x + e)[0] - mlp.forward(p, x - e)[0]) / (2 * eps)
        assert np.allclose(fd, gx[:, l], rtol=1e-7, atol=1e-8)


def test_cost_gradient_chain_rule():
    p = _params()
    x = np.random.default_rng(4).normal(size=(5, 10))
    c, gc = mlp.cost_and_grad(p, x, 6)
    eps = 1e-6
    for l in range(6):
        e = np.zeros(10)
        e[l] = eps
        cp = np.expm1(mlp.forward(p, x + e)[0])
        cm = np.expm1(mlp.forward(p, x - e)[0])
        assert np.allclose((cp - cm) / (2 * eps), gc[:, l], rtol=1e-6, atol=1e-8)


def test_weight_gradients_match_central_differences():
    p = _params(n_in=6, width=5)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(7, 6))
    t = rng.normal(size=7)
    loss, g = mlp.loss_and_grads(p, x, t)
    eps = 1e-6
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = np.asarray(p[k], dtype=np.float64).ravel()
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            pp, pm = dict(p), dict(p)
            a, b = flat.copy(), flat.copy()
            a[idx] += eps
            b[idx] -= eps
            pp[k], pm[k] = a.reshape(np.shape(p[k])), b.reshape(np.shape(p[k]))
            fd = (mlp.loss_and_grads(pp, x, t)[0] - mlp.loss_and_grads(pm, x, t)[0]) / (2 * eps)
            assert abs(fd - g[k].ravel()[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_matches_torch():
    p = _params(n_in=6, width=5)
    rng = np.random.default_rng(6)
    names = ["W1", "b1", "W2", "b2", "w3", "b3"]
    tp = [torch.nn.Parameter(torch.tensor(np.asarray(p[k], dtype=np.float64))) for k in names]
    opt = torch.optim.Adam(tp, lr=1e-2)
    m = {k: np.zeros(np.shape(p[k])) for k in names}
    v = {k: np.zeros(np.shape(p[k])) for k in names}
    for t in range(1, 6):
        x = rng.normal(size=(9, 6))
        y = rng.normal(size=9)
        _, g = mlp.loss_and_grads(p, x, y)
        p, m, v = mlp.adam_update(p, g, m, v, t, lr=1e-2)
        for tt, k in zip(tp, names):
            tt.grad = torch.tensor(g[k])
        opt.step()
    for tt, k in zip(tp, names):
        assert np.allclose(tt.detach().numpy(), p[k], rtol=1e-12, atol=1e-13)


def test_surrogate_cost_adds_the_exact_bound_term():
    """With a network that outputs a constant log(1 + c0), C_hat is c0 plus
    the bound term, whose value and gradient are checked by hand: o = 0.07
    and D = -0.01 on push 0, D = 0.35 on push 1 (o_max 0.05, d_max 0.3)."""
    H, n_enc = 2, 3
    d = 6 * H
    p = W.mlp_init(d + n_enc, 8, 0)
    for k in ("W1", "W2", "w3"):
        p[k] = np.zeros_like(p[k])
    c0 = 2.5
    p["b3"] = np.array([math.log1p(c0)])
    w = W.cost_weights()
    th = np.zeros((2, d))
    th[0, 4], th[0, 5] = 0.07, -0.01
    th[0, 11] = 0.35
    th[1, 4], th[1, 5], th[1, 10], th[1, 11] = 0.01, 0.1, -0.03, 0.2  # inside every bound
    C, g = mlp.surrogate_cost_and_grad(p, th, np.ones(n_enc), w)
    b = w["bound"]
    L0 = (0.07 - w["o_max"]) ** 2 + 0.01 ** 2 + (0.35 - w["d_max"]) ** 2
    assert abs(C[0] - (c0 + b * L0)) < 1e-12 * (1 + b * L0)
    assert abs(C[1] - c0) < 1e-12
    want = np.zeros(d)
    want[4] = b * 2 * (0.07 - w["o_max"])
    want[5] = b * (-2) * 0.01
    want[11] = b * 2 * (0.35 - w["d_max"])
    assert np.allclose(g[0], want, rtol=1e-12, atol=1e-12)
    assert np.allclose(g[1], 0.0, atol=1e-15)


def test_surrogate_cost_without_bound_is_the_network_cost():
    p = _params(n_in=15, width=8)
    th = np.random.default_rng(5).normal(size=(4, 12)) * 0.02
    enc = np.random.default_rng(6).normal(size=3)
    w = dict(W.cost_weights(), bound=0.0)
    C, g = mlp.surrogate_cost_and_grad(p, th, enc, w)
    x = np.concatenate([th, np.repeat(enc[None], 4, 0)], 1)
    C2, g2 = mlp.cost_and_grad(p, x, 12)
    assert np.allclose(C, C2, rtol=1e-13) and np.allclose(g, g2, rtol=1e-12, atol=1e-14)


def test_standardization_is_mean_and_population_std():
    x = np.random.default_rng(8).normal(size=(500, 4)) * [1.0, 3.0, 1e-5, 0.0] + [0.0, 2.0, 1.0, 7.0]
    mu, isg = mlp.standardization(x)
    assert np.allclose(mu, [x[:, 0].mean(), x[:, 1].mean(), 1.0 + x[:, 2].mean() - 1.0, 7.0], atol=1e-12)
    assert abs(1 / isg[1] - np.sqrt(((x[:, 1] - x[:, 1].mean()) ** 2).mean())) < 1e-12
    assert isg[2] == 1e3 and isg[3] == 1e3  # floor of the standard deviation

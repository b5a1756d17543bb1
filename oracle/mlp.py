"""FP64 oracle of the learned surrogate of the rollout cost.

Test infrastructure only (see the package docstring).  The workload spec adds
a small network that predicts a plan's cost from the plan and a scene
encoding, so that early SVGD iterations can use its gradient instead of the
simulator's (the paper's method differentiates the simulator; the surrogate is
an extension evaluated only by the final true cost).

Network (float64 here):
    u  = (x - mu) * inv_sigma                  x = [theta (d), scene encoding (24)]
    h1 = gelu(W1 u + b1)                       W1: 256 x n_in
    h2 = gelu(W2 h1 + b2)                      W2: 256 x 256
    y  = w3 . h2 + b3                          y predicts log(1 + C)
    gelu(z) = z * Phi(z) = 0.5 z (1 + erf(z / sqrt 2))
    C_hat = exp(y) - 1,   grad_theta C_hat = exp(y) * grad_theta y
Training: mean squared error of y against log(1 + C) over a minibatch, Adam on
the weights (mu and inv_sigma are fixed standardisation constants).

In the solver the network learns the rollout part of the cost only (the cost
of Appendix E-B with its bound weight set to zero); the bound term, a closed
form in the plan, is added exactly:
    C_hat(theta) = exp(y(theta, enc)) - 1 + b_b L_bound(theta)
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import sim

DT = torch.float64
WIDTH = 256


def gelu(z):
    return 0.5 * z * (1.0 + torch.erf(z / math.sqrt(2.0)))


def unpack(params: dict):
    return {k: torch.as_tensor(np.asarray(v, dtype=np.float64)) for k, v in params.items()}


def forward(params: dict, x, need_input_grad=False):
    """y [M] and, optionally, dy/dx [M][n_in] (by autodiff)."""
    P = unpack(params)
    X = torch.as_tensor(np.asarray(x, dtype=np.float64)).clone().requires_grad_(need_input_grad)
    u = (X - P["mu"]) * P["inv_sigma"]
    h1 = gelu(u @ P["W1"].T + P["b1"])
    h2 = gelu(h1 @ P["W2"].T + P["b2"])
    y = h2 @ P["w3"] + P["b3"]
    if not need_input_grad:
        return y.detach().numpy(), None
    (gx,) = torch.autograd.grad(y.sum(), X)
    return y.detach().numpy(), gx.numpy()


def cost_and_grad(params: dict, x, d):
    """Surrogate cost C_hat = exp(y) - 1 and dC_hat/dtheta over the first d inputs."""
    y, gx = forward(params, x, need_input_grad=True)
    return np.expm1(y), np.exp(y)[:, None] * gx[:, :d]


def loss_and_grads(params: dict, x, target):
    """Mean squared error of y against target and its gradient w.r.t. every
    trained tensor (W1, b1, W2, b2, w3, b3)."""
    P = unpack(params)
    names = ["W1", "b1", "W2", "b2", "w3", "b3"]
    for k in names:
        P[k].requires_grad_(True)
    X = torch.as_tensor(np.asarray(x, dtype=np.float64))
    t = torch.as_tensor(np.asarray(target, dtype=np.float64))
    u = (X - P["mu"]) * P["inv_sigma"]
    h1 = gelu(u @ P["W1"].T + P["b1"])
    h2 = gelu(h1 @ P["W2"].T + P["b2"])
    y = h2 @ P["w3"] + P["b3"]
    loss = ((y - t) ** 2).mean()
    grads = torch.autograd.grad(loss, [P[k] for k in names])
    return float(loss), {k: g.numpy() for k, g in zip(names, grads)}


def adam_update(params: dict, grads: dict, m: dict, v: dict, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on the trained tensors (in place on copies); returns new dicts."""
    out_p, out_m, out_v = dict(params), dict(m), dict(v)
    for k, g in grads.items():
        mm = beta1 * np.asarray(m[k]) + (1 - beta1) * g
        vv = beta2 * np.asarray(v[k]) + (1 - beta2) * g * g
        mhat = mm / (1 - beta1 ** t)
        vhat = vv / (1 - beta2 ** t)
        out_p[k] = np.asarray(params[k], dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        out_m[k], out_v[k] = mm, vv
    return out_p, out_m, out_v


def _net(P, X):
    u = (X - P["mu"]) * P["inv_sigma"]
    h1 = gelu(u @ P["W1"].T + P["b1"])
    h2 = gelu(h1 @ P["W2"].T + P["b2"])
    return h2 @ P["w3"] + P["b3"]


def surrogate_cost_and_grad(params: dict, theta, enc, w: dict):
    """C_hat and dC_hat/dtheta of plans theta [N][d] (d = 6H) in the scene
    encoded by enc [n_in - d]: the network's rollout-cost prediction plus the
    exact bound term."""
    P = unpack(params)
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    N, d = th.shape
    e = torch.as_tensor(np.asarray(enc, dtype=np.float64)).reshape(1, -1).expand(N, -1)
    y = _net(P, torch.cat([th, e], dim=1))
    C = torch.expm1(y) + float(w["bound"]) * sim.bound_term(th, w, d // 6)
    (g,) = torch.autograd.grad(C.sum(), th)
    return C.detach().numpy(), g.numpy()


def training_loss_and_grads(params: dict, x, cost):
    """loss_and_grads against the targets log(1 + cost) of labelled rollouts."""
    return loss_and_grads(params, x, np.log1p(np.asarray(cost, dtype=np.float64)))


def standardization(x):
    """mu and inv_sigma = 1/max(sigma, 1e-3) of inputs x [M][n_in] (population
    standard deviation)."""
    x = np.asarray(x, dtype=np.float64)
    return x.mean(0), 1.0 / np.maximum(x.std(0), 1e-3)

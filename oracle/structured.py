"""FP64 oracle of the SVGD direction under the structured pusher kernel.

Test infrastructure only (see the package docstring).  Plain PyTorch CPU ops
in float64.

Appendix E-C builds the kernel additively, one group of terms per action k:

    K(theta, theta') = sum_k [ alpha_g RBF(g_k, g_k') + alpha_z RBF(softmax a_k, softmax a_k')
                               + alpha_p VM(phi_k, phi_k') ]

with RBF(x, x') = exp(-|x - x'|^2 / h) and the von Mises kernel read as
VM(p, p') = exp(kappa (cos(p - p') - 1)) (its value at p = p' is 1, like the
RBF terms; the paper names the kernel without its normalisation).  Two
particle layouts:

* LAYOUT_PUSH: per action [a_k (4 logits), o_k, D_k]; g_k = (o_k, D_k), the
  action's continuous parameters; no angle (d = 6K).
* LAYOUT_POSE: the paper's [a_1..a_K, g_1..g_K] with g_k = (x, y, phi) an
  intermediate goal pose; the RBF takes (x, y), the von Mises term phi (d = 7K).

The SVGD direction is Eq. (1) (Eq. (4) with importance weights w_j):

    phi_i = (1/N) sum_j w_j [ K(theta_j, theta_i) grad log rho(theta_j) + grad_{theta_j} K(theta_j, theta_i) ]

the kernel gradient taken by reverse-mode autodiff of the kernel's definition.

Bandwidths (the paper gives none for this kernel): per RBF component c, the
median heuristic applied to the component's features over all actions,
h_c = max(m2_c / ln N, 1e-12) / K with m2_c the lower median over pairs
i < j of sum_k |c_ik - c_jk|^2, so that each single action's term sits near
1/N at the median spread; a positive caller value overrides it.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import svgd as _svgd

LAYOUT_PUSH = 0
LAYOUT_POSE = 1
DT = torch.float64


def dim(layout: int, K: int) -> int:
    return (6 if layout == LAYOUT_PUSH else 7) * K


def blocks(layout: int, K: int):
    """Coordinate indices: a [K][4], g [K][2], p [K] (None for the push layout)."""
    if layout == LAYOUT_PUSH:
        a = [[6 * k + c for c in range(4)] for k in range(K)]
        g = [[6 * k + 4, 6 * k + 5] for k in range(K)]
        return a, g, None
    if layout == LAYOUT_POSE:
        a = [[4 * k + c for c in range(4)] for k in range(K)]
        g = [[4 * K + 3 * k, 4 * K + 3 * k + 1] for k in range(K)]
        p = [4 * K + 3 * k + 2 for k in range(K)]
        return a, g, p
    raise ValueError(f"unknown layout {layout}")


def make_spec(layout=LAYOUT_PUSH, K=1, alpha_g=1.0, alpha_z=1.0, alpha_p=1.0, h_g=0.0, h_z=0.0, kappa=1.0):
    return dict(layout=layout, K=K, alpha_g=alpha_g, alpha_z=alpha_z, alpha_p=alpha_p, h_g=h_g, h_z=h_z,
                kappa=kappa)


def features(theta, spec):
    """Per-action softmax(a_k) [N][K][4], g_k [N][K][2] and phi_k [N][K] (or None)."""
    th = torch.as_tensor(theta, dtype=DT)
    a, g, p = blocks(spec["layout"], spec["K"])
    s = torch.softmax(th[:, torch.tensor(a)], dim=-1)
    gg = th[:, torch.tensor(g)]
    pp = th[:, torch.tensor(p)] if p is not None else None
    return s, gg, pp


def bandwidths(theta, spec):
    """(h_g, h_z): fixed if positive, else the per-component median heuristic."""
    th = np.asarray(theta, dtype=np.float64)
    N, K = th.shape[0], spec["K"]
    s, gg, _ = features(th, spec)

    def heur(f):
        if N < 2:
            return 1.0
        return max(_svgd.median_sqdist(f.reshape(N, -1).numpy()) / math.log(N), _svgd.H_FLOOR) / K

    hg = spec["h_g"] if spec["h_g"] > 0 else heur(gg)
    hz = spec["h_z"] if spec["h_z"] > 0 else heur(s)
    return float(hg), float(hz)


def kernel_pairs(x, y, spec, hg, hz):
    """K(x_m, y_m) for particle rows x, y of equal leading shape [..., d]."""
    a, g, p = blocks(spec["layout"], spec["K"])
    out = torch.zeros(x.shape[:-1], dtype=DT)
    for k in range(spec["K"]):
        sx = torch.softmax(x[..., a[k]], dim=-1)
        sy = torch.softmax(y[..., a[k]], dim=-1)
        out = out + spec["alpha_z"] * torch.exp(-((sx - sy) ** 2).sum(-1) / hz)
        out = out + spec["alpha_g"] * torch.exp(-((x[..., g[k]] - y[..., g[k]]) ** 2).sum(-1) / hg)
        if p is not None:
            out = out + spec["alpha_p"] * torch.exp(spec["kappa"] * (torch.cos(x[..., p[k]] - y[..., p[k]]) - 1.0))
    return out


def kernel_matrix(theta, spec, hg, hz):
    """K[i][j] = K(theta_i, theta_j)."""
    th = torch.as_tensor(theta, dtype=DT)
    N = th.shape[0]
    return kernel_pairs(th[:, None, :].expand(N, N, -1), th[None, :, :].expand(N, N, -1), spec, hg, hz)


def phi(theta, grad, spec, hg=None, hz=None, w=None, rows=None):
    """The SVGD direction for rows i (all rows by default): [len(rows)][d].
    N = 1 has no pairs: phi = grad."""
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    gr = torch.as_tensor(np.asarray(grad, dtype=np.float64))
    N, d = th.shape
    if rows is None:
        rows = np.arange(N)
    rows = np.asarray(rows)
    if N == 1:
        return gr[rows].numpy().copy()
    if hg is None or hz is None:
        hg, hz = bandwidths(th.numpy(), spec)
    wt = torch.ones(N, dtype=DT) if w is None else torch.as_tensor(np.asarray(w, dtype=np.float64))
    xj = th[None, :, :].expand(len(rows), N, d).clone().requires_grad_(True)  # the differentiated argument
    yi = th[torch.as_tensor(rows)][:, None, :].expand(len(rows), N, d)
    Kij = kernel_pairs(xj, yi, spec, hg, hz)  # [i][j] = K(theta_j, theta_i)
    (dK,) = torch.autograd.grad(Kij.sum(), xj)  # [i][j] = grad_{theta_j} K(theta_j, theta_i)
    Kw = Kij.detach() * wt[None, :]
    out = Kw @ gr + (dK * wt[None, :, None]).sum(dim=1)
    return (out / N).numpy()

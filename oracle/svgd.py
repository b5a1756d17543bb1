"""FP64 oracle of the SVGD step, the update rules and the solve loop.

Test infrastructure only (see the package docstring).  numpy float64.

* Eq. (1): theta_i <- theta_i + (eps/n) sum_j [ grad log p(theta_j) k_ji + grad_{theta_j} k_ji ].
  With the RBF kernel k(t, t') = exp(-|t - t'|^2 / h) the repulsive term is
  grad_{theta_j} k_ji = (2/h)(theta_i - theta_j) k_ji, so the direction is
      phi_i = (1/N) sum_j K_ij [ g_j + (2/h)(theta_i - theta_j) ],  g = grad log rho.
* Bandwidth by the median heuristic (Appendix D-B): m2 = the lower median of
  the N(N-1)/2 squared distances with i < j (the ceil(P/2)-th smallest),
  h = max(m2 / ln N, 1e-12); a positive caller bandwidth overrides it.
* Update: Adam on -phi (bias-corrected, step t counted from 1) or the plain
  step theta += lr * phi of Algorithm 1.
* Solve (Algorithm 1, SVGD phase): rollout -> log-posterior gradient ->
  bandwidth -> phi -> update, for a fixed number of iterations; then the
  discrete plan Gamma(a) and the final true cost.
"""
from __future__ import annotations

import math

import numpy as np

from . import sim

H_FLOOR = 1e-12


def pairwise_sqdist(theta: np.ndarray) -> np.ndarray:
    """D_ij = sum_l (theta_il - theta_jl)^2 by direct differences."""
    diff = theta[:, None, :] - theta[None, :, :]
    return np.einsum("ijl,ijl->ij", diff, diff)


def median_sqdist(theta: np.ndarray) -> float:
    """Lower median of the squared distances over pairs i < j."""
    N = theta.shape[0]
    if N < 2:
        raise ValueError("median needs N >= 2")
    D = pairwise_sqdist(theta)
    iu = np.triu_indices(N, k=1)
    vals = np.sort(D[iu])
    P = vals.size
    return float(vals[(P + 1) // 2 - 1])


def bandwidth(theta: np.ndarray, fixed: float = 0.0) -> float:
    """h = m2 / ln N (median heuristic), or the fixed bandwidth if positive.
    N = 1 has no pairs; h = 1 is returned (phi = g for any h)."""
    if fixed > 0:
        return float(fixed)
    N = theta.shape[0]
    if N == 1:
        return 1.0
    return max(median_sqdist(theta) / math.log(N), H_FLOOR)


def kernel_matrix(theta: np.ndarray, h: float) -> np.ndarray:
    return np.exp(-pairwise_sqdist(theta) / h)


def svgd_phi(theta: np.ndarray, g: np.ndarray, h: float, w: np.ndarray | None = None) -> np.ndarray:
    """phi_i = (1/N) sum_j K_ij [ g_j + (2/h)(theta_i - theta_j) ]  (Eq. 1);
    with importance weights w (mean 1) each term j is scaled by w_j, which is
    Eq. (4)'s sum of (w_j / sum w) [...]."""
    N = theta.shape[0]
    K = kernel_matrix(theta, h)
    if w is not None:
        K = K * np.asarray(w, dtype=np.float64)[None, :]
    drive = K @ g
    repulse = (2.0 / h) * (theta * K.sum(axis=1, keepdims=True) - K @ theta)
    return (drive + repulse) / N


def svgd_phi_rows(theta: np.ndarray, g: np.ndarray, h: float, rows, w: np.ndarray | None = None,
                  chunk: int = 32) -> np.ndarray:
    """phi_i of Eq. (1) for the particles i in ``rows`` only: the same sum as
    ``svgd_phi`` written per row (direct differences to every particle j),
    so large particle sets need no N x N matrix.  Returns [len(rows)][d]."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    N = theta.shape[0]
    wj = np.ones(N) if w is None else np.asarray(w, dtype=np.float64)
    out = np.empty((rows.size, theta.shape[1]))
    for s in range(0, rows.size, chunk):
        r = rows[s:s + chunk]
        diff = theta[r][:, None, :] - theta[None, :, :]          # theta_i - theta_j
        k = np.exp(-np.einsum("rjl,rjl->rj", diff, diff) / h) * wj[None, :]
        out[s:s + chunk] = (k @ g + (2.0 / h) * np.einsum("rj,rjl->rl", k, diff)) / N
    return out


def median_sqdist_blocked(theta: np.ndarray, block: int = 16) -> float:
    """The same lower median as ``median_sqdist``, with the pair distances
    (direct differences) of a block of rows i against the columns j > i
    formed one block at a time: P values held, no N x N x d array."""
    theta = np.asarray(theta, dtype=np.float64)
    N = theta.shape[0]
    if N < 2:
        raise ValueError("median needs N >= 2")
    parts = []
    for s in range(0, N - 1, block):
        e = min(s + block, N - 1)
        diff = theta[s:e][:, None, :] - theta[None, s + 1:, :]      # rows s..e-1, columns s+1..N-1
        D = np.einsum("rjl,rjl->rj", diff, diff)
        i = np.arange(s, e)[:, None]
        j = np.arange(s + 1, N)[None, :]
        parts.append(D[j > i])
    D = np.concatenate(parts)
    k = (D.size + 1) // 2
    return float(np.partition(D, k - 1)[k - 1])


def dsvgd_weights(c_relaxed: np.ndarray, c_discrete: np.ndarray) -> np.ndarray:
    """Importance weights of Eq. (4): the relaxed plan's likelihood over the
    discrete plan's, exp(-C_rel) / exp(-C_disc), scaled to mean 1.  A
    non-finite log-weight gives weight 0; all non-finite gives weights 1."""
    lw = np.asarray(c_discrete, dtype=np.float64) - np.asarray(c_relaxed, dtype=np.float64)
    ok = np.isfinite(lw)
    if not ok.any():
        return np.ones_like(lw)
    e = np.where(ok, np.exp(np.where(ok, lw, 0.0) - lw[ok].max()), 0.0)
    return e * (lw.size / e.sum())


def adam_step(theta, phi, m, v, t, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step minimising along -phi; returns new (theta, m, v)."""
    grad = -phi
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def plain_step(theta, phi, lr):
    """theta <- theta + eps * Delta theta (Algorithm 1)."""
    return theta + lr * phi


def solve(scene, w, theta0, iters, t0=0, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8,
          use_adam=True, fixed_bandwidth=0.0, m0=None, v0=None, grad_fn=None,
          history=False, sgd_iters=0, dsvgd=False, kernel=None):
    """Algorithm 1 for fixed iteration counts: `iters` SVGD iterations, then
    `sgd_iters` SGD refinement iterations whose update takes each particle's
    own gradient of log rho (the second phase of Algorithm 1, Sec. III-C),
    with the same step rule and a continuing step counter.  dsvgd: the SVGD
    iterations weight the sum by the importance weights of Eq. (4), from the
    relaxed cost and the cost of executing each particle's discrete plan.

    kernel: None for the RBF kernel on theta, or a structured-kernel spec
    (``oracle.structured``, push layout; K is the scene's H) for the kernel of
    Appendix E-C in every SVGD iteration.

    grad_fn(theta) -> (cost, dC/dtheta) defaults to the simulator rollout.
    Returns dict(theta, m, v, cost, modes, h, [hist]).
    """
    th = np.array(theta0, dtype=np.float64, copy=True)
    m = np.zeros_like(th) if m0 is None else np.array(m0, dtype=np.float64, copy=True)
    v = np.zeros_like(th) if v0 is None else np.array(v0, dtype=np.float64, copy=True)
    if grad_fn is None:
        def grad_fn(x):
            return sim.cost_and_grad(scene, w, x)
    hist = []
    h = float("nan")
    for it in range(iters + sgd_iters):
        c, dC = grad_fn(th)
        g = -dC
        if it < iters:
            wts = dsvgd_weights(c, sim.readout(scene, w, th)[1]) if dsvgd else None
            if kernel is not None:
                from . import structured
                phi = structured.phi(th, g, dict(kernel, K=int(scene["H"])), w=wts)
            else:
                h = bandwidth(th, fixed_bandwidth)
                phi = g if th.shape[0] == 1 else svgd_phi(th, g, h, wts)
        else:
            phi = g
        if use_adam:
            th, m, v = adam_step(th, phi, m, v, t0 + it + 1, lr, beta1, beta2, eps)
        else:
            th = plain_step(th, phi, lr)
        if history:
            hist.append(dict(mean_cost=float(np.mean(c)), min_cost=float(np.min(c)), h=h))
    cost = sim.cost_np(scene, w, th)
    out = dict(theta=th, m=m, v=v, cost=cost, modes=sim.discrete_plan(th, int(scene["H"])), h=h)
    if history:
        out["hist"] = hist
    return out

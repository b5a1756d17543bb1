"""The FP32 floor of the 100-iteration solve parity test, measured on its own metric.

Runs the oracle's arithmetic in float32 on the CPU (``oracle.sim.rollout`` on
float32 tensors with its autodiff gradient; float32 median, SVGD direction and
Adam), from the seeded N = 1024, B = 3, H = 3, T = 200 workload at lr 1e-3, and
scores the particle states after 100 iterations against the stored FP64 result
(``cfg2_solve_lr1e-3_it100.npz``) exactly as ``tests/test_gpu_solve.py`` does:
the error of each coordinate divided by that coordinate's largest magnitude
over the particle set, normwise error, 99.9th percentile and worst coordinate.

Every variant is a correct FP32 evaluation of the same method; they differ only
in rounding, as any two FP32 implementations do:
  ieee        float32 arithmetic as torch/numpy round it
  gram        the SVGD distances in the centred Gram form
  theta_ulp:S the initial particles moved by one ulp in random directions
  grad_ulp:S  every iteration's gradient moved by one ulp in random directions
  trans_ulp:S every sqrt/exp/sin/cos/softplus result moved by one ulp in a
              random direction (what ~1-ulp hardware transcendentals do)
  all_ulp:S   all of the above together
The spread of the worst coordinate over these variants is the floor the GPU
bar is derived from.  Nothing here comes from the GPU path; the script calls
only ``oracle`` and ``workloads``.  Each run takes a few minutes on 2 threads:
    python tests/golden/fp32_floor.py VARIANT [threads [CASE]]
(CASE: a stored solve, cfg2_solve_lr1e-3_it100 by default)
"""
import math
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
import workloads as W  # noqa: E402
from oracle import sim  # noqa: E402

F32 = torch.float32


class _OneUlp:
    """Stand-in for torch / torch.nn.functional inside the oracle's rollout:
    transcendental results moved by one ulp in a random direction (value
    only; the derivative is the exact function's)."""

    def __init__(self, base, gen):
        self._b, self._g = base, gen

    def __getattr__(self, n):
        return getattr(self._b, n)

    def _pert(self, y):
        u = torch.rand(y.shape, generator=self._g)
        dirn = torch.where(u < 0.5, torch.full_like(y, -math.inf), torch.full_like(y, math.inf))
        return y + (torch.nextafter(y.detach(), dirn) - y.detach())

    def sqrt(self, x):
        return self._pert(torch.sqrt(x))

    def exp(self, x):
        return self._pert(torch.exp(x))

    def cos(self, x):
        return self._pert(torch.cos(x))

    def sin(self, x):
        return self._pert(torch.sin(x))

    def softplus(self, z, beta=1.0, threshold=20.0):
        return self._pert(torch.nn.functional.softplus(z, beta=beta, threshold=threshold))


def _grad32(scene, w, th):
    t = torch.as_tensor(th, dtype=F32).clone().requires_grad_(True)
    c = sim.rollout(scene, w, t)["cost"]
    (g,) = torch.autograd.grad(c.sum(), t)
    return g.numpy()


def _median32(th):
    diff = th[:, None, :] - th[None, :, :]
    D = (diff * diff).sum(axis=2, dtype=np.float32)
    v = np.sort(D[np.triu_indices(th.shape[0], k=1)])
    return np.float32(v[(v.size + 1) // 2 - 1])


def _phi32(th, g, h, gram):
    N = th.shape[0]
    if gram:
        x = (th - th.mean(axis=0, dtype=np.float32)).astype(np.float32)
        n2 = (x * x).sum(axis=1, dtype=np.float32)
        D = np.maximum(n2[:, None] + n2[None, :] - np.float32(2) * (x @ x.T), np.float32(0))
    else:
        diff = th[:, None, :] - th[None, :, :]
        D = (diff * diff).sum(axis=2, dtype=np.float32)
    K = np.exp(-D / np.float32(h)).astype(np.float32)
    rep = np.float32(2.0 / h) * (th * K.sum(axis=1, keepdims=True, dtype=np.float32) - K @ th)
    return ((K @ g + rep) / np.float32(N)).astype(np.float32)


def _ulp_noise(a, rng):
    s = rng.integers(-1, 2, size=a.shape)
    return np.where(s > 0, np.nextafter(a, np.float32(np.inf)),
                    np.where(s < 0, np.nextafter(a, np.float32(-np.inf)), a)).astype(np.float32)


def run(variant, case="cfg2_solve_lr1e-3_it100"):
    gold = np.load(os.path.join(HERE, case + ".npz"))
    iters, lr = int(gold["iters"]), float(gold["lr"])
    name, _, seed = variant.partition(":")
    seed = int(seed or 0)
    sim.DT = F32
    sim.NORMALS = sim.NORMALS.to(F32)
    sim.TANGENTS = sim.TANGENTS.to(F32)
    if name in ("trans_ulp", "all_ulp"):
        gen = torch.Generator().manual_seed(seed)
        sim.torch = _OneUlp(torch, gen)
        sim.F = _OneUlp(torch.nn.functional, gen)
    rng = np.random.default_rng(seed)
    scene, w, th0 = W.config_problem(int(gold["cfg"]))
    th = th0.astype(np.float32)
    if name in ("theta_ulp", "all_ulp"):
        th = _ulp_noise(th, rng)
    m, v = np.zeros_like(th), np.zeros_like(th)
    b1, b2, eps = 0.9, 0.999, 1e-8
    for it in range(iters):
        g = (-_grad32(scene, w, th)).astype(np.float32)
        if name in ("grad_ulp", "all_ulp"):
            g = _ulp_noise(g, rng)
        h = np.float32(max(_median32(th) / math.log(th.shape[0]), 1e-12))
        phi = _phi32(th, g, h, gram=name in ("gram", "all_ulp"))
        t = it + 1
        m = (np.float32(b1) * m - np.float32(1 - b1) * phi).astype(np.float32)
        v = (np.float32(b2) * v + np.float32(1 - b2) * phi * phi).astype(np.float32)
        th = (th - np.float32(lr) * (m / np.float32(1 - b1 ** t))
              / (np.sqrt(v / np.float32(1 - b2 ** t)) + np.float32(eps))).astype(np.float32)
    ref = gold["theta"]
    got = th.astype(np.float64)
    e = np.abs(got - ref) / np.abs(ref).max(axis=0, keepdims=True)
    i, l = np.unravel_index(e.argmax(), e.shape)
    return dict(case=case, variant=variant, norm=float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                p999=float(np.percentile(e, 99.9)), max=float(e.max()), particle=int(i), coord=int(l))


if __name__ == "__main__":
    torch.set_num_threads(int(sys.argv[2]) if len(sys.argv) > 2 else 2)
    t0 = time.time()
    print(run(sys.argv[1], *sys.argv[3:4]), "%.0f s" % (time.time() - t0), flush=True)

"""Pins of the oracle's relaxation, cost terms and gradient.  CPU only."""
import math

import numpy as np
import pytest
import scipy.special
import scipy.stats
import torch

import workloads as W
from oracle import sim


def test_relaxation_matches_scipy_softmax():
    a = np.random.default_rng(0).standard_normal((50, 4)) * 5
    got = sim.relax(torch.tensor(a)).numpy()
    assert np.allclose(got, scipy.special.softmax(a, axis=1), rtol=1e-14, atol=0)


def test_discrete_plan_ties_pick_lowest_index():
    th = np.zeros((3, 12))
    th[0, 0:4] = [1, 3, 3, 0]
    th[1, 0:4] = [2, 2, 2, 2]
    th[2, 6:10] = [0, -1, 5, 5]
    modes = sim.discrete_plan(th, 2)
    assert modes[0, 0] == 1 and modes[1, 0] == 0 and modes[2, 1] == 2 and modes[2, 0] == 0


def test_even_partition_of_the_base_distribution():
    # Eq. (2)/Appendix A: Gamma splits the base density into m^K equal cells.
    # The proof is for a uniform base; N(0,1) logits are exchangeable too.
    H = 2
    th = np.zeros((400_000, 6 * H))
    rng = np.random.default_rng(1)
    for k in range(H):
        th[:, 6 * k:6 * k + 4] = rng.standard_normal((th.shape[0], 4))
        th[:, 6 * k + 4] = rng.uniform(-1, 1, th.shape[0])   # must not influence Gamma
        th[:, 6 * k + 5] = rng.uniform(5, 9, th.shape[0])
    m = sim.discrete_plan(th, H)
    cells = np.bincount(m[:, 0] * 4 + m[:, 1], minlength=16)
    p = scipy.stats.chisquare(cells).pvalue
    assert p > 1e-3, cells


def _costs(P, phiT, theta, scene, w):
    f64 = dict(dtype=torch.float64)
    Pt = [(torch.tensor([x], **f64), torch.tensor([y], **f64)) for x, y in P]
    return sim.total_cost(scene, w, torch.tensor(np.atleast_2d(theta), **f64), Pt,
                          torch.tensor([phiT], **f64)).item()


def test_target_loss_dead_zone_and_quadratic_outside():
    scene = W.make_scene(1, 0, 1, 1, 50, 0.01)
    scene["goal"] = [0.2, -0.1, 0.0]
    w = W.cost_weights(traj=0.0, bound=0.0, rot=0.0, target=1.0)
    th = np.array([0, 0, 0, 0, 0.0, 0.1])
    tol = scene["goal_tol"]
    assert _costs([(0, 0), (0.2 + 0.9 * tol, -0.1 - 0.9 * tol)], 0, th, scene, w) == 0.0
    c = _costs([(0, 0), (0.2 + tol + 0.03, -0.1 - tol - 0.01)], 0, th, scene, w)
    assert abs(c - (0.03 ** 2 + 0.01 ** 2)) < 1e-15


def test_rot_loss_closed_form():
    scene = W.make_scene(1, 0, 1, 1, 50, 0.01)
    w = W.cost_weights(traj=0.0, bound=0.0, rot=1.0, target=0.0)
    th = np.array([0, 0, 0, 0, 0.0, 0.1])
    c = _costs([(0, 0), (0, 0)], 0.7, th, scene, w)
    assert abs(c - (1 - math.cos(0.7 - scene["goal"][2]))) < 1e-15


def test_traj_loss_nonnegative_and_near_zero_on_monotone_paths():
    H = 4
    scene = W.make_scene(1, 0, 1, H, 50, 0.01)
    w = W.cost_weights(traj=1.0, bound=0.0, rot=0.0, target=0.0)
    th = np.tile([0, 0, 0, 0, 0.0, 0.1], H)
    rng = np.random.default_rng(3)
    eps = w["traj_eps"]
    for _ in range(200):
        P = [tuple(v) for v in rng.uniform(-0.3, 0.3, (H + 1, 2))]
        assert _costs(P, 0, th, scene, w) >= 0.0
    # a monotone staircase: detour-free, so only the k=H term's constant 2*eps
    # and O(eps^2 / step) smoothing remain
    P = [(0.05 * k, 0.03 * k) for k in range(H + 1)]
    c = _costs(P, 0, th, scene, w)
    assert 2 * eps <= c < 2 * eps + 40 * eps ** 2 / 0.03
    # a detour (out and back along x) costs about twice the overshoot
    P = [(0, 0), (0.1, 0), (0.0, 0.0), (0.0, 0.1), (0.0, 0.2)]
    c = _costs(P, 0, th, scene, w)
    assert abs(c - 2 * eps - 0.2) < 0.01


def test_bound_loss():
    scene = W.make_scene(1, 0, 1, 2, 50, 0.01)
    w = W.cost_weights(traj=0.0, target=0.0, rot=0.0, bound=1.0)
    P = [(0, 0)] * 3
    inside = np.array([0, 0, 0, 0, 0.04, 0.2, 0, 0, 0, 0, -0.04, 0.0])
    assert _costs(P, 0, inside, scene, w) == 0.0
    out = np.array([0, 0, 0, 0, 0.07, 0.35, 0, 0, 0, 0, -0.06, -0.02])
    om, dm = w["o_max"], w["d_max"]
    want = (0.07 - om) ** 2 + (0.35 - dm) ** 2 + (0.06 - om) ** 2 + 0.02 ** 2
    assert abs(_costs(P, 0, out, scene, w) - want) < 1e-15


def _central_fd(scene, w, th, eps):
    d = th.shape[1]
    fd = np.empty_like(th)
    for l in range(d):
        e = np.zeros(d)
        e[l] = eps
        fd[:, l] = (sim.cost_np(scene, w, th + e) - sim.cost_np(scene, w, th - e)) / (2 * eps)
    return fd


@pytest.mark.parametrize("cfg_like", ["cfg1", "cfg2"])
def test_gradient_matches_central_differences(cfg_like):
    # central FD at eps = 1e-6 in FP64 on every coordinate.  Stiff contact
    # coordinates carry an O(eps^2) truncation term above 1e-6; Richardson
    # extrapolation over eps and eps/2 removes it and must agree to 1e-6.
    if cfg_like == "cfg1":
        scene, w, th = W.config_problem(1)
        th = th[:4]
    else:
        scene = W.make_scene(2, 0, 3, 3, 60, 0.005)
        w = W.cost_weights(rot=2.0)
        th = W.make_particles(2, 0, 3, 3)
    _, g = sim.cost_and_grad(scene, w, th)
    fd = _central_fd(scene, w, th, 1e-6)
    fd2 = _central_fd(scene, w, th, 5e-7)
    rich = (4 * fd2 - fd) / 3
    scale = np.abs(g).max(axis=1, keepdims=True)
    assert (np.abs(rich - g) <= 1e-6 * scale).all()
    rel = np.abs(fd - g) / np.maximum(np.abs(g), 1e-3 * scale)
    assert np.median(rel) < 1e-6 and rel.max() < 1e-4


def test_fd_error_shrinks_quadratically():
    scene, w, th = W.config_problem(1)
    th = th[2:3]
    _, g = sim.cost_and_grad(scene, w, th)
    l = 5  # push distance of push 0
    errs = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        e = np.zeros(th.shape[1])
        e[l] = eps
        fd = (sim.cost_np(scene, w, th + e) - sim.cost_np(scene, w, th - e)) / (2 * eps)
        errs.append(abs(fd[0] - g[0, l]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs


def test_cost_bar_scales_gradient():
    scene, w, th = W.config_problem(1)
    th = th[:5]
    cb = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    _, g1 = sim.cost_and_grad(scene, w, th)
    _, g2 = sim.cost_and_grad(scene, w, th, cost_bar=cb)
    assert np.allclose(g2, g1 * cb[:, None], rtol=1e-13, atol=1e-12)


def test_long_horizon_gradient_matches_fd():
    # the 1-block, 5-push, T=1000 workload: the GPU checkpointed adjoint is held
    # to this gradient, pinned here to central differences in FP64 on all 16
    # randomly drawn particles (every perturbed particle in one batched
    # rollout), at eps = 1e-6 and, Richardson-extrapolated with eps = 5e-7,
    # to 1e-6 of each particle's largest gradient entry
    scene, w, th = W.config_problem(3)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(th.shape[0], 16, replace=False))
    x = th[pick]
    _, g = sim.cost_and_grad(scene, w, x)
    n, d = x.shape
    base = np.repeat(x, d, axis=0)
    fds = []
    for eps in (1e-6, 5e-7):
        steps = np.tile(np.eye(d) * eps, (n, 1))
        c = sim.cost_np(scene, w, np.concatenate([base + steps, base - steps]))
        fds.append(((c[: n * d] - c[n * d:]) / (2 * eps)).reshape(n, d))
    fd, fd2 = fds
    scale = np.abs(g).max(axis=1, keepdims=True)
    rel = np.abs(fd - g) / np.maximum(np.abs(g), 1e-3 * scale)
    assert np.median(rel) < 1e-6 and rel.max() < 1e-4
    rich = (4 * fd2 - fd) / 3
    err = (np.abs(rich - g) / scale).max(axis=1)
    print("FD (Richardson) error per particle, of its largest entry:", err.max(), flush=True)
    assert (err <= 1e-6).all(), err

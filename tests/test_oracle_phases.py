"""Pins of the oracle's per-phase split of the cost (the appendix on exploding
gradients: C = sum_k C_k with each C_k reading one action's trajectory, so
each action's parameters can follow their own term).  CPU only."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import sim


def _cases():
    s1, w1, th1 = W.config_problem(1)
    s2 = W.make_scene(2, 3, 3, 3, 60, 0.005)      # 3 blocks in contact range, 3 pushes
    w2 = W.cost_weights(rot=2.0)
    th2 = W.make_particles(2, 3, 5, 3)
    return [(s1, w1, th1[:5]), (s2, w2, th2)]


@pytest.mark.parametrize("case", [0, 1])
def test_phase_costs_sum_to_the_cost(case):
    scene, w, th = _cases()[case]
    with torch.no_grad():
        r = sim.phase_costs(scene, w, torch.as_tensor(th))
    total = torch.stack(r["costs"]).sum(0).numpy()
    ref = sim.cost_np(scene, w, th)
    assert len(r["costs"]) == scene["H"]
    assert np.allclose(total, ref, rtol=1e-13, atol=1e-12)
    assert np.array_equal(r["cost"].numpy(), ref)  # detaching phases keeps the value


@pytest.mark.parametrize("case", [0, 1])
def test_each_phase_cost_reaches_its_own_action_only(case):
    scene, w, th = _cases()[case]
    H = scene["H"]
    x = torch.as_tensor(th).clone().requires_grad_(True)
    r = sim.phase_costs(scene, w, x)
    for k in range(H):
        (g,) = torch.autograd.grad(r["costs"][k].sum(), x, retain_graph=True)
        g = g.numpy()
        outside = np.delete(g, np.s_[6 * k:6 * k + 6], axis=1)
        assert not outside.any(), k
        assert np.abs(g[:, 6 * k:6 * k + 6]).max() > 0


def test_single_push_split_equals_the_full_gradient():
    scene = W.make_scene(1, 0, 2, 1, 80, 0.005)
    w = W.cost_weights(rot=1.5)
    th = W.make_particles(1, 0, 6, 1)
    c0, g0 = sim.cost_and_grad(scene, w, th)
    c1, g1 = sim.per_phase_cost_and_grad(scene, w, th)
    assert np.allclose(c1, c0, rtol=1e-14)
    assert np.allclose(g1, g0, rtol=1e-12, atol=1e-12 * np.abs(g0).max())


@pytest.mark.parametrize("case", [0, 1])
def test_per_phase_gradient_matches_central_differences(case):
    """Block k of the split's gradient against central differences of C_k in
    theta_k with the other phases' positions held at their unperturbed values
    (eps 1e-6 and 5e-7, Richardson-extrapolated): to 1e-6 of each particle's
    largest entry."""
    scene, w, th = _cases()[case]
    H = scene["H"]
    n, d = th.shape
    _, g = sim.per_phase_cost_and_grad(scene, w, th)
    with torch.no_grad():
        frz = sim.phase_costs(scene, w, torch.as_tensor(th))["frozen"]
    fds = []
    for eps in (1e-6, 5e-7):
        fd = np.zeros_like(th)
        for l in range(d):
            k = l // 6
            e = np.zeros(d)
            e[l] = eps
            with torch.no_grad():
                cp = sim.phase_costs(scene, w, torch.as_tensor(th + e), frozen=frz)["costs"][k].numpy()
                cm = sim.phase_costs(scene, w, torch.as_tensor(th - e), frozen=frz)["costs"][k].numpy()
            fd[:, l] = (cp - cm) / (2 * eps)
        fds.append(fd)
    rich = (4 * fds[1] - fds[0]) / 3
    scale = np.abs(g).max(axis=1, keepdims=True)
    err = (np.abs(rich - g) / scale).max()
    print("per-phase FD error", err, flush=True)
    assert err <= 1e-6
    assert H >= 2 and not np.allclose(g, sim.cost_and_grad(scene, w, th)[1])  # the split does change it

"""Host side of the plan read-out, and the oracle's two-phase solve and
discrete read-out (CPU only)."""
import math

import numpy as np

import workloads as W
from oracle import sim, svgd
from tests.test_oracle_physics import discrete_rollout


def test_solution_histogram_counts_solutions_per_plan():
    from paper_2310_01775_amd.readout import plan_names, solution_histogram
    modes = np.array([[0, 1, 0, 3, 0], [2, 2, 2, 0, 2]])  # [H=2][N=5]
    cost = np.array([0.5, 3.0, 0.7, 0.1, 9.0])
    assert plan_names(modes) == ["N-S", "E-S", "N-S", "W-N", "N-S"]
    assert solution_histogram(modes, cost, 1.0) == {"N-S": 2, "W-N": 1}
    assert solution_histogram(modes, cost, 0.0) == {}


def test_oracle_refinement_is_plain_gradient_steps():
    # with the plain step and no SVGD iterations, each refinement iteration is
    # theta <- theta + lr * grad log rho = theta - lr * dC/dtheta
    scene = W.make_scene(62, 0, 2, 2, 30, 0.005)
    w = W.cost_weights()
    th = W.make_particles(62, 0, 3, 2)
    out = svgd.solve(scene, w, th, 0, lr=1e-3, use_adam=False, sgd_iters=2)
    x = th.astype(np.float64)
    for _ in range(2):
        _, dC = sim.cost_and_grad(scene, w, x)
        x = x - 1e-3 * dC
    assert np.allclose(out["theta"], x, rtol=0, atol=1e-15)


def test_oracle_readout_executes_the_discrete_plan():
    # the read-out particle rolls out like the separately written discrete rollout
    rng = np.random.default_rng(5)
    scene = W.make_scene(2, 11, 3, 3, 60, 0.005)
    th = W.make_particles(2, 11, 1, 3).astype(np.float64)
    th[0, [0, 1, 2, 3, 6, 7, 8, 9, 12, 13, 14, 15]] = rng.normal(0.0, 1.0, 12)
    modes = sim.discrete_plan(th, 3)[0]
    st, P = discrete_rollout(scene, [int(s) for s in modes], [th[0, 6 * k + 4] for k in range(3)],
                             [th[0, 6 * k + 5] for k in range(3)])
    _, _, _, bl = sim.record(scene, W.cost_weights(), sim.discrete_particles(th, 3))
    assert np.allclose(bl[-1][:, 0], np.array(st).ravel(), rtol=0, atol=1e-12)
    got_modes, cost = sim.readout(scene, W.cost_weights(), th)
    assert list(got_modes[0]) == list(modes)
    assert np.isfinite(cost).all()


def test_importance_weights_closed_form():
    c_rel = np.array([1.0, 2.0, 0.5, 4.0])
    c_disc = np.array([3.0, 2.0, 0.5, np.inf])
    w = svgd.dsvgd_weights(c_rel, c_disc)
    assert abs(w.mean() - 1.0) < 1e-15
    assert w[3] == 0.0
    # w_j / w_k = exp((C_disc,j - C_rel,j) - (C_disc,k - C_rel,k))
    assert abs(w[0] / w[1] - np.exp(2.0)) < 1e-12 and abs(w[1] / w[2] - 1.0) < 1e-15
    assert np.array_equal(svgd.dsvgd_weights(c_rel, c_rel), np.ones(4))


def test_weighted_direction_against_a_double_loop():
    rng = np.random.default_rng(3)
    N, d, h = 5, 3, 0.7
    th, g = rng.normal(size=(N, d)), rng.normal(size=(N, d))
    w = rng.uniform(0.0, 2.0, N)
    w *= N / w.sum()
    ref = np.zeros((N, d))
    for i in range(N):
        for j in range(N):
            k = math.exp(-((th[i] - th[j]) ** 2).sum() / h)
            ref[i] += (w[j] / w.sum()) * k * (g[j] + (2.0 / h) * (th[i] - th[j]))
    assert np.allclose(svgd.svgd_phi(th, g, h, w), ref, rtol=0, atol=1e-14)
    # equal weights are the unweighted direction
    assert np.allclose(svgd.svgd_phi(th, g, h, np.ones(N)), svgd.svgd_phi(th, g, h), rtol=0, atol=1e-15)

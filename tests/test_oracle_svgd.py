"""Pins of the oracle's SVGD step (Eq. 1), bandwidth, kernel and updates.  CPU only."""
import itertools
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import svgd


def brute_lower_median(theta):
    vals = []
    N = len(theta)
    for i in range(N):
        for j in range(i + 1, N):
            vals.append(sum((a - b) ** 2 for a, b in zip(theta[i], theta[j])))
    P = len(vals)
    k = math.ceil(P / 2)
    # the k-th smallest: the value v with #(<v) < k <= #(<=v)
    for v in vals:
        if sum(u < v for u in vals) < k <= sum(u <= v for u in vals):
            return v
    raise AssertionError


@pytest.mark.parametrize("N", [2, 3, 4, 7, 12])
def test_median_matches_brute_force_count(N):
    th = np.random.default_rng(N).standard_normal((N, 3))
    assert svgd.median_sqdist(th) == pytest.approx(brute_lower_median(th.tolist()), rel=1e-14)


def test_median_with_ties_is_exact_order_statistic():
    th = np.array([[0.0], [1.0], [2.0], [3.0]])  # distances 1,1,1,4,4,9 -> P=6, k=3 -> 1
    assert svgd.median_sqdist(th) == 1.0
    th = np.array([[0.0], [0.0], [0.0]])
    assert svgd.median_sqdist(th) == 0.0
    assert svgd.bandwidth(th) == svgd.H_FLOOR


def test_kernel_symmetric_psd_unit_diagonal():
    th = np.random.default_rng(0).standard_normal((64, 18))
    h = svgd.bandwidth(th)
    K = svgd.kernel_matrix(th, h)
    assert np.array_equal(K, K.T)
    assert np.array_equal(np.diag(K), np.ones(64))
    assert np.linalg.eigvalsh(K).min() > -1e-10 * 64


def test_phi_matches_double_loop():
    rng = np.random.default_rng(5)
    N, d = 6, 3
    th = rng.standard_normal((N, d))
    g = rng.standard_normal((N, d))
    h = 0.7
    want = np.zeros((N, d))
    for i in range(N):
        for j in range(N):
            k = math.exp(-sum((th[i, l] - th[j, l]) ** 2 for l in range(d)) / h)
            for l in range(d):
                # grad_{theta_j} k(theta_j, theta_i) = -(2/h)(theta_j - theta_i) k
                want[i, l] += g[j, l] * k - (2.0 / h) * (th[j, l] - th[i, l]) * k
    want /= N
    assert np.allclose(svgd.svgd_phi(th, g, h), want, rtol=1e-13, atol=1e-14)


def test_two_particle_closed_form():
    th = np.array([[0.0, 0.0], [1.0, 2.0]])
    g = np.array([[1.0, -1.0], [0.5, 0.25]])
    h = svgd.bandwidth(th)
    D = 5.0
    assert h == pytest.approx(D / math.log(2))
    k12 = 0.5  # exp(-D / (D / ln 2))
    phi = svgd.svgd_phi(th, g, h)
    rep = (2 / h) * (th[0] - th[1]) * k12
    assert np.allclose(phi[0], 0.5 * (g[0] + k12 * g[1] + rep), rtol=1e-14)
    assert np.allclose(phi[1], 0.5 * (g[1] + k12 * g[0] - rep), rtol=1e-14)


def test_single_particle_reduces_to_gradient_ascent():
    scene, w, th = W.config_problem(1)
    out = svgd.solve(scene, w, th[:1], iters=3, use_adam=False, lr=1e-4)
    # same as plain gradient ascent on log rho
    from oracle import sim
    x = th[:1].copy()
    for _ in range(3):
        _, dC = sim.cost_and_grad(scene, w, x)
        x = x - 1e-4 * dC
    assert np.allclose(out["theta"], x, rtol=0, atol=1e-15)


def test_gaussian_target_recovers_mean_and_variance():
    # the Gaussian-mixture illustration of Section IV reduced to one component:
    # grad log p = -Sigma^-1 (theta - mu); SVGD particles recover mu and Sigma
    mu = np.array([1.0, -2.0])
    var = np.array([0.5, 2.0])
    rng = np.random.default_rng(11)
    th = rng.standard_normal((200, 2)) * 0.3
    for _ in range(4000):
        g = -(th - mu) / var
        th = svgd.plain_step(th, svgd.svgd_phi(th, g, svgd.bandwidth(th)), 0.05)
    assert np.allclose(th.mean(axis=0), mu, atol=0.03)
    # finite-N SVGD with the median bandwidth under-disperses by a few percent
    assert np.allclose(th.var(axis=0), var, rtol=0.1)


def test_adam_matches_torch_optim_adam():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6))
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    p = torch.nn.Parameter(torch.tensor(x))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 30):
        phi = rng.standard_normal((4, 6)) * (10.0 ** rng.integers(-3, 3))
        x, m, v = svgd.adam_step(x, phi, m, v, t, 1e-2, 0.9, 0.999, 1e-8)
        p.grad = torch.tensor(-phi)  # Adam minimises; SVGD ascends along phi
        opt.step()
    assert np.allclose(x, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_solve_runs_and_reduces_cost():
    scene, w, th = W.config_problem(1)
    out = svgd.solve(scene, w, th, iters=30, lr=1e-2, history=True)
    assert out["hist"][-1]["mean_cost"] < 0.7 * out["hist"][0]["mean_cost"]
    assert out["modes"].shape == (32, 2)


def _double_loop_phi(th, g, h, w=None):
    """Eq. (1) written as a plain double loop (the weights of Eq. (4) scale term j)."""
    N, d = th.shape
    w = np.ones(N) if w is None else w
    want = np.zeros((N, d))
    for i in range(N):
        for j in range(N):
            k = w[j] * math.exp(-sum((th[i, l] - th[j, l]) ** 2 for l in range(d)) / h)
            for l in range(d):
                want[i, l] += g[j, l] * k + (2.0 / h) * (th[i, l] - th[j, l]) * k
    return want / N


@pytest.mark.parametrize("weighted", [False, True])
def test_row_sampled_phi_matches_double_loop_and_full_phi(weighted):
    rng = np.random.default_rng(11)
    N, d = 9, 4
    th = rng.standard_normal((N, d))
    g = rng.standard_normal((N, d)) * 3
    w = rng.uniform(0.2, 2.0, N) if weighted else None
    h = 1.3
    rows = np.array([7, 0, 4, 4])
    want = _double_loop_phi(th, g, h, w)[rows]
    got = svgd.svgd_phi_rows(th, g, h, rows, w=w, chunk=3)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-14)
    big = rng.standard_normal((300, 30))
    gb = rng.standard_normal((300, 30))
    hb = svgd.bandwidth(big)
    r = rng.choice(300, 40, replace=False)
    assert np.allclose(svgd.svgd_phi_rows(big, gb, hb, r), svgd.svgd_phi(big, gb, hb)[r], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("N", [2, 5, 12])
def test_blocked_median_matches_brute_force(N):
    th = np.random.default_rng(100 + N).standard_normal((N, 3))
    assert svgd.median_sqdist_blocked(th, block=4) == pytest.approx(brute_lower_median(th.tolist()), rel=1e-14)
    big = np.random.default_rng(N).standard_normal((257, 6))
    assert svgd.median_sqdist_blocked(big, block=16) == svgd.median_sqdist(big)

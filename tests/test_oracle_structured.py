"""Pins of the structured-kernel oracle (Appendix E-C) against facts fixed
outside it: the plain RBF oracle in the special cases the kernel reduces to,
a hand-derived per-pair double loop, a closed form of the von Mises term,
symmetries of the softmax and of angles, positive semi-definiteness, and
central finite differences of the kernel's definition."""
import math

import numpy as np
import pytest
import torch

from oracle import structured as S
from oracle import svgd

PUSH, POSE = S.LAYOUT_PUSH, S.LAYOUT_POSE


def _theta(rng, N, layout, K, scale=1.0):
    return rng.normal(0.0, scale, (N, S.dim(layout, K)))


def test_layout_blocks_cover_each_coordinate_once():
    for layout in (PUSH, POSE):
        for K in (1, 3, 8):
            a, g, p = S.blocks(layout, K)
            idx = [i for blk in a for i in blk] + [i for blk in g for i in blk] + (p or [])
            assert sorted(idx) == list(range(S.dim(layout, K)))


def test_rbf_only_reduces_to_the_plain_svgd_direction():
    # alpha_z = 0 and one action: K = exp(-|g - g'|^2 / h) on (o, D) only, so the
    # (o, D) part of phi is the plain Eq. (1) direction on those coordinates and
    # the logits only see the drive term K grad
    rng = np.random.default_rng(1)
    N, h = 9, 0.7
    th = _theta(rng, N, PUSH, 1)
    gr = rng.normal(0.0, 2.0, th.shape)
    spec = S.make_spec(PUSH, 1, alpha_g=1.0, alpha_z=0.0, h_g=h, h_z=1.0)
    got = S.phi(th, gr, spec)
    G = th[:, 4:6]
    assert np.allclose(got[:, 4:6], svgd.svgd_phi(G, gr[:, 4:6], h), rtol=1e-12, atol=1e-14)
    Kg = svgd.kernel_matrix(G, h)
    assert np.allclose(got[:, :4], Kg @ gr[:, :4] / N, rtol=1e-12, atol=1e-14)


def test_actions_add_up():
    # the kernel is a sum over actions, so phi is the sum of single-action
    # directions once the drive terms of the other actions are accounted for:
    # with grad = 0 only repulsion remains and it splits action by action
    rng = np.random.default_rng(2)
    N, K = 7, 3
    th = _theta(rng, N, PUSH, K)
    gr = np.zeros_like(th)
    spec = S.make_spec(PUSH, K, alpha_g=0.8, alpha_z=1.3, h_g=0.9, h_z=0.4)
    got = S.phi(th, gr, spec)
    for k in range(K):
        sub = th[:, 6 * k:6 * k + 6]
        one = S.phi(sub, np.zeros_like(sub), dict(spec, K=1))
        assert np.allclose(got[:, 6 * k:6 * k + 6], one, rtol=1e-12, atol=1e-15)


def _softmax(v):
    e = np.exp(v - v.max())
    return e / e.sum()


def test_matches_hand_derived_double_loop():
    # the kernel gradient written out by hand, pair by pair:
    #   RBF on x:       grad_{x_j} = (2/h)(x_i - x_j) e
    #   RBF on softmax: grad_{a_j} = J(a_j) (2/h)(s_i - s_j) e, J = diag(s) - s s^T
    #   von Mises:      grad_{p_j} = kappa sin(p_i - p_j) e
    rng = np.random.default_rng(3)
    for layout in (PUSH, POSE):
        N, K = 5, 2
        th = _theta(rng, N, layout, K)
        gr = rng.normal(0.0, 1.0, th.shape)
        w = rng.uniform(0.2, 2.0, N)
        spec = S.make_spec(layout, K, alpha_g=0.7, alpha_z=1.1, alpha_p=0.6, h_g=0.8, h_z=0.3, kappa=1.7)
        hg, hz = 0.8, 0.3
        a, g, p = S.blocks(layout, K)
        want = np.zeros_like(th)
        for i in range(N):
            for j in range(N):
                Kt, rep = 0.0, np.zeros(th.shape[1])
                for k in range(K):
                    si, sj = _softmax(th[i, a[k]]), _softmax(th[j, a[k]])
                    ez = math.exp(-np.sum((si - sj) ** 2) / hz)
                    J = np.diag(sj) - np.outer(sj, sj)
                    rep[a[k]] += spec["alpha_z"] * J @ ((2.0 / hz) * (si - sj) * ez)
                    xi, xj = th[i, g[k]], th[j, g[k]]
                    eg = math.exp(-np.sum((xi - xj) ** 2) / hg)
                    rep[g[k]] += spec["alpha_g"] * (2.0 / hg) * (xi - xj) * eg
                    Kt += spec["alpha_z"] * ez + spec["alpha_g"] * eg
                    if p is not None:
                        dp = th[i, p[k]] - th[j, p[k]]
                        ev = math.exp(spec["kappa"] * (math.cos(dp) - 1.0))
                        rep[p[k]] += spec["alpha_p"] * spec["kappa"] * math.sin(dp) * ev
                        Kt += spec["alpha_p"] * ev
                want[i] += w[j] * (Kt * gr[j] + rep)
        want /= N
        got = S.phi(th, gr, spec, w=w)
        assert np.allclose(got, want, rtol=1e-11, atol=1e-13), layout


def test_von_mises_two_particle_closed_form():
    # two particles differing only in one angle, zero gradient:
    # phi_1[p] = (1/2) kappa sin(p_1 - p_2) exp(kappa (cos(p_1 - p_2) - 1))
    K, kappa = 1, 2.3
    th = np.zeros((2, S.dim(POSE, K)))
    th[0, 6], th[1, 6] = 0.4, -0.9
    spec = S.make_spec(POSE, K, alpha_g=1.0, alpha_z=1.0, alpha_p=1.0, h_g=1.0, h_z=1.0, kappa=kappa)
    got = S.phi(th, np.zeros_like(th), spec)
    dp = 0.4 - (-0.9)
    want = 0.5 * kappa * math.sin(dp) * math.exp(kappa * (math.cos(dp) - 1.0))
    assert got[0, 6] == pytest.approx(want, rel=1e-13)
    assert got[1, 6] == pytest.approx(-want, rel=1e-13)
    assert np.abs(np.delete(got, 6, axis=1)).max() < 1e-15


def test_angle_wraparound_and_logit_shift_leave_phi_unchanged():
    rng = np.random.default_rng(4)
    N, K = 6, 2
    th = _theta(rng, N, POSE, K)
    gr = rng.normal(0.0, 1.0, th.shape)
    spec = S.make_spec(POSE, K, alpha_g=0.5, alpha_z=1.0, alpha_p=0.8, h_g=0.6, h_z=0.5, kappa=1.2)
    base = S.phi(th, gr, spec)
    a, _, p = S.blocks(POSE, K)
    wrapped = th.copy()
    wrapped[:, p] += 2.0 * math.pi * rng.integers(-2, 3, (N, K))
    assert np.allclose(S.phi(wrapped, gr, spec), base, rtol=1e-10, atol=1e-12)
    shifted = th.copy()
    for k in range(K):
        shifted[:, a[k]] += rng.normal(0.0, 3.0, (N, 1))  # softmax is shift invariant
    assert np.allclose(S.phi(shifted, gr, spec), base, rtol=1e-10, atol=1e-12)


def test_logit_repulsion_sums_to_zero_per_action():
    # the softmax Jacobian annihilates the all-ones direction, so with zero
    # gradient the four logit components of each action sum to zero
    rng = np.random.default_rng(5)
    N, K = 8, 3
    th = _theta(rng, N, PUSH, K, 2.0)
    spec = S.make_spec(PUSH, K, h_g=0.5, h_z=0.2)
    got = S.phi(th, np.zeros_like(th), spec)
    a, _, _ = S.blocks(PUSH, K)
    for k in range(K):
        assert np.abs(got[:, a[k]].sum(axis=1)).max() < 1e-15
        assert np.abs(got[:, a[k]]).max() > 1e-4


def test_kernel_matrix_is_symmetric_psd_with_known_diagonal():
    rng = np.random.default_rng(6)
    for layout in (PUSH, POSE):
        N, K = 40, 3
        th = _theta(rng, N, layout, K, 1.5)
        spec = S.make_spec(layout, K, alpha_g=0.5, alpha_z=2.0, alpha_p=0.7, kappa=3.0)
        hg, hz = S.bandwidths(th, spec)
        Km = S.kernel_matrix(th, spec, hg, hz).numpy()
        assert np.allclose(Km, Km.T, rtol=0, atol=1e-15)
        diag = K * (0.5 + 2.0 + (0.7 if layout == POSE else 0.0))
        assert np.allclose(np.diag(Km), diag, rtol=1e-15)
        assert np.linalg.eigvalsh(Km).min() > -1e-10 * diag


def test_kernel_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    K = 2
    spec = S.make_spec(POSE, K, alpha_g=0.9, alpha_z=1.4, alpha_p=0.5, kappa=2.0)
    hg, hz = 0.7, 0.25
    x = torch.tensor(rng.normal(0.0, 1.0, S.dim(POSE, K)), dtype=torch.float64, requires_grad=True)
    y = torch.tensor(rng.normal(0.0, 1.0, S.dim(POSE, K)), dtype=torch.float64)
    (gx,) = torch.autograd.grad(S.kernel_pairs(x, y, spec, hg, hz), x)
    eps = 1e-6
    for l in range(x.numel()):
        e = torch.zeros_like(x)
        e[l] = eps
        fd = (S.kernel_pairs(x.detach() + e, y, spec, hg, hz) - S.kernel_pairs(x.detach() - e, y, spec, hg, hz)) / (2 * eps)
        assert float(gx[l]) == pytest.approx(float(fd), rel=1e-6, abs=1e-9)


def test_bandwidths_by_brute_force_median():
    rng = np.random.default_rng(8)
    N, K = 11, 2
    th = _theta(rng, N, PUSH, K)
    spec = S.make_spec(PUSH, K)
    hg, hz = S.bandwidths(th, spec)

    def brute(f):
        vals = sorted(float(np.sum((f[i] - f[j]) ** 2)) for i in range(N) for j in range(i + 1, N))
        return vals[(len(vals) + 1) // 2 - 1] / math.log(N) / K

    G = np.concatenate([th[:, 6 * k + 4:6 * k + 6] for k in range(K)], axis=1)
    Z = np.concatenate([np.stack([_softmax(th[i, 6 * k:6 * k + 4]) for i in range(N)]) for k in range(K)], axis=1)
    assert hg == pytest.approx(brute(G), rel=1e-14)
    assert hz == pytest.approx(brute(Z), rel=1e-14)
    assert S.bandwidths(th, dict(spec, h_g=0.3, h_z=0.2)) == (0.3, 0.2)


def test_sampled_rows_and_single_particle():
    rng = np.random.default_rng(9)
    th = _theta(rng, 10, POSE, 2)
    gr = rng.normal(0.0, 1.0, th.shape)
    spec = S.make_spec(POSE, 2)
    full = S.phi(th, gr, spec)
    assert np.array_equal(S.phi(th, gr, spec, rows=[7, 2]), full[[7, 2]])
    one = S.phi(th[:1], gr[:1], spec)
    assert np.array_equal(one, gr[:1])

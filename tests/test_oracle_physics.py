"""Pins of the oracle's rollout (Section III-B) against closed forms, invariants
and a separately written discrete rollout.  CPU only."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import sim


def scene1(B=1, H=1, T=100, dt=0.005, **over):
    s = W.make_scene(99, 0, B, H, T, dt)
    s.update(over)
    return s


def run(scene, theta, vel0=None, w=None):
    w = w or W.cost_weights()
    return sim.record(scene, w, np.atleast_2d(theta), vel0=vel0)


def final_state(scene, theta, vel0=None):
    _, _, _, bl = run(scene, theta, vel0)
    return bl[-1][:, 0]  # [6B] of particle 0


def onehot_theta(sides, o, D):
    th = []
    for s, oo, dd in zip(sides, o, D):
        a = [-20.0] * 4
        a[s] = 20.0
        th += a + [oo, dd]
    return np.array([th])


def test_static_scene_is_bitwise_still():
    # no pusher stiffness, blocks far apart: nothing may move, not even by rounding
    s = scene1(B=2, k_push=0.0)
    s["pose0"] = [[0.0, 0.0, 0.3], [1.0, 1.0, -0.2]]
    st = final_state(s, onehot_theta([0], [0.01], [0.1]))
    want = np.array([0.0, 0.0, 0.3, 0, 0, 0, 1.0, 1.0, -0.2, 0, 0, 0])
    assert np.array_equal(st, want)


def test_momentum_conserved_without_friction_and_pusher():
    s = scene1(B=2, H=1, T=400, k_push=0.0, mu=[0.0, 0.0])
    s["pose0"] = [[0.0, 0.0, 0.0], [0.3, 0.02, 0.0]]
    vel0 = [[0.5, 0.0, 0.0], [-0.3, 0.0, 0.0]]
    _, tape, ends, bl = run(s, onehot_theta([0], [0.0], [0.0]), vel0)
    fin = bl[-1][:, 0]
    p0 = np.array([0.5 - 0.3, 0.0])
    p1 = np.array([fin[3] + fin[9], fin[4] + fin[10]])
    assert np.allclose(p1, p0, atol=1e-12)
    # the blocks did collide: block 0 reversed
    assert fin[3] < 0.0
    # elastic penalty spring + symplectic integrator: kinetic energy returns
    ke0 = 0.5 * (0.5 ** 2 + 0.3 ** 2)
    ke1 = 0.5 * (fin[3] ** 2 + fin[4] ** 2 + fin[9] ** 2 + fin[10] ** 2)
    assert abs(ke1 - ke0) / ke0 < 0.02


def test_sliding_decay_matches_coulomb_stop_distance():
    # v0 >> eps_v: deceleration ~ mu g; stop distance v0^2 / (2 mu g)
    s = scene1(B=1, T=400, dt=0.0025, k_push=0.0)
    v0 = 1.0
    fin = final_state(s, onehot_theta([0], [0.0], [0.0]), [[v0, 0.0, 0.0]])
    mu, g = s["mu"][0], s["g"]
    d = v0 ** 2 / (2 * mu * g)
    assert abs(fin[0] - d) < 0.02 * d
    assert abs(fin[3]) < 1e-3 and abs(fin[1]) < 1e-12


def test_spin_decay_matches_closed_form():
    # angular deceleration mu m g rho / I, rho = mean distance of a square's points
    s = scene1(B=1, T=400, dt=0.0025, k_push=0.0)
    w0 = 20.0
    fin = final_state(s, onehot_theta([0], [0.0], [0.0]), [[0.0, 0.0, w0]])
    h, m, mu, g = s["half"][0], s["mass"][0], s["mu"][0], s["g"]
    rho = 2 * h * (math.sqrt(2) + math.log(1 + math.sqrt(2))) / 6
    inertia = m * (2 * h) ** 2 / 6
    alpha = mu * m * g * rho / inertia
    ang = w0 ** 2 / (2 * alpha)
    assert abs(fin[2] - ang) < 0.02 * ang
    assert abs(fin[0]) < 1e-12 and abs(fin[1]) < 1e-12


def test_mean_distance_constant_of_a_square():
    # rho/(2h) = E|r| over a unit square about its centre, by quadrature
    n = 2000
    u = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(u, u)
    assert abs(np.sqrt(X ** 2 + Y ** 2).mean() - sim.RHO_SQUARE) < 1e-6


@pytest.mark.parametrize("side,axis,sign", [(0, 1, -1), (1, 0, -1), (2, 1, +1), (3, 0, +1)])
def test_centred_push_translates_along_minus_normal(side, axis, sign):
    s = scene1(B=1, H=1, T=200)
    D = 0.15
    fin = final_state(s, onehot_theta([side], [0.0], [D]))
    moved = fin[axis] * sign
    other = fin[1 - axis]
    # quasi-static: D - standoff minus the spring's equilibrium compression
    comp = s["mu"][0] * s["mass"][0] * s["g"] / s["k_push"]
    assert D - s["standoff"] - 4 * comp < moved < D - s["standoff"] + 0.01
    assert abs(other) < 1e-12 and abs(fin[2]) < 1e-12


def test_offset_push_turns_counter_clockwise():
    # South face pushed (force +y) at o>0 along t_S=(1,0): torque x*F_y > 0
    s = scene1(B=1, H=1, T=200)
    fin = final_state(s, onehot_theta([2], [0.03], [0.1]))
    assert fin[2] > 0.02
    fin2 = final_state(s, onehot_theta([2], [-0.03], [0.1]))
    assert abs(fin2[2] + fin[2]) < 1e-10  # mirror symmetry


def _cost(scene, theta):
    return sim.cost_np(scene, W.cost_weights(rot=3.0), theta)


def test_cost_invariant_under_translation_and_quarter_turns():
    base = W.make_scene(2, 5, 3, 3, 120, 0.005)
    th = W.make_particles(2, 5, 6, 3)
    c0 = _cost(base, th)
    moved = dict(base)
    moved["pose0"] = [[p[0] + 0.3, p[1] - 0.2, p[2]] for p in base["pose0"]]
    moved["goal"] = [base["goal"][0] + 0.3, base["goal"][1] - 0.2, base["goal"][2]]
    assert np.allclose(_cost(moved, th), c0, rtol=1e-9, atol=1e-9)
    for q in (1, 2, 3):
        ang = q * math.pi / 2
        c, sn = round(math.cos(ang)), round(math.sin(ang))
        rot = dict(base)
        rot["pose0"] = [[c * p[0] - sn * p[1], sn * p[0] + c * p[1], p[2] + ang] for p in base["pose0"]]
        g = base["goal"]
        rot["goal"] = [c * g[0] - sn * g[1], sn * g[0] + c * g[1], g[2] + ang]
        assert np.allclose(_cost(rot, th), c0, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------
# A separately written discrete rollout: one particle, one pusher per phase,
# scalar Python arithmetic.  One-hot relaxed logits must reproduce it.
# ---------------------------------------------------------------------------
def discrete_rollout(scene, sides, offs, dists):
    H, B, T, dt = scene["H"], scene["B"], scene["T"], scene["dt"]
    g, beta = scene["g"], scene["sp_beta"]

    def sp(z):
        return max(z, 0.0) + math.log1p(math.exp(-beta * abs(z))) / beta

    st = [list(scene["pose0"][b]) + [0.0, 0.0, 0.0] for b in range(B)]
    normal = {0: (0, 1), 1: (1, 0), 2: (0, -1), 3: (-1, 0)}
    P = []
    for k in range(H):
        t0 = math.ceil(k * T / H)
        t1 = math.ceil((k + 1) * T / H)
        anchor = tuple(st[0][:3])
        P.append((st[0][0], st[0][1]))
        n = normal[sides[k]]
        tg = (-n[1], n[0])
        for t in range(t0, t1):
            tau = (t - t0 + 1) / (t1 - t0)
            s5 = tau ** 3 * (10 - 15 * tau + 6 * tau * tau)
            F = [[0.0, 0.0, 0.0] for _ in range(B)]
            for b in range(B):
                h, m, mu = scene["half"][b], scene["mass"][b], scene["mu"][b]
                I = m * 4 * h * h / 6
                rho = 2 * h * (math.sqrt(2) + math.log(1 + math.sqrt(2))) / 6
                ev = max(scene["eps_v_scale"] * dt * mu * g, 1e-6)
                ew = ev * m * rho / I
                vx, vy, w = st[b][3:]
                nv = math.sqrt(vx * vx + vy * vy + ev * ev)
                F[b][0] -= mu * m * g * vx / nv
                F[b][1] -= mu * m * g * vy / nv
                F[b][2] -= mu * m * g * rho * w / math.sqrt(w * w + ew * ew)
            for b in range(B):
                for c in range(b + 1, B):
                    dx, dy = st[b][0] - st[c][0], st[b][1] - st[c][1]
                    r = math.sqrt(dx * dx + dy * dy + scene["eps_r"] ** 2)
                    f = scene["k_block"] * sp(scene["half"][b] + scene["half"][c] - r)
                    F[b][0] += f * dx / r
                    F[b][1] += f * dy / r
                    F[c][0] -= f * dx / r
                    F[c][1] -= f * dy / r
            h0 = scene["half"][0]
            dep = h0 + scene["standoff"] - dists[k] * s5
            lqx, lqy = dep * n[0] + offs[k] * tg[0], dep * n[1] + offs[k] * tg[1]
            ca, sa = math.cos(anchor[2]), math.sin(anchor[2])
            wx, wy = anchor[0] + ca * lqx - sa * lqy, anchor[1] + sa * lqx + ca * lqy
            rx, ry = wx - st[0][0], wy - st[0][1]
            c0, s0 = math.cos(st[0][2]), math.sin(st[0][2])
            bx, by = c0 * rx + s0 * ry, -s0 * rx + c0 * ry
            f = scene["k_push"] * sp(h0 - (n[0] * bx + n[1] * by))
            fx, fy = -f * (c0 * n[0] - s0 * n[1]), -f * (s0 * n[0] + c0 * n[1])
            F[0][0] += fx
            F[0][1] += fy
            F[0][2] += rx * fy - ry * fx
            for b in range(B):
                h, m = scene["half"][b], scene["mass"][b]
                I = m * 4 * h * h / 6
                st[b][3] += dt * F[b][0] / m
                st[b][4] += dt * F[b][1] / m
                st[b][5] += dt * F[b][2] / I
                st[b][0] += dt * st[b][3]
                st[b][1] += dt * st[b][4]
                st[b][2] += dt * st[b][5]
    P.append((st[0][0], st[0][1]))
    return st, P


@pytest.mark.parametrize("seed", [0, 1])
def test_one_hot_logits_reproduce_the_discrete_plan(seed):
    rng = np.random.default_rng(seed)
    scene = W.make_scene(2, 7 + seed, 3, 3, 60, 0.005)
    sides = [int(v) for v in rng.integers(0, 4, 3)]
    offs = [float(v) for v in rng.uniform(-0.04, 0.04, 3)]
    dists = [float(v) for v in rng.uniform(0.05, 0.2, 3)]
    st, P = discrete_rollout(scene, sides, offs, dists)
    # relaxed logits 40 e_s - 20: softmax weight of the chosen side = 1 - O(e^-40)
    th = np.array([sum(([40.0 * (s == j) - 20.0 for j in range(4)] + [o, d]
                        for s, o, d in zip(sides, offs, dists)), [])])
    _, _, _, bl = run(scene, th)
    assert np.allclose(bl[-1][:, 0], np.array(st).ravel(), rtol=0, atol=1e-12)
    for k in range(3):
        assert np.allclose(bl[k][0:2, 0], P[k], atol=1e-12)
    assert list(sim.discrete_plan(th, 3)[0]) == sides


def test_phase_mixture_is_the_weighted_outcome():
    # with mixed logits the next phase starts at sum_s z_s X_s(end)
    scene = W.make_scene(2, 3, 2, 2, 40, 0.005)
    th = W.make_particles(2, 3, 3, 2)
    _, tape, ends, bl = run(scene, th)
    z = torch.softmax(torch.tensor(th[:, 0:4]), dim=1).numpy()  # [N,4]
    mix = (ends[0] * z[None, :, :]).sum(axis=2)
    assert np.allclose(bl[1], mix, atol=1e-15)
    # every side sub-rollout starts from the shared phase-start state
    for s in range(4):
        assert np.array_equal(tape[0][:, :, s], bl[0])
        assert np.array_equal(tape[20][:, :, s], bl[1])

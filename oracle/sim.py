"""FP64 oracle of the differentiable block-pushing rollout and its cost.

Test infrastructure only (see the package docstring).  Plain PyTorch CPU ops
in float64, vectorised over particles (the batch dimension) and over the four
push sides; the time loop is an explicit Python loop over steps.  The gradient
of the cost with respect to the particle is taken by ``torch.autograd`` over
this exact code -- the paper obtains it the same way, by automatic
differentiation through the simulated trajectory (Section III-B).

Model (Section III-B: semi-implicit Euler, spring-based penalty contacts;
Section IV-A / Appendix E: the pushing task, N/E/S/W sides in the block frame):

  particle, push k:  a_k (4 logits), o_k (contact offset), D_k (push distance)
  relaxation:        z~_k = softmax(a_k)   (Eq. 5, the smooth surrogate of Gamma)
  phase of step t:   k(t) = floor(t H / T), t_k = ceil(k T / H), L_k = t_{k+1}-t_k
                     tau = (t - t_k + 1) / L_k,  s(tau) = 10tau^3 - 15tau^4 + 6tau^5
  phase mixture:     phase k runs once per side s from the shared start state S_k
                     (sub-rollout X_s with the pusher of side s only); the next
                     phase starts from S_{k+1} = sum_s z~_{k,s} X_s(t_{k+1})
  anchor:            A_k = block-0 pose of S_k
  virtual pusher s:  p_s = A.xy + R(A.phi) [ (h0 + delta - D_k s(tau)) n_s + o_k t_s ]
                     pen_s = h0 - n_s . R(phi0)^T (p_s - x0),  f_s = k_push sp(pen_s)
                     F_s = -f_s R(phi0) n_s acts on block 0 at p_s (force and torque)
  friction (each b): F = -mu m g v / sqrt(|v|^2 + ev^2),
                     tau = -mu m g rho w / sqrt(w^2 + ew^2),  rho = 2h(sqrt2 + ln(1+sqrt2))/6
                     ev = max(eps_v_scale dt mu g, 1e-6), ew = ev m rho / I, I = m (2h)^2 / 6
  block pairs b<c:   Delta = x_b - x_c, r = sqrt(|Delta|^2 + eps_r^2),
                     f = k_block sp(h_b + h_c - r),  F_b += f Delta/r, F_c -= f Delta/r
  integrator:        v += dt F/m, w += dt tau/I, then x += dt v, phi += dt w
  softplus:          sp(z) = log(1 + exp(beta z)) / beta
  cost (Appendix E-B, with the readings listed in the design notes):
     P_k = block-0 xy at t_k (P_0 start, P_H final)
     L_target = sum_{c in x,y} relu(|P_H,c - g_c| - tol)^2
     L_rot    = 1 - cos(phi0_T - g_phi)
     L_traj   = sum_{k=1..H} MH(P_{k-1},P_k) + MH(P_k,P_H) - MH(P_{k-1},P_H),
                MH(a,b) = sum_c sqrt((a_c-b_c)^2 + eps_a^2)
     L_bound  = sum_k relu(|o_k|-o_max)^2 + relu(-D_k)^2 + relu(D_k-D_max)^2
     C = b_t L_target + b_r L_rot + b_tr L_traj + b_b L_bound;  log rho = -C
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

DT = torch.float64

# Outward face normals in the block frame, sides in the order North, East,
# South, West (Section V-A lists the four sides; indices 0..3).
NORMALS = torch.tensor([[0.0, 1.0], [1.0, 0.0], [0.0, -1.0], [-1.0, 0.0]], dtype=DT)
# Face tangent t_s = (-n_y, n_x): the direction along which o_k offsets the contact.
TANGENTS = torch.stack([-NORMALS[:, 1], NORMALS[:, 0]], dim=1)

EPS_V_FLOOR = 1e-6  # m/s, keeps the frictionless case (mu = 0) finite at rest
RHO_SQUARE = (math.sqrt(2.0) + math.log(1.0 + math.sqrt(2.0))) / 6.0  # mean |r| / side


def phase_bounds(k: int, T: int, H: int) -> tuple[int, int]:
    """Start t_k = ceil(kT/H) and end t_{k+1} of push phase k."""
    return -((-k * T) // H), -((-(k + 1) * T) // H)


def softplus(z, beta):
    return F.softplus(z, beta=beta, threshold=60.0)


def relax(a):
    """Smooth surrogate z~ = softmax(a) over the last axis (Eq. 5)."""
    e = torch.exp(a - a.max(dim=-1, keepdim=True).values)
    return e / e.sum(dim=-1, keepdim=True)


def discrete_plan(theta: np.ndarray, H: int) -> np.ndarray:
    """Gamma(a_k) = index of the largest logit per push, lowest index on ties
    (Eq. 5 and its footnote).  theta [N][6H] -> modes [N][H] int32."""
    a = np.asarray(theta).reshape(theta.shape[0], H, 6)[:, :, :4]
    return np.argmax(a, axis=2).astype(np.int32)  # argmax returns the first max


def discrete_particles(theta: np.ndarray, H: int) -> np.ndarray:
    """The discrete plans Gamma of theta [N][6H] as particles: each push's logits
    become 40 e_Gamma - 20 (softmax weight of the chosen side 1 - O(e^-40)),
    offsets and depths kept."""
    th = np.array(theta, dtype=np.float64, copy=True)
    modes = discrete_plan(th, H)
    for k in range(H):
        th[:, 6 * k:6 * k + 4] = -20.0
        th[np.arange(th.shape[0]), 6 * k + modes[:, k]] = 20.0
    return th


def block_inertia(half, mass):
    return mass * (2.0 * half) ** 2 / 6.0


def _t(v, n):
    return torch.full((n,), float(v), dtype=DT)


def rollout(scene: dict, w: dict, theta: torch.Tensor, vel0=None, record=False, detach_phases=False):
    """Roll every particle forward and evaluate its cost.

    Each push phase k runs once per side s from the same start state S_k
    (the sub-rollouts X_s, one virtual pusher each); the next phase starts
    from their z~_k-weighted mixture S_{k+1} = sum_s z~_{k,s} X_s(t_{k+1}).

    theta: [N][6H] float64 tensor (may require grad).
    vel0:  optional [B][3] initial (vx, vy, omega), used only by physics pins.
    Returns dict(cost [N], P list of (x, y), phiT) and, with ``record``:
      tape    [T][6B][N][4]  pre-step state of every side sub-rollout,
      ends    [H][6B][N][4]  sub-rollout states after the last step of a phase,
      blended [H+1][6B][N]   the mixed phase-start states S_0..S_H,
    as detached numpy arrays (state order per block: x, y, phi, vx, vy, omega).

    detach_phases: each phase starts from a detached copy of S_k, so gradients
    stop at phase boundaries (the per-phase split of the appendix on exploding
    gradients); the result then also holds Pend, the block-0 (x, y) of every
    phase's end state S_{k+1} before detaching (k = 0..H-1), through which
    phase k's own gradient flows.  ``cost`` keeps its value either way.
    """
    N = theta.shape[0]
    H, B, T = int(scene["H"]), int(scene["B"]), int(scene["T"])
    dt = float(scene["dt"])
    gacc = float(scene["g"])
    beta = float(scene["sp_beta"])
    kp, kb = float(scene["k_push"]), float(scene["k_block"])
    delta = float(scene["standoff"])
    half = [float(v) for v in scene["half"]]
    mass = [float(v) for v in scene["mass"]]
    mu = [float(v) for v in scene["mu"]]
    inertia = [block_inertia(half[b], mass[b]) for b in range(B)]
    rho = [2.0 * half[b] * RHO_SQUARE for b in range(B)]
    ev = [max(float(scene["eps_v_scale"]) * dt * mu[b] * gacc, EPS_V_FLOOR) for b in range(B)]
    ew = [ev[b] * mass[b] * rho[b] / inertia[b] for b in range(B)]
    eps_r2 = float(scene["eps_r"]) ** 2

    # S[b] = [x, y, phi, vx, vy, omega], each [N]
    S = []
    for b in range(B):
        v0 = (0.0, 0.0, 0.0) if vel0 is None else vel0[b]
        S.append([_t(scene["pose0"][b][0], N), _t(scene["pose0"][b][1], N),
                  _t(scene["pose0"][b][2], N), _t(v0[0], N), _t(v0[1], N), _t(v0[2], N)])

    tape = ends = blended = None
    if record:
        tape = np.empty((T, 6 * B, N, 4))
        ends = np.empty((H, 6 * B, N, 4))
        blended = np.empty((H + 1, 6 * B, N))

    def snap_sides(dst, X):
        for b in range(B):
            for c in range(6):
                dst[6 * b + c] = X[b][c].detach().numpy()

    nx, ny = NORMALS[:, 0], NORMALS[:, 1]
    tx, ty = TANGENTS[:, 0], TANGENTS[:, 1]
    P = []
    Pend = []
    for k in range(H):
        tk, tk1 = phase_bounds(k, T, H)
        if detach_phases:
            S = [[c.detach() for c in blk] for blk in S]
        if record:
            for b in range(B):
                for c in range(6):
                    blended[k, 6 * b + c] = S[b][c].detach().numpy()
        Ax, Ay, Aph = S[0][0][:, None], S[0][1][:, None], S[0][2][:, None]
        P.append((S[0][0], S[0][1]))
        zt = relax(theta[:, 6 * k:6 * k + 4])                 # [N,4]
        o = theta[:, 6 * k + 4:6 * k + 5]                      # [N,1]
        Dk = theta[:, 6 * k + 5:6 * k + 6]                     # [N,1]
        cA, sA = torch.cos(Aph), torch.sin(Aph)
        # side sub-rollouts: every state component becomes [N,4]
        X = [[S[b][c][:, None].expand(N, 4) for c in range(6)] for b in range(B)]
        for t in range(tk, tk1):
            if record:
                snap_sides(tape[t], X)
            tau = (t - tk + 1) / (tk1 - tk)
            sig = 10 * tau ** 3 - 15 * tau ** 4 + 6 * tau ** 5
            px = [X[b][0] for b in range(B)]
            py = [X[b][1] for b in range(B)]
            ph = [X[b][2] for b in range(B)]
            vx = [X[b][3] for b in range(B)]
            vy = [X[b][4] for b in range(B)]
            om = [X[b][5] for b in range(B)]
            Fx, Fy, Tq = [None] * B, [None] * B, [None] * B

            # ground friction (regularised Coulomb), every block
            for b in range(B):
                c = mu[b] * mass[b] * gacc
                spd = torch.sqrt(vx[b] ** 2 + vy[b] ** 2 + ev[b] ** 2)
                Fx[b] = -c * vx[b] / spd
                Fy[b] = -c * vy[b] / spd
                Tq[b] = -c * rho[b] * om[b] / torch.sqrt(om[b] ** 2 + ew[b] ** 2)

            # block-block penalty contact, inscribed-disk proxy, central force
            for b in range(B):
                for c in range(b + 1, B):
                    dx, dy = px[b] - px[c], py[b] - py[c]
                    r = torch.sqrt(dx * dx + dy * dy + eps_r2)
                    f = kb * softplus(half[b] + half[c] - r, beta)
                    Fx[b] = Fx[b] + f * dx / r
                    Fy[b] = Fy[b] + f * dy / r
                    Fx[c] = Fx[c] - f * dx / r
                    Fy[c] = Fy[c] - f * dy / r

            # the virtual pusher of side s acts on block 0 in sub-rollout s
            depth = half[0] + delta - Dk * sig                 # [N,1]
            qx = depth * nx + o * tx                           # anchor frame
            qy = depth * ny + o * ty
            psx = Ax + cA * qx - sA * qy                       # world
            psy = Ay + sA * qx + cA * qy
            relx, rely = psx - px[0], psy - py[0]
            c0, s0 = torch.cos(ph[0]), torch.sin(ph[0])
            lx = c0 * relx + s0 * rely                         # R(phi0)^T rel
            ly = -s0 * relx + c0 * rely
            pen = half[0] - (nx * lx + ny * ly)
            fs = kp * softplus(pen, beta)
            Fsx = -fs * (c0 * nx - s0 * ny)                    # -f R(phi0) n_s
            Fsy = -fs * (s0 * nx + c0 * ny)
            Fx[0] = Fx[0] + Fsx
            Fy[0] = Fy[0] + Fsy
            Tq[0] = Tq[0] + relx * Fsy - rely * Fsx

            # semi-implicit Euler: velocities first, positions with the new velocities
            for b in range(B):
                nvx = vx[b] + dt * Fx[b] / mass[b]
                nvy = vy[b] + dt * Fy[b] / mass[b]
                nom = om[b] + dt * Tq[b] / inertia[b]
                X[b] = [px[b] + dt * nvx, py[b] + dt * nvy, ph[b] + dt * nom, nvx, nvy, nom]
        if record:
            snap_sides(ends[k], X)
        # mixture of the side outcomes, weighted by the relaxed action z~_k
        S = [[(zt * X[b][c]).sum(dim=1) for c in range(6)] for b in range(B)]
        Pend.append((S[0][0], S[0][1]))
    if record:
        for b in range(B):
            for c in range(6):
                blended[H, 6 * b + c] = S[b][c].detach().numpy()
    P.append((S[0][0], S[0][1]))

    cost = total_cost(scene, w, theta, P, S[0][2])
    out = dict(cost=cost, P=P, phiT=S[0][2], Pend=Pend)
    if record:
        out.update(tape=tape, ends=ends, blended=blended)
    return out


def _relu(x):
    return torch.clamp(x, min=0.0)


def total_cost(scene, w, theta, P, phiT):
    """C = b_t L_target + b_r L_rot + b_tr L_traj + b_b L_bound (Appendix E-B)."""
    H = int(scene["H"])
    gx, gy, gphi = (float(v) for v in scene["goal"])
    tol = float(scene["goal_tol"])
    PHx, PHy = P[H]
    L_target = _relu(torch.abs(PHx - gx) - tol) ** 2 + _relu(torch.abs(PHy - gy) - tol) ** 2
    L_rot = 1.0 - torch.cos(phiT - gphi)
    ea2 = float(w["traj_eps"]) ** 2

    def mh(p, q):
        return torch.sqrt((p[0] - q[0]) ** 2 + ea2) + torch.sqrt((p[1] - q[1]) ** 2 + ea2)

    L_traj = torch.zeros_like(PHx)
    for k in range(1, H + 1):
        L_traj = L_traj + mh(P[k - 1], P[k]) + mh(P[k], P[H]) - mh(P[k - 1], P[H])
    return (float(w["target"]) * L_target + float(w["rot"]) * L_rot
            + float(w["traj"]) * L_traj + float(w["bound"]) * bound_term(theta, w, H))


def bound_term(theta, w, H):
    """L_bound = sum_k relu(|o_k|-o_max)^2 + relu(-D_k)^2 + relu(D_k-D_max)^2
    (Appendix E-B): keeps each push's offset on its face and its depth in
    range.  theta [N][d] tensor; a closed form in the plan, no rollout."""
    L_bound = torch.zeros(theta.shape[0], dtype=theta.dtype)
    for k in range(H):
        o, Dk = theta[:, 6 * k + 4], theta[:, 6 * k + 5]
        L_bound = (L_bound + _relu(torch.abs(o) - float(w["o_max"])) ** 2
                   + _relu(-Dk) ** 2 + _relu(Dk - float(w["d_max"])) ** 2)
    return L_bound


def bound_term_push(theta, w, k):
    """Push k's share of L_bound: relu(|o_k|-o_max)^2 + relu(-D_k)^2 + relu(D_k-D_max)^2."""
    o, Dk = theta[:, 6 * k + 4], theta[:, 6 * k + 5]
    return (_relu(torch.abs(o) - float(w["o_max"])) ** 2 + _relu(-Dk) ** 2
            + _relu(Dk - float(w["d_max"])) ** 2)


def phase_costs(scene, w, theta, frozen=None):
    """Per-phase costs C_0..C_{H-1} whose sum is the cost C -- the split the
    appendix on exploding gradients proposes for costs that are sums of
    per-action terms, so that each action's parameters follow their own term
    and no gradient crosses a phase boundary.

    Terms go to the phase whose end state they read: push k's bound term to
    phase k; L_traj's term j (MH(P_{j-1},P_j) + MH(P_j,P_H) - MH(P_{j-1},P_H),
    j = 1..H) to phase j-1, whose end is P_j; L_target and L_rot, which read
    the final state, to the last phase.  Inside C_k every position another
    phase produces -- its start P_k and, for k < H-1, the final P_H -- is a
    constant, and the rollout restarts each phase from a detached state, so
    dC_k/dtheta reaches theta_k only, through phase k's own trajectory.

    frozen: optional (starts, final) from a previous call's ``frozen`` to hold
    in place of this theta's own (the constants of a finite-difference check).
    Returns dict(costs: list of H tensors [N], cost [N] (the rollout's C),
    frozen: ([(x, y)] * H starts, (x, y) final) as numpy)."""
    H = int(scene["H"])
    out = rollout(scene, w, theta, detach_phases=True)
    Pend, P = out["Pend"], out["P"]
    if frozen is None:
        starts = [(x.detach(), y.detach()) for x, y in P[:H]]
        final = (Pend[H - 1][0].detach(), Pend[H - 1][1].detach())
    else:
        starts = [(torch.as_tensor(x), torch.as_tensor(y)) for x, y in frozen[0]]
        final = tuple(torch.as_tensor(v) for v in frozen[1])
    ea2 = float(w["traj_eps"]) ** 2

    def mh(p, q):
        return torch.sqrt((p[0] - q[0]) ** 2 + ea2) + torch.sqrt((p[1] - q[1]) ** 2 + ea2)

    gx, gy, gphi = (float(v) for v in scene["goal"])
    tol = float(scene["goal_tol"])
    costs = []
    for k in range(H):
        end = Pend[k]
        c = float(w["bound"]) * bound_term_push(theta, w, k)
        if k < H - 1:
            c = c + float(w["traj"]) * (mh(starts[k], end) + mh(end, final) - mh(starts[k], final))
        else:
            c = c + float(w["traj"]) * (mh(starts[k], end) + mh(end, end) - mh(starts[k], end))
            c = c + float(w["target"]) * (_relu(torch.abs(end[0] - gx) - tol) ** 2
                                          + _relu(torch.abs(end[1] - gy) - tol) ** 2)
            c = c + float(w["rot"]) * (1.0 - torch.cos(out["phiT"] - gphi))
        costs.append(c)
    frz = ([(x.numpy(), y.numpy()) for x, y in starts], (final[0].numpy(), final[1].numpy()))
    return dict(costs=costs, cost=out["cost"].detach(), frozen=frz)


def per_phase_cost_and_grad(scene, w, theta, cost_bar=None):
    """(C [N], cost_bar * sum_k dC_k/dtheta [N][d]): the gradient of the
    per-phase split (``phase_costs``), block k of which is dC_k/dtheta_k."""
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    r = phase_costs(scene, w, th)
    c = torch.stack(r["costs"]).sum(dim=0)
    cb = torch.ones_like(c) if cost_bar is None else torch.as_tensor(np.asarray(cost_bar, dtype=np.float64))
    (g,) = torch.autograd.grad(c, th, grad_outputs=cb)
    return c.detach().numpy(), g.numpy()


def cost_np(scene, w, theta, **kw):
    """Cost [N] of particles theta [N][d] (numpy in, numpy out)."""
    with torch.no_grad():
        return rollout(scene, w, torch.as_tensor(np.asarray(theta, dtype=np.float64)), **kw)["cost"].numpy()


def readout(scene, w, theta):
    """Plan read-out: (modes [N][H], cost of executing each discrete plan [N])."""
    H = int(scene["H"])
    return discrete_plan(theta, H), cost_np(scene, w, discrete_particles(theta, H))


def cost_and_grad(scene, w, theta, cost_bar=None):
    """(C [N], cost_bar * dC/dtheta [N][d]) by reverse-mode autodiff through the
    whole rollout (Section III-B)."""
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64)).clone().requires_grad_(True)
    c = rollout(scene, w, th)["cost"]
    cb = torch.ones_like(c) if cost_bar is None else torch.as_tensor(np.asarray(cost_bar, dtype=np.float64))
    (g,) = torch.autograd.grad(c, th, grad_outputs=cb)
    return c.detach().numpy(), g.numpy()


def record(scene, w, theta, **kw):
    """Cost [N] and the recorded trajectories (tape, ends, blended)."""
    with torch.no_grad():
        out = rollout(scene, w, torch.as_tensor(np.asarray(theta, dtype=np.float64)), record=True, **kw)
    return out["cost"].numpy(), out["tape"], out["ends"], out["blended"]

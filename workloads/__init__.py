"""Seeded synthetic workloads for the block-pushing planner.

This module holds *inputs only*: the configuration sizes, the default scene
and cost constants, and seeded samplers for scenes and initial particles.  It
contains none of the method's arithmetic (no dynamics, no cost, no kernel), so
both the FP64 oracle and the GPU path may draw their inputs from it.

The paper's block-pushing scenes (Section V-A, Appendix E) are not published,
so these samplers stand in for them: a square block at the origin, a goal
pose at random bearing, and optional obstacle blocks placed without initial
overlap.  Every random draw comes from ``numpy.random.default_rng([cfg_id,
problem_id, stream])`` and every floating-point input is rounded to FP32 once,
so both sides start from bit-identical values.

Particle layout on the host is particle-major ``[N][d]`` with, for push k,
``theta[6k:6k+4]`` = side logits a_k (N, E, S, W), ``theta[6k+4]`` = contact
offset o_k along the face (m) and ``theta[6k+5]`` = push distance D_k (m).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

M_MODES = 4          # push sides North, East, South, West
PARAMS_PER_PUSH = 6  # 4 logits + offset + distance
MAX_BLOCKS = 4
MAX_PUSHES = 8

# RNG stream ids: rng = default_rng([cfg_id, problem_id, stream])
STREAM_SCENE = 0
STREAM_PARTICLES = 1
STREAM_SURROGATE = 2
STREAM_SIZES = 3


def f32(x):
    """Round to FP32 once (returned as float64 holding an FP32 value)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# Default model constants (the scene's physical parameters and cost weights).
# --------------------------------------------------------------------------
DEFAULT_SCENE_CONSTANTS = dict(
    k_push=2000.0,      # N/m, pusher penalty stiffness
    k_block=2000.0,     # N/m, block-block penalty stiffness
    sp_beta=1000.0,     # 1/m, softplus sharpness of the penalty
    standoff=0.005,     # m, pusher starts this far outside the face
    g=9.81,             # m/s^2
    eps_v_scale=2.0,    # friction regulariser eps_v = eps_v_scale*dt*mu*g
    eps_r=1e-4,         # m, regulariser of the block-block centre distance
)
DEFAULT_BLOCK = dict(half=0.05, mass=1.0, mu=0.5)
DEFAULT_COST = dict(target=1000.0, rot=0.0, traj=10.0, bound=1000.0,
                    o_max=0.05, d_max=0.3, traj_eps=1e-3)
DEFAULT_GOAL_TOL = 0.02
DEFAULT_ADAM = dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)


@dataclass
class Config:
    cfg_id: int
    name: str
    B: int
    H: int
    T: int
    dt: float
    N: int
    iters: int
    ckpt_every: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return PARAMS_PER_PUSH * self.H


# The five workloads.  cfg4's problems draw (N, H, B) per problem (see
# ``batched_problem_sizes``); the fields here are its common T and dt.
CONFIGS = {
    1: Config(1, "plain-fp64-cpu", B=1, H=2, T=50, dt=0.01, N=32, iters=100),
    2: Config(2, "plain-fp32-gpu", B=3, H=3, T=200, dt=0.005, N=1024, iters=200),
    3: Config(3, "differentiation", B=1, H=5, T=1000, dt=0.001, N=4096, iters=1,
              ckpt_every=32),
    4: Config(4, "batched", B=0, H=0, T=200, dt=0.005, N=0, iters=200,
              extra=dict(n_problems=64, N_range=(64, 2048), H_range=(2, 5),
                         B_range=(1, 4))),
    5: Config(5, "surrogate", B=3, H=5, T=200, dt=0.005, N=16384, iters=300,
              extra=dict(surrogate_frac=0.8, width=256, scene_enc=24,
                         n_train=1_000_000)),
}


def rng_for(cfg_id: int, problem_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(cfg_id), int(problem_id), int(stream)])


def make_scene(cfg_id: int, problem_id: int, B: int, H: int, T: int, dt: float,
               **overrides) -> dict:
    """Seeded scene: block 0 at the origin (phi=0), goal at radius U[0.1,0.3] m,
    bearing U[-pi,pi), heading U[-pi/4,pi/4]; blocks 1..B-1 uniformly in
    [-0.35,0.35]^2 at random heading, rejection-sampled so that every pair of
    centres is at least h_b + h_c + 0.01 m apart."""
    if not (1 <= B <= MAX_BLOCKS):
        raise ValueError("B must be in [1, 4]")
    rng = rng_for(cfg_id, problem_id, STREAM_SCENE)
    r = rng.uniform(0.1, 0.3)
    bearing = rng.uniform(-math.pi, math.pi)
    gphi = rng.uniform(-math.pi / 4, math.pi / 4)
    goal = [r * math.cos(bearing), r * math.sin(bearing), gphi]
    half = [DEFAULT_BLOCK["half"]] * B
    poses = [[0.0, 0.0, 0.0]]
    for b in range(1, B):
        for _ in range(10000):
            x, y = rng.uniform(-0.35, 0.35, size=2)
            ok = all(math.hypot(x - p[0], y - p[1]) >= half[b] + half[i] + 0.01
                     for i, p in enumerate(poses))
            if ok:
                break
        else:  # pragma: no cover - the box is large enough for 4 blocks
            raise RuntimeError("scene rejection sampling failed")
        poses.append([x, y, rng.uniform(-math.pi, math.pi)])
    scene = dict(
        H=int(H), M=M_MODES, B=int(B), T=int(T), dt=float(f32(dt)),
        half=[float(f32(h)) for h in half],
        mass=[float(f32(DEFAULT_BLOCK["mass"]))] * B,
        mu=[float(f32(DEFAULT_BLOCK["mu"]))] * B,
        pose0=[[float(v) for v in f32(p)] for p in poses],
        goal=[float(v) for v in f32(goal)],
        goal_tol=float(f32(DEFAULT_GOAL_TOL)),
    )
    for k, v in DEFAULT_SCENE_CONSTANTS.items():
        scene[k] = float(f32(v))
    for k, v in overrides.items():
        scene[k] = v
    return scene


def cost_weights(**overrides) -> dict:
    w = {k: float(f32(v)) for k, v in DEFAULT_COST.items()}
    w.update(overrides)
    return w


def make_particles(cfg_id: int, problem_id: int, N: int, H: int) -> np.ndarray:
    """Initial particles [N][6H]: logits ~ N(0,1), offset ~ U[-0.04,0.04] m,
    distance ~ U[0,0.2] m, rounded to FP32 (returned as float64)."""
    rng = rng_for(cfg_id, problem_id, STREAM_PARTICLES)
    th = np.empty((N, PARAMS_PER_PUSH * H), dtype=np.float64)
    for k in range(H):
        th[:, 6 * k:6 * k + 4] = rng.standard_normal((N, 4))
        th[:, 6 * k + 4] = rng.uniform(-0.04, 0.04, size=N)
        th[:, 6 * k + 5] = rng.uniform(0.0, 0.2, size=N)
    return f32(th)


def batched_problem_sizes(cfg_id: int = 4, n_problems: int = 64,
                          N_range=(64, 2048), H_range=(2, 5), B_range=(1, 4)):
    """Per-problem (N, H, B) drawn uniformly over the inclusive integer ranges."""
    rng = rng_for(cfg_id, 0, STREAM_SIZES)
    N = rng.integers(N_range[0], N_range[1] + 1, size=n_problems)
    H = rng.integers(H_range[0], H_range[1] + 1, size=n_problems)
    B = rng.integers(B_range[0], B_range[1] + 1, size=n_problems)
    return [(int(n), int(h), int(b)) for n, h, b in zip(N, H, B)]


def config_problem(cfg_id: int, problem_id: int = 0):
    """(scene, cost weights, initial particles) of a single-problem config."""
    c = CONFIGS[cfg_id]
    scene = make_scene(cfg_id, problem_id, c.B, c.H, c.T, c.dt)
    return scene, cost_weights(), make_particles(cfg_id, problem_id, c.N, c.H)


def batched_problems(cfg_id: int = 4):
    """List of (scene, cost weights, initial particles) for the batched config."""
    c = CONFIGS[cfg_id]
    out = []
    sizes = batched_problem_sizes(cfg_id, c.extra["n_problems"], c.extra["N_range"],
                                  c.extra["H_range"], c.extra["B_range"])
    for p, (N, H, B) in enumerate(sizes):
        out.append((make_scene(cfg_id, p, B, H, c.T, c.dt), cost_weights(),
                    make_particles(cfg_id, p, N, H)))
    return out


# --------------------------------------------------------------------------
# Surrogate inputs: scene encoding, random scenes and plans, initial weights.
# --------------------------------------------------------------------------
SCENE_ENC = 24  # 4 block slots x (x, y, cos phi, sin phi, present) + goal (x, y, cos, sin)


def scene_encoding(scene: dict) -> np.ndarray:
    """Fixed 24-float description of a scene: for block slots 0..3 (x, y,
    cos phi, sin phi, present) -- absent slots are zero -- then the goal's
    (x, y, cos phi, sin phi).  Rounded to FP32."""
    enc = np.zeros(SCENE_ENC)
    for b in range(MAX_BLOCKS):
        if b < scene["B"]:
            x, y, ph = scene["pose0"][b]
            enc[5 * b:5 * b + 5] = [x, y, math.cos(ph), math.sin(ph), 1.0]
    gx, gy, gph = scene["goal"]
    enc[20:24] = [gx, gy, math.cos(gph), math.sin(gph)]
    return f32(enc)


def surrogate_dataset_scenes(n_scenes: int, B: int = 3, H: int = 5, T: int = 200, dt: float = 0.005,
                             cfg_id: int = 5):
    """Training scenes of the surrogate: the config's scene sampler over problem
    ids 1000.. (disjoint from the evaluation scene, problem 0)."""
    return [make_scene(cfg_id, 1000 + p, B, H, T, dt) for p in range(n_scenes)]


def surrogate_dataset_particles(n_scenes: int, per_scene: int, H: int = 5, cfg_id: int = 5):
    """Plans of the training set: the particle sampler, per training scene."""
    return [make_particles(cfg_id, 1000 + p, per_scene, H) for p in range(n_scenes)]


def mlp_init(n_in: int, width: int = 256, seed: int = 0) -> dict:
    """He-uniform initial weights of the surrogate network, float64 holding FP32
    values; mu / inv_sigma start as the identity standardisation."""
    rng = rng_for(5, 0, STREAM_SURROGATE + 10 + seed)

    def u(shape, fan_in):
        lim = math.sqrt(6.0 / fan_in)
        return f32(rng.uniform(-lim, lim, size=shape))

    return dict(mu=np.zeros(n_in), inv_sigma=np.ones(n_in),
                W1=u((width, n_in), n_in), b1=np.zeros(width),
                W2=u((width, width), width), b2=np.zeros(width),
                w3=f32(u((width,), width) * 0.1), b3=np.zeros(1))


def surrogate_training_plans(p: int, per: int, H: int = 5, cfg_id: int = 5) -> np.ndarray:
    """Random plans of training scene p [per][6H]: the first half from the
    particle sampler, the second half wider (logits ~ N(0, 1.3^2), offsets
    U[-0.05, 0.05] m, depths U[0, 0.3] m: the whole in-bounds box), so the
    network also sees plans the solver moves to.  Rounded to FP32."""
    rng = rng_for(cfg_id, 1000 + p, STREAM_SURROGATE)
    th = make_particles(cfg_id, 1000 + p, per, H)
    half = per // 2
    for k in range(H):
        th[half:, 6 * k:6 * k + 4] = rng.normal(0.0, 1.3, (per - half, 4))
        th[half:, 6 * k + 4] = rng.uniform(-0.05, 0.05, per - half)
        th[half:, 6 * k + 5] = rng.uniform(0.0, 0.3, per - half)
    return f32(th)


# Training recipe of the surrogate for the N=16384 workload: 2^20 labelled
# rollouts = random plans on 128 scenes x 2048, then 2 on-policy rounds of the
# surrogate solver on 64 scenes x 2048 particles labelled at iterations 80,
# 160 and 240 (3 x 131072 rows per round); Adam steps on minibatches of 8192
# after the random phase and after each round.
# A plan counts as a solution when executing its discrete plan costs less than
# this: with the default weights, about 2 cm past the goal's dead zone on one
# axis (1000 * 0.022^2 = 0.48) on a near-monotone path.
SOLUTION_COST = 0.5

SURROGATE_RECIPE = dict(random_scenes=128, per=2048, rounds=2, round_scenes=64, round_iters=240,
                        snapshot_every=80, steps=4000, round_steps=2000, batch=8192, lr=1e-3, seed=0)

"""Training of the learned cost surrogate on the GPU (orchestration only).

Every step runs in libstamp's kernels: labelling plans with the simulator
(stamp_mlp_label), standardisation (stamp_mlp_standardize), Adam steps of the
network on the BF16 matrix cores (stamp_mlp_train_step), and the on-policy
rounds, which run the surrogate solver (stamp_solve_surrogate) on training
scenes and label the plans it visits, so that the network learns the region
the solver actually drives the particles into.  This module allocates the
dataset, draws minibatch indices from the caller's seeded generator and
sequences the calls.

The network predicts the rollout part of the cost (Appendix E-B without the
bound term); the solver adds the bound term exactly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import Context, CostW, Scene, make_cfg, pack_mlp


class Dataset:
    """Labelled rollouts resident in HBM: inputs x [capacity][n_in], rollout
    costs c [capacity]; rows [0, n) are filled."""

    def __init__(self, ctx: Context, capacity: int, n_in: int):
        self.ctx, self.n_in, self.n = ctx, n_in, 0
        self.x = torch.empty((capacity, n_in), dtype=torch.float32, device=ctx.device)
        self.c = torch.empty(capacity, dtype=torch.float32, device=ctx.device)

    @property
    def capacity(self) -> int:
        return self.x.shape[0]

    def label(self, scene: Scene, w: CostW, theta: torch.Tensor, enc: torch.Tensor, status=None):
        """Roll theta [d][N] through the simulator and append its rows."""
        N = theta.shape[1]
        if self.n + N > self.capacity:
            raise ValueError("dataset full (%d + %d > %d)" % (self.n, N, self.capacity))
        self.ctx.mlp_label(scene, w, theta, self.n_in, enc, x=self.x[self.n:self.n + N],
                           cost=self.c[self.n:self.n + N], status=status)
        self.n += N


@dataclass
class Network:
    """FP32 master parameters and their BF16 working copies."""
    params: torch.Tensor
    wbf16: torch.Tensor
    n_in: int

    @classmethod
    def create(cls, ctx: Context, init: dict, n_in: int) -> "Network":
        P = torch.as_tensor(pack_mlp(init), device=ctx.device)
        Wb = ctx.mlp_weights()
        ctx.mlp_prepare(P, Wb)
        return cls(P, Wb, n_in)


@dataclass
class TrainLog:
    steps: int = 0
    losses: list = field(default_factory=list)  # (step, loss of the minibatch before the step)


def fit(ctx: Context, net: Network, ds: Dataset, steps: int, gen: torch.Generator, batch: int = 8192,
        lr: float = 1e-3, lr_min: float = 2e-5, log_every: int = 500, log: TrainLog | None = None) -> TrainLog:
    """Adam on the mean squared error of y against log(1 + c) over random
    minibatches of the dataset, cosine learning-rate decay from lr to lr_min.
    The moments start from zero on every call."""
    log = log or TrainLog()
    m = torch.zeros_like(net.params)
    v = torch.zeros_like(net.params)
    status = ctx.status_word()
    ws = ctx._bytes(ctx.mlp_train_workspace_bytes(batch))
    X, C = ds.x[:ds.n], ds.c[:ds.n]
    # steps go to the library in chunks (one call launches a chunk's kernels
    # back to back); every step's loss is kept, the logged ones read per chunk
    chunk = 256
    losses = torch.zeros(chunk, dtype=torch.float32, device=ctx.device)
    for c0 in range(1, steps + 1, chunk):
        n = min(chunk, steps + 1 - c0)
        idx = torch.randint(0, ds.n, (n, batch), generator=gen, device=ctx.device, dtype=torch.int32)
        lrs = [lr_min + (lr - lr_min) * 0.5 * (1.0 + math.cos(math.pi * (t - 1) / steps)) for t in range(c0, c0 + n)]
        ctx.mlp_train_steps(net.params, net.wbf16, m, v, X, C, c0 - 1, idx, lrs, loss=losses, status=status,
                            workspace=ws)
        logged = [t for t in range(c0, c0 + n) if log_every and (t == 1 or t % log_every == 0 or t == steps)]
        if logged:
            host = losses[:n].cpu()
            for t in logged:
                log.losses.append((log.steps + t, float(host[t - c0])))
    log.steps += steps
    if int(status.item()) != 0:
        raise RuntimeError("training reported status %#x" % int(status.item()))
    return log


def on_policy_round(ctx: Context, net: Network, ds: Dataset, problems, iters: int, snapshot_every: int,
                    lr: float = 1e-3):
    """Run the surrogate solver on training problems [(scene, w, theta0 [d][N],
    enc)] in one batched solve, labelling the particles every snapshot_every
    iterations with the simulator.  Returns the solver's last report."""
    scenes = [p[0] for p in problems]
    ws_ = [p[1] for p in problems]
    Ns = [p[2].shape[1] for p in problems]
    theta = torch.cat([p[2].reshape(-1) for p in problems]).contiguous()
    enc = torch.cat([p[3].reshape(-1) for p in problems]).contiguous()
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    cfg = make_cfg(snapshot_every, lr=lr)
    work = ctx._bytes(ctx.solve_workspace_bytes(scenes, Ns, cfg))
    rep = None
    for s in range(iters // snapshot_every):
        cfg = make_cfg(snapshot_every, t0=s * snapshot_every, lr=lr)
        _, rep = ctx.solve_surrogate(scenes, ws_, Ns, cfg, snapshot_every, net.params, net.wbf16, net.n_in, enc,
                                     theta, m, v, workspace=work)
        off = 0
        for (scene, w, th0, e), N in zip(problems, Ns):
            d = th0.shape[0]
            ds.label(scene, w, theta[off:off + d * N].view(d, N), e)
            off += d * N
    return rep


def train_recipe(ctx: Context, recipe: dict, problem, random_plans, prior_plans, init: dict, n_in: int,
                 gen: torch.Generator, progress=None):
    """The whole training procedure.

    recipe: random_scenes, per, rounds, round_scenes, round_iters,
      snapshot_every, steps, round_steps, batch, lr.
    problem(p) -> (Scene, CostW, enc [n_in - d] device tensor) of training scene p;
    random_plans(p, per) -> [d][per] device plans labelled in the random phase;
    prior_plans(p, per) -> [d][per] initial particles of an on-policy problem;
    init: initial network weights (dict of arrays).
    Returns (Network, Dataset, TrainLog, reports of the on-policy rounds)."""
    R = recipe
    per = R["per"]
    cap = R["random_scenes"] * per + R["rounds"] * R["round_scenes"] * per * (R["round_iters"] // R["snapshot_every"])
    ds = Dataset(ctx, cap, n_in)
    for p in range(R["random_scenes"]):
        sc, w, enc = problem(p)
        ds.label(sc, w, random_plans(p, per), enc)
    net = Network.create(ctx, init, n_in)
    ctx.mlp_standardize(net.params, ds.x[:ds.n], ds.c[:ds.n])
    ctx.mlp_prepare(net.params, net.wbf16)
    log = fit(ctx, net, ds, R["steps"], gen, R["batch"], R["lr"])
    if progress:
        progress("random phase: %d rows, loss %.4f -> %.4f" % (ds.n, log.losses[0][1], log.losses[-1][1]))
    reports = []
    for r in range(R["rounds"]):
        probs = []
        for q in range(R["round_scenes"]):
            p = r * R["round_scenes"] + q
            sc, w, enc = problem(p)
            probs.append((sc, w, prior_plans(p, per), enc))
        reports.append(on_policy_round(ctx, net, ds, probs, R["round_iters"], R["snapshot_every"], R["lr"]))
        fit(ctx, net, ds, R["round_steps"], gen, R["batch"], R["lr"], log=log)
        if progress:
            progress("on-policy round %d: %d rows, solver log-error %.3f, loss %.4f" %
                     (r, ds.n, reports[-1].log_err, log.losses[-1][1]))
    return net, ds, log, reports

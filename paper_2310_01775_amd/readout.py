"""Plan read-out of a solve (Algorithm 1's result): the discrete plan of each
particle, the cost of executing it, and how the solutions spread over plans
(the analogue of the paper's solution counts and plan histograms, Sec. V).

The plans and their costs come from stamp_plan_readout; this module only
counts them on the host.
"""
from __future__ import annotations

import numpy as np

SIDES = "NESW"  # side index 0..3 = north, east, south, west of block 0


def plan_names(modes) -> list[str]:
    """modes [H][N] (side index per push) -> one name per particle, e.g. "N-E-S"."""
    m = np.asarray(modes)
    return ["-".join(SIDES[int(s)] for s in m[:, i]) for i in range(m.shape[1])]


def solution_histogram(modes, cost, threshold: float) -> dict[str, int]:
    """Solutions = particles whose discrete plan costs less than `threshold`;
    returns {plan name: number of solutions}, largest first."""
    names = plan_names(modes)
    c = np.asarray(cost)
    counts: dict[str, int] = {}
    for n, ok in zip(names, c < threshold):
        if ok:
            counts[n] = counts.get(n, 0) + 1
    return dict(sorted(counts.items(), key=lambda kv: (-kv[1], kv[0])))


def report(ctx, scene, w, theta, threshold: float) -> dict:
    """Read out theta [d][N] on the GPU and summarise: particles, solutions,
    distinct plans among them, the histogram, and cost quantiles."""
    modes, cost = ctx.plan_readout(scene, w, theta)
    m = modes.cpu().numpy()
    c = cost.cpu().double().numpy()
    hist = solution_histogram(m, c, threshold)
    return {"particles": int(c.size), "solutions": int((c < threshold).sum()), "plans": len(hist),
            "histogram": hist, "cost_median": float(np.median(c)), "cost_p10": float(np.quantile(c, 0.1))}

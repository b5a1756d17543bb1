"""The oracle's own sensitivity: how far a 1e-7 relative perturbation of the
initial particles travels after 100 Adam-SVGD iterations (FP64 vs FP64).
This fixes the horizon on which any FP32 implementation can match the oracle."""
import numpy as np

import workloads as W
from oracle import svgd


def _spread(lr, iters):
    scene, w, th = W.config_problem(1)
    rng = np.random.default_rng(0)
    th2 = th * (1 + 1e-7 * rng.standard_normal(th.shape))
    a = svgd.solve(scene, w, th, iters, lr=lr)["theta"]
    b = svgd.solve(scene, w, th2, iters, lr=lr)["theta"]
    return np.abs(a - b).max()


def test_default_lr_is_well_conditioned_over_100_iterations():
    assert W.DEFAULT_ADAM["lr"] == 1e-3
    assert _spread(1e-3, 100) < 1e-5


def test_large_lr_is_chaotic_within_100_iterations():
    assert _spread(1e-2, 100) > 1e-3

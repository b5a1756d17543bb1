"""GPU solve (Algorithm 1, SVGD phase) against the FP64 oracle.

Parity bar on the particle states after 100 iterations at the default lr 1e-3
(the regime in which the FP64 oracle is itself well-conditioned; see the
conditioning test), each coordinate's error scaled by its largest magnitude
over the particle set.  The bar comes from the FP32 floor measured on this very
metric by tests/golden/fp32_floor.py: twelve FP32 evaluations of the oracle's
own arithmetic that differ only in rounding (IEEE float32; Gram-form distances;
one-ulp moves of the initial particles, of every gradient, of every
transcendental result, and all together) land at
  normwise 2.6e-7 .. 4.2e-7,  99.9th percentile 5.1e-6 .. 1.06e-5,
  worst coordinate 3.2e-5 .. 3.2e-4 (always particle 23 or 131: a sensitive
  contact state that amplifies any rounding difference),
so an FP32 result is held to normwise < 2e-6, 99.9th percentile < 2e-5 and
worst coordinate < 5e-4 (about 5x, 2x and 1.6x the largest of the twelve)."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import svgd

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gpu_solve(ctx, scene, w, th, iters, lr, ckpt=0):
    import paper_2310_01775_amd as S
    N, d = th.shape
    theta = S.soa(th)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    cfg = S.make_cfg(iters, lr=lr, ckpt_every=ckpt)
    modes = torch.empty(scene["H"] * N, dtype=torch.int32, device="cuda")
    st = ctx.status_word()
    cost = ctx.solve([S.make_scene(scene)], [S.make_cost(w)], [N], cfg, theta, m, v, modes_out=modes, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return S.aos(theta), cost.cpu().double().numpy(), modes.cpu().numpy().reshape(scene["H"], N).T


def _rel_err(got, ref):
    scale = np.abs(ref).max(axis=0, keepdims=True)
    return (np.abs(got - ref) / scale).max()


def _err_stats(got, ref):
    """Normwise relative error, and per-coordinate errors (each scaled by the
    coordinate's magnitude over the particle set): percentiles and the worst."""
    e = np.abs(got - ref) / np.abs(ref).max(axis=0, keepdims=True)
    return dict(norm=float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                p50=float(np.percentile(e, 50)), p99=float(np.percentile(e, 99)),
                p999=float(np.percentile(e, 99.9)), max=float(e.max()),
                worst_particle=int(np.unravel_index(e.argmax(), e.shape)[0]))


def test_cfg1_solve_100_iterations(ctx):
    scene, w, th = W.config_problem(1)
    got, cost, modes = _gpu_solve(ctx, scene, w, th, 100, 1e-3)
    ref = svgd.solve(scene, w, th, 100, lr=1e-3)
    err = _rel_err(got, ref["theta"])
    print("cfg1 100-iteration state error", err, flush=True)
    assert err < 1e-4
    assert np.allclose(cost, ref["cost"], rtol=1e-3, atol=1e-3)
    assert np.array_equal(modes, ref["modes"])


def test_cfg1_checkpointed_solve_equals_full_tape(ctx):
    scene, w, th = W.config_problem(1)
    a = _gpu_solve(ctx, scene, w, th, 10, 1e-3, ckpt=0)
    b = _gpu_solve(ctx, scene, w, th, 10, 1e-3, ckpt=8)
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("name", ["cfg2_solve_lr1e-3_it100", "cfg2_solve_lr1e-2_it10"])
def test_cfg2_solve_matches_stored_oracle(ctx, name):
    path = os.path.join(GOLDEN, name + ".npz")
    gold = np.load(path)
    scene, w, th = W.config_problem(int(gold["cfg"]))
    got, cost, modes = _gpu_solve(ctx, scene, w, th, int(gold["iters"]), float(gold["lr"]))
    st = _err_stats(got, gold["theta"])
    print(name, "state error", st, flush=True)
    # the FP32-floor bar of the module docstring
    assert st["norm"] < 2e-6 and st["p999"] < 2e-5 and st["max"] < 5e-4
    agree = (modes == gold["modes"]).mean()
    print("mode agreement", agree, flush=True)
    assert agree == 1.0

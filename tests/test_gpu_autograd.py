"""Checkpointed differentiation behind torch.autograd.Function on the long-
horizon workload: 1 block, 5 pushes (d=30), T=1000 steps of dt=0.001, N=4096,
checkpoints every 32 steps.  16 random particles are checked against the FP64
oracle's reverse-mode gradient, which is itself pinned to central finite
differences (eps = 1e-6, FP64) on the same particles."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import sim

pytestmark = pytest.mark.gpu


def _cfg3():
    import paper_2310_01775_amd as S
    scene, w, th = W.config_problem(3)
    return S, scene, w, th


def test_autograd_function_gradient_on_16_particles(ctx):
    S, scene, w, th = _cfg3()
    from paper_2310_01775_amd.autograd import rollout_cost, tape_bytes
    N = th.shape[0]
    sc, cw = S.make_scene(scene), S.make_cost(w)
    theta = S.soa(th).requires_grad_(True)
    cost = rollout_cost(theta, ctx, sc, cw, 32)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(N, 16, replace=False))
    wts = torch.zeros(N, device="cuda")
    wts[torch.as_tensor(pick, device="cuda")] = 1.0
    (cost * wts).sum().backward()
    torch.cuda.synchronize()
    g = S.aos(theta.grad)[pick]
    c_ref, g_ref = sim.cost_and_grad(scene, w, th[pick])
    assert np.allclose(cost.detach().cpu().double().numpy()[pick], c_ref, rtol=1e-4)
    scale = np.abs(g_ref).max(axis=1, keepdims=True)
    err = (np.abs(g - g_ref) / scale).max()
    print("cfg3 checkpointed gradient error / particle scale", err, flush=True)
    assert err < 1e-3
    # non-picked particles receive exactly zero gradient
    rest = np.setdiff1d(np.arange(N), pick)
    assert np.abs(S.aos(theta.grad)[rest]).max() == 0.0
    # memory kept between forward and backward: checkpoints vs the full tape
    full, ck = tape_bytes(sc, N, 0), tape_bytes(sc, N, 32)
    print("tape bytes: full %.1f MB, checkpointed %.1f MB (%.1fx less)" % (full / 1e6, ck / 1e6, full / ck),
          flush=True)
    assert full / ck > 10


def test_autograd_full_and_checkpointed_agree_bitwise(ctx):
    S, scene, w, th = _cfg3()
    from paper_2310_01775_amd.autograd import rollout_cost
    sc, cw = S.make_scene(scene), S.make_cost(w)
    x = S.soa(th[:256])
    grads = []
    for K in (0, 32):
        t = x.clone().requires_grad_(True)
        rollout_cost(t, ctx, sc, cw, K).sum().backward()
        grads.append(t.grad.clone())
    torch.cuda.synchronize()
    assert torch.equal(grads[0], grads[1])

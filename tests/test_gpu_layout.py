"""The two rollout lane layouts (one lane per block of a sub-rollout, or one
lane per sub-rollout holding all its blocks) give the same results bit for
bit: costs, tapes, gradients (full tape, checkpoints, per-phase split) and
whole solves, single and batched."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

SCENES = [("b1h2", 1, 2, 50, 33), ("b2h3", 2, 3, 60, 41), ("b3h3", 3, 3, 60, 37), ("b4h2", 4, 2, 40, 70),
          ("b3h5", 3, 5, 47, 5)]


@pytest.fixture
def layout_ctx(ctx):
    yield ctx
    ctx.set_rollout_layout(0)


def _run(ctx, S, layout, sc, cw, theta, N, ckpt, per_phase):
    ctx.set_rollout_layout(layout)
    tape = torch.zeros(ctx.tape_floats(sc, N, ckpt), dtype=torch.float32, device="cuda")
    cost = ctx.rollout_fwd(sc, cw, theta, tape=tape, ckpt_every=ckpt)
    cb = torch.linspace(-1.5, 2.0, N, device="cuda")
    grad = ctx.rollout_adj(sc, cw, theta, tape, ckpt_every=ckpt, cost_bar=cb, per_phase=per_phase)
    torch.cuda.synchronize()
    return cost, tape, grad


@pytest.mark.parametrize("ckpt,per_phase", [(0, False), (6, False), (0, True)])
@pytest.mark.parametrize("label,B,H,T,N", SCENES, ids=[s[0] for s in SCENES])
def test_layouts_agree_bit_for_bit(layout_ctx, label, B, H, T, N, ckpt, per_phase):
    import paper_2310_01775_amd as S
    ctx = layout_ctx
    print("case", label, ckpt, per_phase, flush=True)
    scene = W.make_scene(6, B * 10 + H, B, H, T, 0.005)
    w = W.cost_weights(rot=1.0)
    sc, cw = S.make_scene(scene), S.make_cost(w)
    theta = S.soa(W.make_particles(6, B, N, H))
    a = _run(ctx, S, S.LAYOUT_BLOCKS, sc, cw, theta, N, ckpt, per_phase)
    b = _run(ctx, S, S.LAYOUT_PACKED, sc, cw, theta, N, ckpt, per_phase)
    assert torch.equal(a[0], b[0]), "cost"
    assert torch.equal(a[1], b[1]), "tape"
    assert torch.equal(a[2], b[2]), "grad"
    assert torch.isfinite(a[2]).all()


def test_layouts_give_the_same_solves(layout_ctx):
    import paper_2310_01775_amd as S
    ctx = layout_ctx
    probs = []
    for pid, (N, B, H) in enumerate([(90, 3, 3), (33, 4, 2), (50, 2, 4), (17, 1, 3)]):
        probs.append((W.make_scene(8, pid, B, H, 60, 0.005), W.cost_weights(), W.make_particles(8, pid, N, H)))
    outs = []
    for layout in (S.LAYOUT_BLOCKS, S.LAYOUT_PACKED):
        ctx.set_rollout_layout(layout)
        for sub in (probs, probs[:1]):  # batched kernels, and the single-problem path
            flat = torch.cat([S.soa(th).reshape(-1) for _, _, th in sub]).contiguous()
            m, v = torch.zeros_like(flat), torch.zeros_like(flat)
            cost = ctx.solve([S.make_scene(s) for s, _, _ in sub], [S.make_cost(w) for _, w, _ in sub],
                             [th.shape[0] for _, _, th in sub], S.make_cfg(4, lr=1e-3, ckpt_every=5), flat, m, v)
            torch.cuda.synchronize()
            outs.append((flat.clone(), cost.clone()))
    assert torch.equal(outs[0][0], outs[2][0]) and torch.equal(outs[0][1], outs[2][1])
    assert torch.equal(outs[1][0], outs[3][0]) and torch.equal(outs[1][1], outs[3][1])


def test_layout_argument_is_checked(layout_ctx):
    import paper_2310_01775_amd as S
    with pytest.raises(S.StampError) as e:
        layout_ctx.set_rollout_layout(3)
    assert e.value.code == S.EINVAL

"""The SVGD direction under the structured pusher kernel (Appendix E-C),
through the C ABI, against the FP64 oracle.

Bars: phi within 2e-5 of each coordinate's scale (max over particles of the
oracle's |phi|), as for the plain FP32 step; the median-heuristic bandwidths
within 3e-6 relative (an exact order statistic of FP32 features); the solve
with the structured kernel equal to the per-call loop bit for bit and within
the solve's state bar of the oracle."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import structured as OS
from oracle import svgd

pytestmark = pytest.mark.gpu

PUSH, POSE = OS.LAYOUT_PUSH, OS.LAYOUT_POSE


def _err(got, ref):
    return (np.abs(got - ref) / np.maximum(np.abs(ref).max(axis=0, keepdims=True), 1e-30)).max()


def _inputs(seed, N, layout, K):
    rng = np.random.default_rng(seed)
    d = OS.dim(layout, K)
    th = rng.normal(0.0, 1.0, (N, d))
    a, _, p = OS.blocks(layout, K)
    for blk in a:
        th[:, blk] *= 2.0  # logits spread enough to make the softmax terms vary
    if p is not None:
        th[:, p] = rng.uniform(-math.pi, math.pi, (N, K))
    return W.f32(th), W.f32(rng.normal(0.0, 3.0, (N, d)))


def _spec_pair(S, layout, K, **kw):
    spec = OS.make_spec(layout, K, **kw)
    return spec, S.struct_kernel(layout, K, spec["alpha_g"], spec["alpha_z"], spec["alpha_p"], spec["h_g"],
                                 spec["h_z"], spec["kappa"])


@pytest.mark.parametrize("N,layout,K", [(1, PUSH, 2), (2, PUSH, 1), (37, PUSH, 3), (300, PUSH, 5), (513, POSE, 2),
                                        (1000, POSE, 8), (777, PUSH, 8), (64, POSE, 1)])
def test_structured_direction_matches_oracle(ctx, N, layout, K):
    import paper_2310_01775_amd as S
    print("case", N, layout, K, flush=True)
    th, g = _inputs(N * 10 + K, N, layout, K)
    spec, kern = _spec_pair(S, layout, K, alpha_g=0.8, alpha_z=1.3, alpha_p=0.6, kappa=1.5)
    h = torch.zeros(2, device="cuda")
    phi = ctx.svgd_step_structured(S.soa(th), S.soa(g), kern, h_out=h)
    torch.cuda.synchronize()
    hg, hz = (float(v) for v in h.cpu())
    ref_h = OS.bandwidths(th, spec)
    assert abs(hg - ref_h[0]) <= 3e-6 * ref_h[0] and abs(hz - ref_h[1]) <= 3e-6 * ref_h[1], (hg, hz, ref_h)
    ref = OS.phi(th, g, spec, hg, hz)  # the oracle at the step's own bandwidths
    err = _err(S.aos(phi), ref)
    print("structured phi err", err, flush=True)
    assert err < 2e-5


@pytest.mark.parametrize("layout", [PUSH, POSE])
def test_structured_fixed_bandwidths_and_weights(ctx, layout):
    import paper_2310_01775_amd as S
    N, K = 259, 3
    th, g = _inputs(7 + layout, N, layout, K)
    rng = np.random.default_rng(11)
    w = rng.uniform(0.0, 3.0, N)
    w = W.f32(w * N / w.sum())
    spec, kern = _spec_pair(S, layout, K, alpha_g=1.0, alpha_z=0.5, alpha_p=2.0, h_g=0.9, h_z=0.15, kappa=0.7)
    h = torch.zeros(2, device="cuda")
    phi = ctx.svgd_step_structured(S.soa(th), S.soa(g), kern, torch.tensor(w, dtype=torch.float32, device="cuda"), h_out=h)
    torch.cuda.synchronize()
    assert h.cpu().tolist() == pytest.approx([0.9, 0.15], rel=1e-7)
    err = _err(S.aos(phi), OS.phi(th, g, spec, 0.9, 0.15, w=w.astype(np.float64)))
    print("weighted structured phi err", err, flush=True)
    assert err < 2e-5


def test_structured_direction_at_full_size_on_sampled_rows(ctx):
    # 16384 particles of five actions (the large pushing workload's shape):
    # sampled rows against the oracle at the step's bandwidths
    import paper_2310_01775_amd as S
    scene, w, th = W.config_problem(5)
    th = W.f32(th)
    N, d = th.shape
    K = int(scene["H"])
    rng = np.random.default_rng(5)
    g = W.f32(rng.normal(0.0, 20.0, (N, d)))
    spec, kern = _spec_pair(S, PUSH, K)
    h = torch.zeros(2, device="cuda")
    phi = ctx.svgd_step_structured(S.soa(th), S.soa(g), kern, h_out=h)
    torch.cuda.synchronize()
    hg, hz = (float(v) for v in h.cpu())
    assert hg > 0 and hz > 0 and math.isfinite(hg) and math.isfinite(hz)
    rows = np.concatenate([[0, 1, N - 1], rng.choice(N, 13, replace=False)])
    ref = OS.phi(th.astype(np.float64), g.astype(np.float64), spec, hg, hz, rows=rows)
    got = S.aos(phi)[rows]
    scale = np.abs(ref).max(axis=0, keepdims=True)
    err = (np.abs(got - ref) / scale).max()
    print("full-size structured phi err (sampled rows)", err, flush=True)
    assert err < 2e-5


def test_structured_argument_errors(ctx):
    import paper_2310_01775_amd as S
    th, g = _inputs(3, 16, PUSH, 2)
    theta, grad = S.soa(th), S.soa(g)
    bad = [S.struct_kernel(PUSH, 3), S.struct_kernel(POSE, 2), S.struct_kernel(2, 2), S.struct_kernel(PUSH, 0),
           S.struct_kernel(PUSH, 2, alpha_g=-1.0), S.struct_kernel(PUSH, 2, kappa=float("nan")),
           S.struct_kernel(PUSH, 2, h_z=float("inf"))]
    for k in bad:
        with pytest.raises(S.StampError):
            ctx.svgd_step_structured(theta, grad, k)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.StampError):
        ctx.svgd_step_structured(theta, grad, S.struct_kernel(PUSH, 2), workspace=small)
    scene, w, th1 = W.config_problem(1)
    t1 = S.soa(th1)
    m, v = torch.zeros_like(t1), torch.zeros_like(t1)
    with pytest.raises(S.StampError):  # the solve's particles take the push layout
        ctx.solve([S.make_scene(scene)], [S.make_cost(w)], [th1.shape[0]],
                  S.make_cfg(2, kernel=S.struct_kernel(POSE, 1)), t1, m, v)


def test_structured_solve_equals_the_per_call_loop(ctx):
    import paper_2310_01775_amd as S
    sizes = [(90, 3, 3), (41, 2, 1)]
    probs = [(W.make_scene(64, p, B, H, 40, 0.005), W.cost_weights(rot=0.5), W.make_particles(64, p, N, H))
             for p, (N, H, B) in enumerate(sizes)]
    kern = S.struct_kernel(PUSH, 0, alpha_g=1.0, alpha_z=0.7)
    flat = torch.cat([S.soa(th).reshape(-1) for _, _, th in probs]).contiguous()
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    st = ctx.status_word()
    ctx.solve([S.make_scene(s) for s, _, _ in probs], [S.make_cost(c) for _, c, _ in probs],
              [th.shape[0] for _, _, th in probs], S.make_cfg(4, lr=1e-3, sgd_iters=1, kernel=kern), flat, m, v,
              status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    off = 0
    for scene, w, th in probs:
        sc, cw = S.make_scene(scene), S.make_cost(w)
        N, H = th.shape[0], int(scene["H"])
        kp = S.struct_kernel(PUSH, H, alpha_g=1.0, alpha_z=0.7)
        theta = S.soa(th)
        mm, vv = torch.zeros_like(theta), torch.zeros_like(theta)
        tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")
        minus = torch.full((N,), -1.0, device="cuda")
        for t in range(1, 6):
            ctx.rollout_fwd(sc, cw, theta, tape=tape)
            gr = ctx.rollout_adj(sc, cw, theta, tape, cost_bar=minus)
            phi = ctx.svgd_step_structured(theta, gr, kp) if t <= 4 else gr
            ctx.adam_step(theta, phi, mm, vv, t, lr=1e-3)
        torch.cuda.synchronize()
        n = theta.numel()
        assert torch.equal(flat[off:off + n].view_as(theta), theta)
        off += n


def test_structured_solve_matches_oracle(ctx):
    import paper_2310_01775_amd as S
    scene, w, th = W.config_problem(1)
    N = th.shape[0]
    theta = S.soa(th)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    kern = S.struct_kernel(PUSH, 0, alpha_g=1.0, alpha_z=1.0)
    ctx.solve([S.make_scene(scene)], [S.make_cost(w)], [N], S.make_cfg(20, lr=1e-3, kernel=kern), theta, m, v)
    torch.cuda.synchronize()
    ref = svgd.solve(scene, w, th, 20, lr=1e-3, kernel=OS.make_spec(PUSH, 0, alpha_g=1.0, alpha_z=1.0))
    got = S.aos(theta)
    err = (np.abs(got - ref["theta"]) / np.abs(ref["theta"]).max(axis=0, keepdims=True)).max()
    norm = np.linalg.norm(got - ref["theta"]) / np.linalg.norm(ref["theta"])
    print("structured solve state error: worst", err, "normwise", norm, flush=True)
    assert norm < 1e-4 and err < 1e-3


def test_structured_dsvgd_solve_equals_the_per_call_loop(ctx):
    """Importance weights (Eq. 4) with the structured kernel: the solve equals
    rollout, discrete read-out, weights and the weighted structured step."""
    import paper_2310_01775_amd as S
    scene = W.make_scene(66, 0, 2, 3, 40, 0.005)
    w = W.cost_weights(rot=0.5)
    th = W.make_particles(66, 0, 70, 3)
    sc, cw = S.make_scene(scene), S.make_cost(w)
    N, H = th.shape[0], int(scene["H"])
    flat = S.soa(th)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    st = ctx.status_word()
    ctx.solve([sc], [cw], [N], S.make_cfg(3, lr=1e-3, dsvgd=True, kernel=S.struct_kernel(PUSH, 0)), flat, m, v,
              status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    kp = S.struct_kernel(PUSH, H)
    theta = S.soa(th)
    mm, vv = torch.zeros_like(theta), torch.zeros_like(theta)
    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")
    minus = torch.full((N,), -1.0, device="cuda")
    for t in range(1, 4):
        c_rel = ctx.rollout_fwd(sc, cw, theta, tape=tape)
        gr = ctx.rollout_adj(sc, cw, theta, tape, cost_bar=minus)
        _, c_disc = ctx.plan_readout(sc, cw, theta)
        phi = ctx.svgd_step_structured(theta, gr, kp, weights=ctx.dsvgd_weights(c_rel, c_disc))
        ctx.adam_step(theta, phi, mm, vv, t, lr=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(flat, theta)

"""Batched, graph-captured solve of many problems of uneven N, H and B in one
call: it must reproduce each problem's own iteration bit for bit (the batched
kernels run the same device code over a work list), and the oracle to the FP32
tolerance."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import svgd

pytestmark = pytest.mark.gpu


def _problems(sizes, T, dt, seed):
    out = []
    for p, (N, H, B) in enumerate(sizes):
        out.append((W.make_scene(40 + seed, p, B, H, T, dt), W.cost_weights(rot=0.5),
                    W.make_particles(40 + seed, p, N, H)))
    return out


def _pack(S, probs):
    return torch.cat([S.soa(th).reshape(-1) for _, _, th in probs]).contiguous()


def _unpack(S, flat, probs):
    out, off = [], 0
    for _, _, th in probs:
        n = th.size
        out.append(flat[off:off + n].reshape(th.shape[1], th.shape[0]))
        off += n
    return out


def _per_problem_loop(ctx, S, scene, w, th, iters, lr):
    sc, cw = S.make_scene(scene), S.make_cost(w)
    N = th.shape[0]
    theta = S.soa(th)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")
    minus = torch.full((N,), -1.0, device="cuda")
    for t in range(1, iters + 1):
        ctx.rollout_fwd(sc, cw, theta, tape=tape)
        g = ctx.rollout_adj(sc, cw, theta, tape, cost_bar=minus)
        phi = ctx.svgd_step(theta, g)
        ctx.adam_step(theta, phi, m, v, t, lr=lr)
    cost = ctx.rollout_fwd(sc, cw, theta)
    return theta, cost


@pytest.mark.parametrize("autotune", [True, False])
def test_batched_solve_equals_per_problem_iterations(ctx, autotune):
    import paper_2310_01775_amd as S
    ctx.set_autotune(autotune)
    try:
        _check_batched_equals_loops(ctx, S)
    finally:
        ctx.set_autotune(True)


def _check_batched_equals_loops(ctx, S):
    # 1600 particles: above 2^20 pairs, so its median's all-pairs passes take
    # the Gram form in both paths (split form at d = 18); H = 6 and 8 (d = 36,
    # 48) take the FP32 matrix-core contraction, and 1500 particles at d = 48
    # its Gram-form median
    sizes = [(64, 2, 1), (200, 5, 4), (1, 3, 2), (97, 3, 3), (130, 4, 2), (33, 2, 4), (1600, 3, 1), (150, 6, 2),
             (1500, 8, 1)]
    probs = _problems(sizes, 40, 0.005, 0)
    iters, lr = 6, 1e-3
    flat = _pack(S, probs)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    Ns = [th.shape[0] for _, _, th in probs]
    times = torch.zeros(len(probs), device="cuda")
    modes = torch.empty(sum(N * s[1] for N, s in zip(Ns, sizes)), dtype=torch.int32, device="cuda")
    st = ctx.status_word()
    cost = ctx.solve([S.make_scene(s) for s, _, _ in probs], [S.make_cost(w) for _, w, _ in probs], Ns,
                     S.make_cfg(iters, lr=lr), flat, m, v, modes_out=modes, solve_time_us=times, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    got = _unpack(S, flat, probs)
    off = 0
    for k, (scene, w, th) in enumerate(probs):
        ref_theta, ref_cost = _per_problem_loop(ctx, S, scene, w, th, iters, lr)
        torch.cuda.synchronize()
        assert torch.equal(got[k], ref_theta), f"problem {k} {sizes[k]}"
        assert torch.equal(cost[off:off + th.shape[0]], ref_cost)
        off += th.shape[0]
    t = times.cpu().numpy()
    print("per-problem solve time us", t, flush=True)
    assert (t > 0).all()


def test_batched_solve_matches_oracle(ctx):
    import paper_2310_01775_amd as S
    # d = 12, 18, 24 (split form), 36 (FP32 matrix-core form).  Every problem
    # is well conditioned: the oracle's own solve moves by at most 3e-5
    # normwise when theta is perturbed by 2^-24 (at H = 6 the (20, 6, 2) draw
    # moves by 3e-4, so FP32 rounding alone puts it above the bar)
    sizes = [(24, 2, 2), (40, 3, 1), (17, 4, 3), (16, 6, 2)]
    probs = _problems(sizes, 60, 0.005, 1)
    iters, lr = 20, 1e-3
    flat = _pack(S, probs)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    Ns = [th.shape[0] for _, _, th in probs]
    ctx.solve([S.make_scene(s) for s, _, _ in probs], [S.make_cost(w) for _, w, _ in probs], Ns,
              S.make_cfg(iters, lr=lr), flat, m, v)
    torch.cuda.synchronize()
    got = _unpack(S, flat, probs)
    for k, (scene, w, th) in enumerate(probs):
        ref = svgd.solve(scene, w, th, iters, lr=lr)["theta"]
        g = S.aos(got[k])
        err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        print("problem", k, "normwise error", err, flush=True)
        assert err < 1e-4


def test_repeated_solves_reuse_the_graph(ctx):
    import paper_2310_01775_amd as S
    probs = _problems([(50, 2, 2), (70, 3, 1)], 30, 0.005, 2)
    Ns = [th.shape[0] for _, _, th in probs]
    scenes = [S.make_scene(s) for s, _, _ in probs]
    ws_ = [S.make_cost(w) for _, w, _ in probs]
    cfg = S.make_cfg(3)
    flat = _pack(S, probs)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    work = torch.empty(ctx.solve_workspace_bytes(scenes, Ns, cfg), dtype=torch.uint8, device="cuda")
    a = flat.clone()
    ctx.solve(scenes, ws_, Ns, cfg, a, m.clone(), v.clone(), workspace=work)
    b = flat.clone()
    mb, vb = m.clone(), v.clone()
    ctx.solve(scenes, ws_, Ns, cfg, b, mb, vb, workspace=work)   # new pointers: new graph
    c = flat.clone()
    ctx.solve(scenes, ws_, Ns, cfg, c, m.clone(), v.clone(), workspace=work)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


@pytest.mark.parametrize("roll_block,roll_grid,phi_rows", [(64, 0, 64), (128, 1024, 128), (256, 0, 256),
                                                          (64, 1024, 256), (256, 1024, 64)])
def test_every_launch_shape_gives_the_same_bits(ctx, roll_block, roll_grid, phi_rows):
    # launch shapes change only how work is grouped, never the arithmetic
    import paper_2310_01775_amd as S
    scene, w, th = W.config_problem(1)
    N = th.shape[0]
    sc, cw = S.make_scene(scene), S.make_cost(w)
    ref, _ = _per_problem_loop(ctx, S, scene, w, th, 3, 1e-3)
    try:
        ctx.set_launch_shape(roll_block, roll_grid, phi_rows)
        theta = S.soa(th)
        m, v = torch.zeros_like(theta), torch.zeros_like(theta)
        ctx.solve([sc], [cw], [N], S.make_cfg(3, lr=1e-3), theta, m, v)
        torch.cuda.synchronize()
    finally:
        ctx.set_launch_shape(0, 0, 0)
    assert torch.equal(theta, ref)


def test_first_autotuned_solve_of_a_large_batch_is_exact():
    """The first solve of a batch signature tunes the contraction row block,
    which changes the length of its work lists; every other workspace region
    must stay where the solve's pointers point (regression: a tuned row block
    below 256 once moved the tape and counter regions under the stale
    pointers, so the first rollout overwrote the work lists).  The tuned run,
    on a fresh context, must equal a run with pinned shapes bit for bit, and
    so must the following calls that resume the Adam step count."""
    import paper_2310_01775_amd as S
    sizes = [(1024, 3, 2)] * 24 + [(2048, 5, 3)] * 8
    probs = _problems(sizes, 20, 0.005, 3)
    Ns = [th.shape[0] for _, _, th in probs]
    scenes = [S.make_scene(s) for s, _, _ in probs]
    ws_ = [S.make_cost(w) for _, w, _ in probs]
    flat = _pack(S, probs)
    results = []
    for pinned in (False, True):
        c = S.Context(0)
        try:
            if pinned:
                c.set_launch_shape(64, 0, 256)
            th, m, v = flat.clone(), torch.zeros_like(flat), torch.zeros_like(flat)
            print("large batch, pinned" if pinned else "large batch, autotuned", flush=True)
            for k in range(3):
                c.solve(scenes, ws_, Ns, S.make_cfg(2, t0=2 * k, lr=1e-3), th, m, v)
            torch.cuda.synchronize()
            results.append(th)
        finally:
            c.close()
    assert torch.equal(results[0], results[1])


def test_full_batch_sampled_against_oracle(ctx):
    """The 64-problem batch itself (N ~ U{64..2048}, H ~ U{2..5}, B ~ U{1..4},
    T = 200), 10 graph-replayed iterations, autotuned; four of its problems
    (one of each block count) checked against the oracle's solve of that
    problem alone (problems in a batch do not interact)."""
    import paper_2310_01775_amd as S
    probs = W.batched_problems(4)
    assert len(probs) == 64
    iters, lr = 10, 1e-3
    flat = _pack(S, probs)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    Ns = [th.shape[0] for _, _, th in probs]
    st = ctx.status_word()
    ctx.solve([S.make_scene(s) for s, _, _ in probs], [S.make_cost(w) for _, w, _ in probs], Ns,
              S.make_cfg(iters, lr=lr), flat, m, v, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    got = _unpack(S, flat, probs)
    for k in (22, 60, 34, 10):  # B = 2, 1, 4, 3; N = 94, 160, 168, 317
        scene, w, th = probs[k]
        print("problem", k, "N", th.shape[0], "B", scene["B"], "H", scene["H"], flush=True)
        ref = svgd.solve(scene, w, th, iters, lr=lr)["theta"]
        g = S.aos(got[k])
        norm = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        worst = (np.abs(g - ref) / np.abs(ref).max(axis=0, keepdims=True)).max()
        print("problem", k, "normwise", norm, "worst coordinate", worst, flush=True)
        assert norm < 2e-6 and worst < 1e-4


def _solve_batch(ctx, S, probs, sizes, cfg):
    flat = _pack(S, probs)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    Ns = [th.shape[0] for _, _, th in probs]
    times = torch.zeros(len(probs), device="cuda")
    modes = torch.empty(sum(N * s[1] for N, s in zip(Ns, sizes)), dtype=torch.int32, device="cuda")
    st = ctx.status_word()
    cost = ctx.solve([S.make_scene(s) for s, _, _ in probs], [S.make_cost(w) for _, w, _ in probs], Ns, cfg,
                     flat, m, v, modes_out=modes, solve_time_us=times, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return flat, m, v, cost, modes, times.cpu().numpy()


def _classes(sizes, T, C):
    """The class of each problem under the library's rule: problems by predicted
    cost per iteration (4 B (T + H) N + 0.26 (d / 30) N^2), cut where the
    running sum reaches c / C of the total, one problem per class at least."""
    cost = [4.0 * B * (T + H) * N + 0.26 * (H / 5.0) * N * N for N, H, B in sizes]
    n = len(sizes)
    order = sorted(range(n), key=lambda p: (cost[p], p))
    C = min(C, n)
    total, run, first = sum(cost), 0.0, [0]
    for q in range(n):
        run += cost[order[q]]
        c, left = len(first) - 1, n - (q + 1)
        need = C - (c + 1)
        if (run >= total * (c + 1) / C and left >= need and need > 0) or left == need:
            first.append(q + 1)
        if len(first) == C + 1:
            break
    first += [n] * (C + 1 - len(first))
    cls = np.empty(n, dtype=int)
    for c in range(C):
        cls[order[first[c]:first[c + 1]]] = c
    return cls


@pytest.mark.parametrize("classes", [2, 3, 7, 50])
def test_class_schedule_equals_the_lockstep_batch(ctx, classes):
    """cfg.classes > 1: the problems run in cost classes, cheapest first, each
    class a batch of its own.  Every output equals the one-batch solve bit for
    bit (the batched kernels reproduce each problem's own iteration), and a
    problem's time is its class's end: never before a cheaper class's."""
    import paper_2310_01775_amd as S
    sizes = [(64, 2, 1), (200, 5, 4), (1, 3, 2), (97, 3, 3), (130, 4, 2), (33, 2, 4), (1600, 3, 1)]
    probs = _problems(sizes, 40, 0.005, 0)
    print("classes", classes, flush=True)
    a = _solve_batch(ctx, S, probs, sizes, S.make_cfg(6, lr=1e-3))
    b = _solve_batch(ctx, S, probs, sizes, S.make_cfg(6, lr=1e-3, classes=classes))
    for x, y in zip(a[:5], b[:5]):
        assert torch.equal(x, y)
    t = b[5]
    print("lockstep us", a[5], "classes us", t, flush=True)
    assert (t > 0).all()
    cls = _classes(sizes, 40, classes)
    for p in range(len(sizes)):
        for q in range(len(sizes)):
            if cls[p] < cls[q]:
                assert t[p] <= t[q], (p, q)
            if cls[p] == cls[q]:
                assert abs(t[p] - t[q]) < 0.05 * t[q] + 50.0, (p, q)


def test_class_schedule_workspace_and_errors(ctx):
    import paper_2310_01775_amd as S
    sizes = [(64, 2, 1), (200, 5, 4), (97, 3, 3)]
    probs = _problems(sizes, 40, 0.005, 3)
    scenes = [S.make_scene(s) for s, _, _ in probs]
    ws_ = [S.make_cost(w) for _, w, _ in probs]
    Ns = [th.shape[0] for _, _, th in probs]
    cfg = S.make_cfg(2, classes=3)
    need = ctx.solve_workspace_bytes(scenes, Ns, cfg)
    assert need > 0
    flat = _pack(S, probs)
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.StampError, match="workspace"):
        ctx.solve(scenes, ws_, Ns, cfg, flat, m, v, workspace=small)
    with pytest.raises(S.StampError, match="classes"):
        ctx.solve(scenes, ws_, Ns, S.make_cfg(2, classes=-1), flat, m, v)


def test_single_problem_graph_follows_the_cost_weights(ctx):
    """A single-problem solve captures its rollout launches with the problem's
    constants (scene, cost weights) as arguments: a second solve on the same
    buffers with other weights must not replay the first one's graph."""
    import paper_2310_01775_amd as S
    (scene, w, th), = _problems([(300, 3, 2)], 40, 0.005, 4)
    w2 = dict(w)
    w2["target"] = 3.0 * w["target"]
    sc = S.make_scene(scene)
    N = th.shape[0]
    cfg = S.make_cfg(4, lr=1e-3)
    work = torch.empty(ctx.solve_workspace_bytes([sc], [N], cfg), dtype=torch.uint8, device="cuda")
    theta = S.soa(th)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    out = []
    for ww in (w, w2):
        theta.copy_(S.soa(th))
        m.zero_()
        v.zero_()
        cost = ctx.solve([sc], [S.make_cost(ww)], [N], cfg, theta, m, v, workspace=work)
        torch.cuda.synchronize()
        out.append((theta.clone(), cost.clone()))
    ref_theta, ref_cost = _per_problem_loop(ctx, S, scene, w2, th, 4, 1e-3)
    torch.cuda.synchronize()
    assert torch.equal(out[1][0], ref_theta) and torch.equal(out[1][1], ref_cost)
    assert not torch.equal(out[0][1], out[1][1])

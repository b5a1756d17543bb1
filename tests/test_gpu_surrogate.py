"""The surrogate pipeline on the GPU: labelling rollouts, standardisation, the
exact bound term, indexed training steps, the surrogate-phase solve (bit for
bit equal to the per-call loop it replaces, the fallback check), and what the
trained network gains over the method without it."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mlp, sim

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _nrm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _net(S, n_in, seed, x=None):
    p = W.mlp_init(n_in, seed=seed)
    rng = np.random.default_rng(seed + 50)
    p["b1"] = W.f32(rng.normal(0, 0.1, 256))
    p["b2"] = W.f32(rng.normal(0, 0.1, 256))
    p["b3"] = W.f32(rng.normal(1.0, 0.3, 1))
    if x is not None:
        mu, isg = mlp.standardization(x)
        p["mu"], p["inv_sigma"] = W.f32(mu), W.f32(isg)
    return p


def test_label_is_the_rollout_cost_without_the_bound_term(ctx):
    import paper_2310_01775_amd as S
    scene = W.make_scene(5, 1003, 3, 5, 200, 0.005)
    w = W.cost_weights()
    th = W.surrogate_training_plans(3, 24)
    th[0, 4] = 0.08  # a plan outside the offset bound: its bound term must not appear
    th = W.f32(th)
    enc = W.scene_encoding(scene)
    n_in = 30 + W.SCENE_ENC
    x, c = ctx.mlp_label(S.make_scene(scene), S.make_cost(w), S.soa(th), n_in, _dev(enc))
    torch.cuda.synchronize()
    ref = sim.cost_np(scene, dict(w, bound=0.0), th)
    got = c.cpu().double().numpy()
    print("label rel err", np.abs(got - ref).max() / np.abs(ref).max(), flush=True)
    assert np.allclose(got, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())
    xs = x.cpu().double().numpy()
    assert np.array_equal(xs[:, :30], th) and np.array_equal(xs[:, 30:], np.repeat(enc[None], 24, 0))


def test_standardize_matches_the_mean_and_std(ctx):
    import paper_2310_01775_amd as S
    rng = np.random.default_rng(4)
    x = W.f32(rng.normal(size=(5000, 40)) * rng.uniform(0.01, 5, 40) + rng.normal(size=40))
    x[:, 7] = 0.25  # a constant input: floor of the standard deviation
    c = W.f32(rng.exponential(20.0, 5000))
    P = _dev(S.pack_mlp(_net(S, 40, 0)))
    ctx.mlp_standardize(P, _dev(x), _dev(c))
    torch.cuda.synchronize()
    q = S.unpack_mlp(P.cpu().numpy(), 40)
    mu, isg = mlp.standardization(x)
    assert np.allclose(q["mu"], mu, rtol=1e-6, atol=1e-7)
    assert np.allclose(q["inv_sigma"], isg, rtol=1e-6)
    assert abs(q["b3"][0] - np.log1p(c).mean()) < 1e-6 * abs(np.log1p(c).mean())
    Pn = P.cpu().numpy()
    assert not Pn[40:64].any() and np.all(Pn[64 + 40:128] == 1.0)  # padded inputs: mu 0, inv_sigma 1


def test_forward_adds_the_exact_bound_term(ctx):
    """A constant network (weights zero, b3 = log(1 + c0)) isolates the bound
    term: value and gradient to FP32 rounding against the oracle.  A trained-
    like random network then matches the oracle's C_hat to the BF16 bar."""
    import paper_2310_01775_amd as S
    H, n_in = 5, 54
    rng = np.random.default_rng(9)
    th = W.make_particles(5, 0, 700, H)
    th[:, 4::6] += rng.normal(0, 0.04, (700, H))   # many offsets outside +-0.05
    th[:, 5::6] += rng.normal(0, 0.08, (700, H))   # depths below 0 and above 0.3
    th = W.f32(th)
    enc = W.scene_encoding(W.make_scene(5, 0, 3, H, 200, 0.005))
    w = W.cost_weights()
    p0 = W.mlp_init(n_in, seed=1)
    for k in ("W1", "W2", "w3"):
        p0[k] = np.zeros_like(p0[k])
    p0["b3"] = W.f32([np.log1p(2.5)])
    for p, bar in ((p0, None), (_net(S, n_in, 2, np.concatenate([th, np.repeat(enc[None], 700, 0)], 1)), 2e-2)):
        P = _dev(S.pack_mlp(p))
        Wb = ctx.mlp_weights()
        ctx.mlp_prepare(P, Wb)
        _, c, g = ctx.mlp_forward(P, Wb, S.soa(th), n_in, 30, x_layout=1, enc=_dev(enc), want_y=False,
                                  want_cost=True, want_grad=True, w=S.make_cost(w))
        torch.cuda.synchronize()
        C_ref, g_ref = mlp.surrogate_cost_and_grad(p, th, enc, w)
        c, g = c.cpu().double().numpy(), S.aos(g)
        if bar is None:
            assert np.allclose(c, C_ref, rtol=2e-6)
            assert np.allclose(g, g_ref, rtol=2e-6, atol=1e-6 * np.abs(g_ref).max())
        else:
            print("C_hat err", _nrm(c, C_ref), "grad err", _nrm(g, g_ref), flush=True)
            assert _nrm(c, C_ref) < bar and _nrm(g, g_ref) < 3e-2


def test_train_step_on_indexed_rows(ctx):
    """The minibatch is a list of dataset rows: the first step's gradient
    (m = (1 - beta1) g) equals the oracle's on exactly those rows; an index
    outside the dataset reads row 0 and raises the status bit."""
    import paper_2310_01775_amd as S
    rng = np.random.default_rng(11)
    n_rows, n_in, M = 3000, 54, 1024
    x = W.f32(rng.normal(size=(n_rows, n_in)))
    c = W.f32(rng.exponential(30.0, n_rows))
    idx = rng.integers(0, n_rows, M).astype(np.int32)
    p = _net(S, n_in, 3, x)
    P = _dev(S.pack_mlp(p))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    m, v = torch.zeros(S.MLP_PARAMS, device="cuda"), torch.zeros(S.MLP_PARAMS, device="cuda")
    st = ctx.status_word()
    ctx.mlp_train_step(P, Wb, m, v, _dev(x), _dev(c), 1, idx=_dev(idx, torch.int32), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _, g_ref = mlp.training_loss_and_grads(p, x[idx], c[idx])
    g = S.unpack_mlp(m.cpu().double().numpy() / 0.1, n_in)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        assert _nrm(g[k], g_ref[k]) < 3e-2, k
    bad = idx.copy()
    bad[5], bad[700] = n_rows, -3
    ctx.mlp_train_step(P, Wb, m, v, _dev(x), _dev(c), 2, idx=_dev(bad, torch.int32), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == S.STATUS_BAD_INDEX


def _enc(e, n_in, d):
    """The scene encoding followed by zeros up to the network's n_in - d inputs."""
    out = np.zeros(n_in - d)
    out[:min(len(e), n_in - d)] = e[:n_in - d]
    return out


def _batch(S, sizes, seed):
    probs = []
    for q, (N, H, B) in enumerate(sizes):
        scene = W.make_scene(60 + seed, q, B, H, 40, 0.005)
        probs.append((scene, W.cost_weights(), W.make_particles(60 + seed, q, N, H), W.scene_encoding(scene)))
    return probs


def _reference_loop(ctx, S, probs, net, n_in, n_sur, n_true, lr=1e-3):
    """Per-call loop: n_sur iterations on the network's gradient, then n_true
    true iterations, each problem on its own."""
    P, Wb = net
    out = []
    for scene, w, th, enc in probs:
        sc, cw = S.make_scene(scene), S.make_cost(w)
        N, d = th.shape
        theta = S.soa(th)
        m, v = torch.zeros_like(theta), torch.zeros_like(theta)
        g = torch.empty_like(theta)
        for t in range(1, n_sur + 1):
            ctx.mlp_forward(P, Wb, theta, n_in, d, x_layout=1, enc=_dev(_enc(enc, n_in, d)), want_y=False, grad=g,
                            grad_scale=-1.0, w=cw)
            phi = ctx.svgd_step(theta, g)
            ctx.adam_step(theta, phi, m, v, t, lr=lr)
        tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")
        minus = torch.full((N,), -1.0, device="cuda")
        for t in range(n_sur + 1, n_sur + n_true + 1):
            ctx.rollout_fwd(sc, cw, theta, tape=tape)
            g2 = ctx.rollout_adj(sc, cw, theta, tape, cost_bar=minus)
            phi = ctx.svgd_step(theta, g2)
            ctx.adam_step(theta, phi, m, v, t, lr=lr)
        out.append(theta)
    return out


def _solve_sur(ctx, S, probs, net, n_in, iters, n_sur, **kw):
    P, Wb = net
    flat = torch.cat([S.soa(th).reshape(-1) for _, _, th, _ in probs]).contiguous()
    enc = _dev(np.concatenate([_enc(e, n_in, 6 * s["H"]) for s, _, _, e in probs]))
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    cost, rep = ctx.solve_surrogate([S.make_scene(s) for s, _, _, _ in probs], [S.make_cost(w) for _, w, _, _ in probs],
                                    [th.shape[0] for _, _, th, _ in probs], S.make_cfg(iters, lr=1e-3), n_sur, P, Wb,
                                    n_in, enc, flat, m, v, **kw)
    torch.cuda.synchronize()
    out, off = [], 0
    for _, _, th, _ in probs:
        out.append(flat[off:off + th.size].view(th.shape[1], th.shape[0]))
        off += th.size
    return out, cost, rep


def _network(ctx, S, n_in, seed):
    P = _dev(S.pack_mlp(_net(S, n_in, seed)))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    return P, Wb


def test_surrogate_solve_equals_the_per_call_loop(ctx):
    import paper_2310_01775_amd as S
    probs = _batch(S, [(100, 3, 2), (64, 2, 1), (37, 3, 3)], 0)
    n_in = 18 + W.SCENE_ENC
    net = _network(ctx, S, n_in, 4)
    got, _, rep = _solve_sur(ctx, S, probs, net, n_in, 8, 5, check_every=2)
    ref = _reference_loop(ctx, S, probs, net, n_in, 5, 3)
    torch.cuda.synchronize()
    assert rep.iters_run == 5 and rep.fell_back == 0 and rep.checks == 3
    for k in range(len(probs)):
        assert torch.equal(got[k], ref[k]), k


def test_surrogate_solve_with_no_surrogate_iterations_is_the_plain_solve(ctx):
    import paper_2310_01775_amd as S
    probs = _batch(S, [(50, 2, 2), (70, 3, 1)], 1)
    n_in = 18 + W.SCENE_ENC
    net = _network(ctx, S, n_in, 5)
    got, cost, rep = _solve_sur(ctx, S, probs, net, n_in, 4, 0)
    flat = torch.cat([S.soa(th).reshape(-1) for _, _, th, _ in probs]).contiguous()
    m, v = torch.zeros_like(flat), torch.zeros_like(flat)
    cost2 = ctx.solve([S.make_scene(s) for s, _, _, _ in probs], [S.make_cost(w) for _, w, _, _ in probs],
                      [th.shape[0] for _, _, th, _ in probs], S.make_cfg(4, lr=1e-3), flat, m, v)
    torch.cuda.synchronize()
    assert rep.iters_run == 0 and rep.checks == 0
    assert torch.equal(torch.cat([g.reshape(-1) for g in got]), flat) and torch.equal(cost, cost2)


def test_surrogate_check_falls_back_to_the_simulator(ctx):
    """An error bound no network meets ends the surrogate phase at the first
    check; the rest are true iterations, bit for bit as in the per-call loop."""
    import paper_2310_01775_amd as S
    probs = _batch(S, [(80, 3, 2), (33, 2, 2)], 2)
    n_in = 18 + W.SCENE_ENC
    net = _network(ctx, S, n_in, 6)
    got, _, rep = _solve_sur(ctx, S, probs, net, n_in, 7, 6, check_every=2, max_log_err=1e-6)
    ref = _reference_loop(ctx, S, probs, net, n_in, 2, 5)
    torch.cuda.synchronize()
    assert rep.fell_back == 1 and rep.iters_run == 2 and rep.checks == 1 and rep.log_err > 1e-6
    for k in range(len(probs)):
        assert torch.equal(got[k], ref[k]), k


def test_surrogate_argument_errors(ctx):
    import paper_2310_01775_amd as S
    probs = _batch(S, [(20, 3, 2)], 3)
    n_in = 18 + W.SCENE_ENC
    net = _network(ctx, S, n_in, 7)
    with pytest.raises(S.StampError):  # more surrogate iterations than iterations
        _solve_sur(ctx, S, probs, net, n_in, 3, 4)
    with pytest.raises(S.StampError):  # network narrower than the plan
        scene, w, th, _ = probs[0]
        theta = S.soa(th)
        ctx.solve_surrogate([S.make_scene(scene)], [S.make_cost(w)], [th.shape[0]], S.make_cfg(3), 1, net[0], net[1],
                            12, None, theta, torch.zeros_like(theta), torch.zeros_like(theta))


def test_trained_network_gains_over_the_method_without_it(ctx):
    """The network, trained by the pipeline (2^20 labelled rollouts on
    training scenes, two on-policy rounds), drives the first 240 of 300 SVGD
    iterations on an unseen scene at N = 16384.  With the same 60 true-sim
    iterations afterwards it ends far below the run that spends only those 60,
    and below the plain method's 300 true iterations."""
    import paper_2310_01775_amd as S
    from paper_2310_01775_amd import surrogate as SG
    R = dict(W.SURROGATE_RECIPE)
    H = 5
    n_in = 6 * H + W.SCENE_ENC
    cw = S.make_cost(W.cost_weights())
    scenes = W.surrogate_dataset_scenes(max(R["random_scenes"], R["rounds"] * R["round_scenes"]))
    structs = [S.make_scene(sc) for sc in scenes]
    encs = [_dev(W.scene_encoding(sc)) for sc in scenes]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(R["seed"])
    print("training the surrogate", flush=True)
    net, ds, log, reps = SG.train_recipe(ctx, R, lambda p: (structs[p], cw, encs[p]),
                                         lambda p, n: S.soa(W.surrogate_training_plans(p, n, H)),
                                         lambda p, n: S.soa(W.make_particles(5, 1000 + p, n, H)),
                                         W.mlp_init(n_in, seed=R["seed"]), n_in, gen, progress=print)
    assert ds.n == 1 << 20
    scene, _, th0 = W.config_problem(5)
    N = th0.shape[0]
    sc = S.make_scene(scene)

    def plain(iters):
        th = S.soa(th0)
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        return ctx.solve([sc], [cw], [N], S.make_cfg(iters, lr=1e-3), th, m, v)

    th = S.soa(th0)
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    c_sur, rep = ctx.solve_surrogate([sc], [cw], [N], S.make_cfg(300, lr=1e-3), 240, net.params, net.wbf16, n_in,
                                     _dev(W.scene_encoding(scene)), th, m, v, check_every=80)
    costs = {k: f().double() for k, f in
             dict(init=lambda: plain(0), true60=lambda: plain(60), plain300=lambda: plain(300)).items()}
    costs["surrogate240+60"] = c_sur.double()
    med = {k: float(c.median()) for k, c in costs.items()}
    mean = {k: float(c.mean()) for k, c in costs.items()}
    print("median true cost", med, "mean", mean, "handoff log-error", rep.log_err, flush=True)
    assert rep.iters_run == 240 and rep.fell_back == 0 and rep.checks == 3
    assert med["surrogate240+60"] < 0.25 * med["true60"]
    # equal cost, in the plain method's mean final true cost and in the median
    assert med["surrogate240+60"] < med["plain300"]
    assert mean["surrogate240+60"] < mean["plain300"]


def test_binding_rejects_64_bit_arrays(ctx):
    """A float64 array (numpy's default) handed to the C ABI, which takes
    float32, is refused by the binding instead of being read as garbage."""
    import paper_2310_01775_amd as S
    probs = _batch(S, [(40, 3, 2)], 1)
    n_in = 18 + W.SCENE_ENC
    P, Wb = _network(ctx, S, n_in, 4)
    scene, w, th, e = probs[0]
    theta = S.soa(th)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    enc64 = torch.as_tensor(_enc(e, n_in, 18), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="float32"):
        ctx.solve_surrogate([S.make_scene(scene)], [S.make_cost(w)], [th.shape[0]], S.make_cfg(2, lr=1e-3), 2, P, Wb,
                            n_in, enc64, theta, m, v)

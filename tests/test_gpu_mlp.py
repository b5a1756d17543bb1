"""GPU surrogate network (BF16 matrix cores, FP32 accumulation) against the
FP64 oracle of the same network, through the C ABI.

Tolerances come from the arithmetic: every matrix product reads BF16 operands
(8 significant bits, unit roundoff 2^-9 = 1.95e-3), one rounding of the
activations and one of the weights per layer, accumulated in FP32.  Summed
over ~n random-signed terms the relative error of a layer output stays a small
multiple of the unit roundoff, so the forward value y is held to 1e-2
normwise and the two extra BF16 layers of the backward pass (delta2 W2 and
delta1 W1) to 3e-2 normwise; per-element bounds are looser because single
outputs can sit near a cancellation."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mlp

pytestmark = pytest.mark.gpu

D_PLAN = 30
N_IN = D_PLAN + W.SCENE_ENC


def _params(seed=0, n_in=N_IN, x=None):
    p = W.mlp_init(n_in, seed=seed)
    rng = np.random.default_rng(100 + seed)
    p["b1"] = W.f32(rng.normal(0, 0.1, 256))
    p["b2"] = W.f32(rng.normal(0, 0.1, 256))
    p["b3"] = W.f32(rng.normal(0, 0.5, 1))
    if x is not None:  # standardisation constants from the data
        p["mu"] = W.f32(x.mean(0))
        p["inv_sigma"] = W.f32(1.0 / np.maximum(x.std(0), 1e-3))
    return p


def _inputs(M, seed=0):
    scenes = W.surrogate_dataset_scenes(4)
    th = np.concatenate(W.surrogate_dataset_particles(4, (M + 3) // 4))[:M]
    enc = np.stack([W.scene_encoding(s) for s in scenes])
    rows = np.repeat(enc, (M + 3) // 4, axis=0)[:M]
    return W.f32(np.concatenate([th, rows], axis=1)), enc


def _nrm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("M", [1, 63, 64, 1000, 4096])
def test_forward_and_input_gradient(ctx, M):
    import paper_2310_01775_amd as S
    print("case M", M, flush=True)
    x, _ = _inputs(M)
    p = _params(0, x=x if M > 1 else None)
    P = _dev(S.pack_mlp(p))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    y, c, g = ctx.mlp_forward(P, Wb, _dev(x), N_IN, D_PLAN, want_cost=True, want_grad=True)
    torch.cuda.synchronize()
    y_ref, gx_ref = mlp.forward(p, x, need_input_grad=True)
    c_ref, gc_ref = mlp.cost_and_grad(p, x, D_PLAN)
    y, c, g = y.cpu().double().numpy(), c.cpu().double().numpy(), g.cpu().double().numpy().T
    ey, eg = _nrm(y, y_ref), _nrm(g, gc_ref)
    print("y err", ey, "grad err", eg, flush=True)
    assert ey < 1e-2
    assert np.abs(y - y_ref).max() < 5e-2 * (np.abs(y_ref).max() + 1e-3)
    assert np.allclose(c, np.expm1(y), rtol=1e-5, atol=1e-6)  # C_hat = e^y - 1 of its own y
    assert _nrm(c, c_ref) < 2e-2
    assert eg < 3e-2
    # the gradient is e^y * dy/dx; undo the scale and compare dy/dx per column scale
    gy = g / np.exp(y)[:, None]
    colscale = np.abs(gx_ref[:, :D_PLAN]).max(axis=0) + 1e-9
    assert (np.abs(gy - gx_ref[:, :D_PLAN]) / colscale).max() < 0.1


@pytest.mark.parametrize("layout", [0, 1])
def test_gradient_writes_exactly_d_rows(ctx, layout):
    """grad is [d][M] with d < n_in in both input layouts: the floats after it
    keep their sentinel (regression: the sample-major layout once wrote n_in
    rows)."""
    import paper_2310_01775_amd as S
    M = 4096
    x, enc = _inputs(M)
    p = _params(0, x=x)
    P = _dev(S.pack_mlp(p))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    buf = torch.full((D_PLAN * M + 4 * M,), 12345.0, device="cuda")
    g = buf[:D_PLAN * M].view(D_PLAN, M)
    if layout == 0:
        ctx.mlp_forward(P, Wb, _dev(x), N_IN, D_PLAN, grad=g)
    else:
        ctx.mlp_forward(P, Wb, _dev(x[:, :D_PLAN].T), N_IN, D_PLAN, x_layout=1, enc=_dev(enc[0]), grad=g)
    torch.cuda.synchronize()
    assert torch.all(buf[D_PLAN * M:] == 12345.0)
    assert torch.isfinite(g).all() and not torch.any(g == 12345.0)


def test_particle_layout_matches_sample_layout(ctx):
    """x_layout 1 (plan [d][M] + one shared scene encoding, grad scaled) gives
    the same numbers as the sample-major layout, bit for bit."""
    import paper_2310_01775_amd as S
    M = 777
    x, enc = _inputs(M)
    x[:, D_PLAN:] = enc[0]  # one scene for every sample
    p = _params(1, x=x)
    P = _dev(S.pack_mlp(p))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    y0, c0, g0 = ctx.mlp_forward(P, Wb, _dev(x), N_IN, D_PLAN, want_cost=True, want_grad=True)
    xs = _dev(x[:, :D_PLAN].T)
    y1, c1, g1 = ctx.mlp_forward(P, Wb, xs, N_IN, D_PLAN, x_layout=1, enc=_dev(enc[0]), want_cost=True,
                                 want_grad=True, grad_scale=-1.0)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1) and torch.equal(c0, c1)
    assert torch.equal(g0, -g1)


def test_training_gradient_matches_oracle(ctx):
    """After one Adam step from zero moments, m = (1 - beta1) g: the kernels'
    loss gradient of every trained tensor against the oracle's."""
    import paper_2310_01775_amd as S
    M = 2048
    x, _ = _inputs(M)
    p = _params(2, x=x)
    rng = np.random.default_rng(7)
    c_np = W.f32(np.expm1(rng.normal(1.0, 1.0, M)))  # targets log(1 + c) ~ N(1, 1)
    P = _dev(S.pack_mlp(p))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    m = torch.zeros(S.MLP_PARAMS, device="cuda")
    v = torch.zeros(S.MLP_PARAMS, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ctx.mlp_train_step(P, Wb, m, v, _dev(x), _dev(c_np), 1, lr=1e-3, loss=loss)
    torch.cuda.synchronize()
    L_ref, g_ref = mlp.training_loss_and_grads(p, x, c_np)
    g_gpu = S.unpack_mlp(m.cpu().double().numpy() / 0.1, N_IN)
    print("loss", float(loss.item()), L_ref, flush=True)
    assert abs(float(loss.item()) - L_ref) < 1e-2 * L_ref
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        e = _nrm(g_gpu[k], g_ref[k])
        print("grad", k, e, flush=True)
        assert e < 3e-2, k
    # untrained entries stay put: standardisation and the zero input padding
    Pn = P.cpu().numpy()
    P0 = S.pack_mlp(p)
    assert np.array_equal(Pn[:128], P0[:128])
    W1 = Pn[128:128 + 256 * 64].reshape(256, 64)
    assert not W1[:, N_IN:].any()
    # the BF16 copies were refreshed from the updated weights
    Wb2 = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb2)
    torch.cuda.synchronize()
    assert torch.equal(Wb.view(torch.int16), Wb2.view(torch.int16))


def test_training_fits_and_oracle_agrees(ctx):
    """A few hundred Adam steps on a smooth synthetic target reduce the loss;
    the oracle, evaluating the trained weights in FP64, sees the same loss."""
    import paper_2310_01775_amd as S
    M = 4096
    x, _ = _inputs(M)
    p = _params(3, x=x)
    u = (x - p["mu"]) * p["inv_sigma"]
    t_np = np.sin(u[:, 0]) + 0.5 * u[:, 4] * u[:, 5] - 0.3 * u[:, D_PLAN + 1]
    c_np = W.f32(np.expm1(t_np))
    t_np = np.log1p(c_np)
    P = _dev(S.pack_mlp(p))
    Wb = ctx.mlp_weights()
    ctx.mlp_prepare(P, Wb)
    m = torch.zeros(S.MLP_PARAMS, device="cuda")
    v = torch.zeros(S.MLP_PARAMS, device="cuda")
    loss = torch.zeros(1, device="cuda")
    X, T = _dev(x), _dev(c_np)
    ws = torch.empty(ctx.mlp_train_workspace_bytes(M), dtype=torch.uint8, device="cuda")
    losses = []
    for t in range(1, 301):
        ctx.mlp_train_step(P, Wb, m, v, X, T, t, lr=2e-3, loss=loss, workspace=ws)
        if t in (1, 300):
            torch.cuda.synchronize()
            losses.append(float(loss.item()))
    y, _, _ = ctx.mlp_forward(P, Wb, X, N_IN, D_PLAN)
    torch.cuda.synchronize()
    print("losses", losses, flush=True)
    assert losses[1] < 0.1 * losses[0]
    p_tr = S.unpack_mlp(P.cpu().numpy(), N_IN)
    y_ref, _ = mlp.forward(p_tr, x)
    L_gpu = float(((y.cpu().double().numpy() - t_np) ** 2).mean())
    L_ref = float(((y_ref - t_np) ** 2).mean())
    print("trained loss gpu", L_gpu, "oracle", L_ref, flush=True)
    assert abs(L_gpu - L_ref) < 0.1 * L_ref + 1e-4


def test_train_steps_equal_single_steps(ctx):
    """stamp_mlp_train_steps launches the steps of stamp_mlp_train_step back to
    back: parameters, moments, BF16 copies and every step's loss are the same
    bits as those of the single-step calls."""
    import paper_2310_01775_amd as S
    n_rows, M, steps = 3000, 1024, 5
    x, _ = _inputs(n_rows)
    p = _params(4, x=x)
    rng = np.random.default_rng(11)
    X = _dev(x)
    Cst = _dev(W.f32(np.expm1(rng.normal(1.0, 1.0, n_rows))))
    idx = torch.as_tensor(rng.integers(0, n_rows, (steps, M)), dtype=torch.int32, device="cuda").contiguous()
    lrs = [1e-3 * (0.9 ** s) for s in range(steps)]
    out = []
    for multi in (False, True):
        P = _dev(S.pack_mlp(p))
        Wb = ctx.mlp_weights()
        ctx.mlp_prepare(P, Wb)
        m = torch.zeros(S.MLP_PARAMS, device="cuda")
        v = torch.zeros(S.MLP_PARAMS, device="cuda")
        loss = torch.zeros(steps, device="cuda")
        st = ctx.status_word()
        if multi:
            ctx.mlp_train_steps(P, Wb, m, v, X, Cst, 2, idx, lrs, loss=loss, status=st)
        else:
            for s in range(steps):
                ctx.mlp_train_step(P, Wb, m, v, X, Cst, 3 + s, idx=idx[s].contiguous(), lr=lrs[s], loss=loss[s:s + 1],
                                   status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        out.append((P, Wb.view(torch.int16), m, v, loss))
    for a, b in zip(*out):
        assert torch.equal(a, b)
    assert bool((out[1][4] > 0).all())


def test_argument_errors(ctx):
    import paper_2310_01775_amd as S
    P = torch.zeros(S.MLP_PARAMS, device="cuda")
    Wb = ctx.mlp_weights()
    x = torch.zeros((100, N_IN), device="cuda")
    with pytest.raises(S.StampError):
        ctx.mlp_forward(P, Wb, torch.zeros((100, 65), device="cuda"), 65, 30)
    with pytest.raises(S.StampError):
        ctx.mlp_forward(P, Wb, x, N_IN, N_IN + 1)
    m = torch.zeros(S.MLP_PARAMS, device="cuda")
    with pytest.raises(S.StampError):  # M not a multiple of 64
        ctx.mlp_train_step(P, Wb, m, m.clone(), x, torch.zeros(100, device="cuda"), 1,
                           workspace=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    with pytest.raises(S.StampError):  # workspace too small
        ctx.mlp_train_step(P, Wb, m, m.clone(), x[:64], torch.zeros(64, device="cuda"), 1,
                           workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    with pytest.raises(S.StampError):  # a minibatch larger than the dataset without indices
        ctx.mlp_train_step(P, Wb, m, m.clone(), x[:64], torch.zeros(64, device="cuda"), 1, M=128)

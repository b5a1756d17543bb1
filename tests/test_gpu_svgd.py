"""GPU SVGD step (median bandwidth + Eq. (1) direction) and update against the
FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import svgd

pytestmark = pytest.mark.gpu


def _pair_sqdist(th):
    diff = th[:, None, :] - th[None, :, :]
    D = (diff * diff).sum(-1)
    return D[np.triu_indices(th.shape[0], 1)]


@pytest.mark.parametrize("N,d", [(2, 6), (3, 2), (37, 12), (64, 18), (65, 18), (130, 30), (1024, 18), (777, 48)])
def test_median_bandwidth_is_the_exact_order_statistic(ctx, N, d):
    import paper_2310_01775_amd as S
    print("case", N, d, flush=True)
    rng = np.random.default_rng(N * 100 + d)
    th = rng.standard_normal((N, d)).astype(np.float32).astype(np.float64)
    g = rng.standard_normal((N, d))
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.svgd_step(S.soa(th), S.soa(g), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    h = float(h_out.item())
    m2 = h * math.log(N)
    ref = svgd.median_sqdist(th)
    assert abs(m2 - ref) <= 3e-6 * ref
    # rank check in FP64: the selected value sits at rank ceil(P/2)
    D = _pair_sqdist(th)
    k = (D.size + 1) // 2
    lo, hi = m2 * (1 - 3e-6), m2 * (1 + 3e-6)
    assert (D < lo).sum() < k <= (D <= hi).sum()


def _median_blocked(th):
    """Exact lower median of the FP64 pair distances over i < j, row by row
    (no N x N x d array)."""
    N = th.shape[0]
    out = []
    for i in range(N - 1):
        diff = th[i + 1:] - th[i]
        out.append((diff * diff).sum(1))
    D = np.concatenate(out)
    k = (D.size + 1) // 2
    return np.partition(D, k - 1)[k - 1], D, k


@pytest.mark.parametrize("N,d", [(129, 18), (3000, 30), (6000, 18)])
def test_median_of_many_pairs_is_exact(ctx, N, d):
    """Above 8192 pairs the median comes from the interval select (sample
    bracket, candidate passes): still the exact order statistic."""
    import paper_2310_01775_amd as S
    print("case", N, d, flush=True)
    rng = np.random.default_rng(N * 7 + d)
    th = rng.standard_normal((N, d)).astype(np.float32).astype(np.float64)
    th[:, 4::6] *= 0.03
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.svgd_step(S.soa(th), S.soa(rng.standard_normal((N, d))), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    m2 = float(h_out.item()) * math.log(N)
    ref, D, k = _median_blocked(th)
    assert abs(m2 - ref) <= 3e-6 * ref
    lo, hi = m2 * (1 - 3e-6), m2 * (1 + 3e-6)
    assert (D < lo).sum() < k <= (D <= hi).sum()


@pytest.mark.parametrize("N", [1000, 2000])
def test_median_with_massive_ties_takes_the_all_pairs_passes(ctx, N):
    """Two clusters of identical particles: just under half the pairs are at
    distance 0 and the rest share one value, the median; the bracket then
    holds more values than the candidate buffer (at 1000 particles) and the
    select finishes with passes over all pairs.  The result is that shared
    distance.  At 2000 particles (above 2^20 pairs) the passes take the
    Gram form, whose identical operands give identical values too."""
    import paper_2310_01775_amd as S
    d = 12
    th = np.zeros((N, d))
    th[N // 2:] = W.f32(np.linspace(0.1, 1.2, d))
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.svgd_step(S.soa(th), S.soa(np.ones((N, d))), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    want = np.float32(0.0)
    for l in range(d):  # FP32 fused multiply-adds in coordinate order, as the kernels add
        df = np.float64(np.float32(0.0) - np.float32(th[N // 2, l]))
        want = np.float32(df * df + np.float64(want))
    m2 = float(h_out.item()) * math.log(N)
    assert abs(m2 - float(want)) <= 2e-6 * float(want)


@pytest.mark.parametrize("N,d,bw", [(1, 6, 0.0), (2, 6, 0.0), (37, 12, 0.0), (65, 18, 2.5), (300, 18, 0.0),
                                    (1024, 18, 0.0), (513, 30, 0.0), (300, 31, 0.0), (300, 32, 0.0),
                                    (200, 48, 0.0)])
def test_phi_matches_oracle(ctx, N, d, bw):
    import paper_2310_01775_amd as S
    print("case", N, d, bw, flush=True)
    rng = np.random.default_rng(N + d)
    th = rng.standard_normal((N, d)).astype(np.float32).astype(np.float64)
    th[:, ::6] *= 0.1  # mixed coordinate scales, like offsets next to logits
    g = (rng.standard_normal((N, d)) * 50).astype(np.float32).astype(np.float64)
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    phi = ctx.svgd_step(S.soa(th), S.soa(g), bw, h_out=h_out)
    torch.cuda.synchronize()
    h = svgd.bandwidth(th, bw)
    ref = g if N == 1 else svgd.svgd_phi(th, g, h)
    got = S.aos(phi)
    scale = np.abs(ref).max(axis=0, keepdims=True) + 1e-9
    err = (np.abs(got - ref) / scale).max()
    print("phi err", err, flush=True)
    assert err < 2e-5
    if N == 1:
        assert np.array_equal(got, g)


@pytest.mark.parametrize("N,d,lo,hi", [(300, 24, 1e-3, 1e2), (257, 31, 1e-2, 1e3)])
def test_phi_matches_oracle_with_mixed_coordinate_scales(ctx, N, d, lo, hi):
    """Coordinates of very different scales side by side (the split form
    carries each FP32 operand as three BF16 parts, whose exponent range is
    FP32's): phi still within 2e-5 of each coordinate's scale."""
    import paper_2310_01775_amd as S
    print("case", N, d, lo, hi, flush=True)
    rng = np.random.default_rng(N * 3 + d)
    scales = np.where(np.arange(d) % 2 == 0, lo, hi)
    th = (rng.standard_normal((N, d)) * scales).astype(np.float32).astype(np.float64)
    g = (rng.standard_normal((N, d)) * 50 / scales).astype(np.float32).astype(np.float64)
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    phi = ctx.svgd_step(S.soa(th), S.soa(g), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    h = svgd.bandwidth(th, 0.0)
    ref = svgd.svgd_phi(th, g, h)
    got = S.aos(phi)
    scale = np.abs(ref).max(axis=0, keepdims=True) + 1e-30
    err = (np.abs(got - ref) / scale).max()
    print("phi err", err, flush=True)
    assert err < 2e-5


def test_adam_and_plain_step_match_oracle(ctx):
    import paper_2310_01775_amd as S
    rng = np.random.default_rng(9)
    x = rng.standard_normal((50, 18)).astype(np.float32).astype(np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    tx, tm, tv = S.soa(x), S.soa(m), S.soa(v)
    for t in range(1, 25):
        phi = (rng.standard_normal(x.shape) * 10.0 ** rng.integers(-3, 3)).astype(np.float32).astype(np.float64)
        x, m, v = svgd.adam_step(x, phi, m, v, t, 1e-2)
        ctx.adam_step(tx, S.soa(phi), tm, tv, t, lr=1e-2)
    torch.cuda.synchronize()
    assert np.allclose(S.aos(tx), x, rtol=1e-5, atol=1e-6)
    phi = rng.standard_normal(x.shape)
    ctx.adam_step(tx, S.soa(phi), None, None, 1, lr=0.5, use_adam=False)
    torch.cuda.synchronize()
    assert np.allclose(S.aos(tx), x + 0.5 * phi.astype(np.float32), rtol=1e-5, atol=1e-6)


def test_svgd_argument_errors(ctx):
    import paper_2310_01775_amd as S
    th = torch.zeros(70, 4, device="cuda")
    with pytest.raises(S.StampError) as e:
        ctx.svgd_step(th, th, 0.0)
    assert e.value.code == S.EUNSUPPORTED
    th = torch.zeros(6, 4, device="cuda")
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.StampError) as e:
        ctx.svgd_step(th, th, 0.0, workspace=small)
    assert e.value.code == S.ENOSPACE


@pytest.mark.parametrize("N,d", [(1, 6), (300, 18), (4096, 30)])
def test_two_half_step_on_two_streams_equals_the_step(ctx, N, d):
    """stamp_svgd_bandwidth on a side stream (as beside a rollout) and
    stamp_svgd_direction on the main stream after an event give the step's
    phi and h bit for bit."""
    import paper_2310_01775_amd as S
    print("case", N, d, flush=True)
    rng = np.random.default_rng(N + d)
    th = S.soa(W.f32(rng.standard_normal((N, d))))
    g = S.soa(W.f32(rng.standard_normal((N, d)) * 3.0))
    h1, h2 = torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda")
    ref = ctx.svgd_step(th, g, 0.0, h_out=h1)
    ws = torch.empty(ctx.svgd_workspace_bytes(N, d), dtype=torch.uint8, device="cuda")
    main, side = torch.cuda.current_stream(), torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(), torch.cuda.Event()
    for _ in range(2):  # the second round reuses the workspace
        ev0.record(main)
        side.wait_event(ev0)
        ctx.svgd_bandwidth(th, 0.0, h_out=h2, workspace=ws, stream=side)
        ev1.record(side)
        main.wait_event(ev1)
        got = ctx.svgd_direction(th, g, ws)
    torch.cuda.synchronize()
    assert torch.equal(got, ref) and torch.equal(h1, h2)


@pytest.mark.parametrize("N,d,use_adam,weighted", [(1, 6, True, False), (300, 18, True, False),
                                                   (1000, 30, False, False), (777, 48, True, True)])
def test_fused_direction_update_equals_direction_then_update(ctx, N, d, use_adam, weighted):
    """stamp_svgd_update = stamp_svgd_direction + stamp_adam_step, bit for bit."""
    import paper_2310_01775_amd as S
    print("case", N, d, use_adam, weighted, flush=True)
    rng = np.random.default_rng(N * 7 + d)
    th = S.soa(W.f32(rng.standard_normal((N, d))))
    g = S.soa(W.f32(rng.standard_normal((N, d)) * 3.0))
    m0 = S.soa(W.f32(rng.standard_normal((N, d)) * 0.1))
    v0 = S.soa(W.f32(rng.uniform(0.0, 0.2, (N, d))))
    w = None
    if weighted:
        w = rng.uniform(0.0, 2.0, N)
        w = torch.tensor(w * N / w.sum(), dtype=torch.float32, device="cuda")
    ws = ctx.svgd_bandwidth(th)
    a, ma, va = th.clone(), m0.clone(), v0.clone()
    phi_a = ctx.svgd_direction(a, g, ws, weights=w)
    ctx.adam_step(a, phi_a, ma, va, 7, lr=1e-2, use_adam=use_adam)
    b, mb, vb = th.clone(), m0.clone(), v0.clone()
    phi_b = torch.empty_like(th)
    ctx.svgd_update(b, g, ws, mb, vb, 7, lr=1e-2, use_adam=use_adam, weights=w, phi=phi_b)
    torch.cuda.synchronize()
    assert torch.equal(phi_a, phi_b) and torch.equal(a, b)
    if use_adam:
        assert torch.equal(ma, mb) and torch.equal(va, vb)


# --------------------------------------------------------------------------
# Full size of the surrogate workload: N = 16384 particles of d = 30 (5 pushes).
# The contraction runs its 2048-column splits and the median its Gram-form
# passes here; the oracle computes phi on 512 sampled rows (svgd_phi_rows,
# pinned against the full svgd_phi) and the exact median over all 134 M pairs.
FULL_N, FULL_D, FULL_ROWS = 16384, 30, 512


def _full_case():
    """The surrogate workload's initial particles (cfg5 scene sampler) and a
    gradient of the rollout's magnitude, FP32-rounded."""
    _, _, th = W.config_problem(5)
    assert th.shape == (FULL_N, FULL_D)
    rng = np.random.default_rng(16384)
    g = W.f32(rng.standard_normal(th.shape) * 20.0)
    rows = np.sort(rng.choice(FULL_N, FULL_ROWS, replace=False))
    rows[0], rows[-1] = 0, FULL_N - 1  # first and last row of the split grid
    return th, g, rows


def test_full_size_median_is_the_exact_order_statistic(ctx):
    import paper_2310_01775_amd as S
    th, g, _ = _full_case()
    print("case N=16384 d=30 exact median", flush=True)
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.svgd_step(S.soa(th), S.soa(g), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    m2 = float(h_out.item()) * math.log(FULL_N)
    ref = svgd.median_sqdist_blocked(th)
    print("median gpu/oracle", m2 / ref, flush=True)
    assert abs(m2 - ref) <= 3e-6 * ref


def test_full_size_fp32_phi_matches_oracle_on_sampled_rows(ctx):
    import paper_2310_01775_amd as S
    th, g, rows = _full_case()
    print("case N=16384 d=30 FP32 phi, 512 rows", flush=True)
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    phi = ctx.svgd_step(S.soa(th), S.soa(g), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    h = float(h_out.item())  # the exact median is checked by the test above
    got = S.aos(phi)[rows]
    ref = svgd.svgd_phi_rows(th, g, h, rows)
    scale = np.abs(ref).max(axis=0, keepdims=True) + 1e-9
    err = (np.abs(got - ref) / scale).max()
    print("phi err (coordinate-scaled)", err, flush=True)
    assert err < 2e-5
    assert np.isfinite(S.aos(phi)).all()


def test_full_size_bf16_phi_matches_oracle_at_its_bandwidth(ctx):
    import paper_2310_01775_amd as S
    th, g, rows = _full_case()
    print("case N=16384 d=30 BF16 phi, 512 rows", flush=True)
    h_out = torch.zeros(1, dtype=torch.float32, device="cuda")
    phi = ctx.svgd_step_bf16(S.soa(th), S.soa(g), 0.0, h_out=h_out)
    torch.cuda.synchronize()
    h = float(h_out.item())
    got = S.aos(phi)[rows]
    ref = svgd.svgd_phi_rows(th, g, h, rows)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("bf16 normwise error", err, flush=True)
    assert err < 2e-2  # the BF16 bar (8-bit significands, FP32 accumulation)
    assert np.isfinite(S.aos(phi)).all()

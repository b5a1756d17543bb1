"""stamp_svgd_step_noalloc (the SVGD step on the library's per-device scratch
array, for callers that cannot allocate) against stamp_svgd_step with a
caller workspace, through the C ABI: two calls in a row, the second on a
smaller input, each equal bit for bit; a step larger than the array is
refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(S, ctx, theta, g, bw, phi, h):
    d, N = theta.shape
    return S._lib.stamp_svgd_step_noalloc(ctx._h, N, d, C.c_void_p(theta.data_ptr()), C.c_void_p(g.data_ptr()),
                                          float(bw), C.c_void_p(phi.data_ptr()), C.c_void_p(h.data_ptr()),
                                          S._stream())


def test_noalloc_step_equals_the_workspace_step_twice(ctx):
    import paper_2310_01775_amd as S
    results = []
    for N, d, bw in [(3000, 30, 0.0), (700, 18, 0.0), (300, 12, 1.7)]:
        print("case", N, d, bw, flush=True)
        rng = np.random.default_rng(N + d)
        theta = S.soa(W.f32(rng.standard_normal((N, d))))
        g = S.soa(W.f32(rng.standard_normal((N, d)) * 10.0))
        phi_a, h_a = torch.empty_like(theta), torch.zeros(1, device="cuda")
        phi_b, h_b = torch.full_like(theta, np.nan), torch.zeros(1, device="cuda")
        ctx.svgd_step(theta, g, bw, phi=phi_a, h_out=h_a)
        assert _noalloc(S, ctx, theta, g, bw, phi_b, h_b) == S.OK
        torch.cuda.synchronize()
        results.append(torch.equal(phi_a, phi_b) and torch.equal(h_a, h_b))
        assert torch.isfinite(phi_b).all()
    assert all(results), results


def test_noalloc_step_refuses_a_step_beyond_its_scratch(ctx):
    import paper_2310_01775_amd as S
    N, d = 4096, 64
    assert S.Context.svgd_workspace_bytes(N, d) > (64 << 20)
    theta = torch.zeros(d, N, device="cuda")
    phi, h = torch.zeros_like(theta), torch.zeros(1, device="cuda")
    assert _noalloc(S, ctx, theta, theta, 0.0, phi, h) == S.ENOSPACE
    assert "no-alloc" in S._lib.stamp_last_error(ctx._h).decode()
    with pytest.raises(S.StampError):
        ctx.svgd_step_noalloc(theta, theta)

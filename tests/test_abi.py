"""The C ABI without a GPU: the library loads, exports every symbol that
include/stamp.h declares, the ctypes structs match the C layout, and the
host-only sizing calls follow the documented layouts."""
import ctypes
import os
import re
import subprocess

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stamp.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(stamp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("stamp_rollout_fwd", "stamp_rollout_adj", "stamp_svgd_step", "stamp_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2310_01775_amd as S
    lib = ctypes.CDLL(S.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(S.EXPORTS) == set(_declared())
    assert "gfx950" in S.version()


def test_struct_layouts_match_the_header(tmp_path):
    import paper_2310_01775_amd as S
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "stamp.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(stamp_scene),'
                    ' sizeof(stamp_cost_w), sizeof(stamp_solver_cfg), offsetof(stamp_scene, goal),'
                    ' offsetof(stamp_scene, eps_r), offsetof(stamp_solver_cfg, ckpt_every),'
                    ' sizeof(stamp_surrogate), offsetof(stamp_surrogate, params), offsetof(stamp_surrogate, enc),'
                    ' sizeof(stamp_surrogate_report));'
                    'printf("%zu %zu %zu\\n", sizeof(stamp_struct_kernel), offsetof(stamp_struct_kernel, kappa),'
                    ' offsetof(stamp_solver_cfg, kernel));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(S.Scene), ctypes.sizeof(S.CostW), ctypes.sizeof(S.SolverCfg),
            S.Scene.goal.offset, S.Scene.eps_r.offset, S.SolverCfg.ckpt_every.offset,
            ctypes.sizeof(S.Surrogate), S.Surrogate.params.offset, S.Surrogate.enc.offset,
            ctypes.sizeof(S.SurrogateReport), ctypes.sizeof(S.StructKernel), S.StructKernel.kappa.offset,
            S.SolverCfg.kernel.offset]
    assert got == want


def _phase_lengths(T, H):
    starts = [-((-k * T) // H) for k in range(H + 1)]
    return [starts[k + 1] - starts[k] for k in range(H)]


@pytest.mark.parametrize("B,H,T,N,K", [(3, 3, 200, 1024, 0), (1, 5, 1000, 4096, 32), (2, 4, 37, 5, 8),
                                       (4, 2, 2, 1, 0), (1, 1, 1, 3, 32)])
def test_tape_and_workspace_sizes(B, H, T, N, K):
    import paper_2310_01775_amd as S
    sc = S.make_scene(W.make_scene(2, 0, B, H, T, 0.005))
    entries = T if K == 0 else sum((L + K - 1) // K for L in _phase_lengths(T, H))
    assert S.Context.tape_floats(sc, N, K) == (entries + H) * 6 * B * 4 * N
    assert S.Context.adj_workspace_bytes(sc, N, K) == (K * 6 * B * 4 * N * 4 if K else 0)
    assert S.Context.svgd_workspace_bytes(N, 6 * H) > 0


def test_sizing_rejects_bad_arguments():
    import paper_2310_01775_amd as S
    sc = S.make_scene(W.make_scene(2, 0, 1, 2, 50, 0.01))
    assert S.Context.tape_floats(sc, 0, 0) == 0
    assert S.Context.tape_floats(sc, 4, -1) == 0
    bad = S.make_scene(W.make_scene(2, 0, 1, 2, 50, 0.01))
    bad.M = 3
    assert S.Context.tape_floats(bad, 4, 0) == 0
    bad = S.make_scene(W.make_scene(2, 0, 1, 2, 50, 0.01))
    bad.T = 1
    assert S.Context.tape_floats(bad, 4, 0) == 0
    assert S.Context.svgd_workspace_bytes(0, 6) == 0
    assert S.Context.svgd_workspace_bytes(16, 65) == 0


def test_null_context_is_rejected():
    import paper_2310_01775_amd as S
    lib = S._lib
    assert lib.stamp_rollout_fwd(None, None, None, 1, None, None, None, 0, 0, None, None) == S.EINVAL
    assert lib.stamp_rollout_adj(None, None, None, 1, None, None, 0, 0, None, None, None, 0, None, None) == S.EINVAL
    assert lib.stamp_svgd_step(None, 1, 1, None, None, 0.0, None, None, None, 0, None) == S.EINVAL
    assert lib.stamp_create(None, 0) == S.EINVAL


def test_mlp_parameter_layout_and_sizing():
    """pack/unpack of the surrogate parameter vector follow the documented
    offsets; the training workspace is defined for multiples of 64 only."""
    import numpy as np
    import paper_2310_01775_amd as S
    src = open(HEADER).read()
    for name, val in (("STAMP_MLP_PARAMS", S.MLP_PARAMS), ("STAMP_MLP_BF16_WEIGHTS", S.MLP_BF16_WEIGHTS),
                      ("STAMP_MLP_WIDTH", S.MLP_WIDTH), ("STAMP_MLP_IN_PAD", S.MLP_IN_PAD),
                      ("STAMP_SCENE_ENC", W.SCENE_ENC)):
        assert re.search(r"#define %s %d\b" % (name, val), src), name
    p = W.mlp_init(54)
    p["b3"] = np.array([0.25])
    flat = S.pack_mlp(p)
    assert flat.shape == (S.MLP_PARAMS,)
    W1 = flat[128:128 + 256 * 64].reshape(256, 64)
    assert np.array_equal(W1[:, :54], p["W1"]) and not W1[:, 54:].any()
    assert np.array_equal(flat[16768:16768 + 65536].reshape(256, 256), p["W2"])
    assert np.array_equal(flat[82560:82816], p["w3"]) and flat[82816] == 0.25
    q = S.unpack_mlp(flat, 54)
    for k in p:
        assert np.array_equal(q[k], p[k]), k
    assert S.Context.mlp_train_workspace_bytes(100) == 0
    assert S.Context.mlp_train_workspace_bytes(64) > 0

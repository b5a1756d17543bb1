"""Python binding of libstamp.so, the gfx950 STAMP SVGD hot path.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  torch supplies device memory and the current HIP stream.  Names follow
include/stamp.h; particle tensors on the device are structure-of-arrays
``[d][N]`` float32 (coordinate-major), see ``soa``/``aos``.

The extension is required: importing this package without a built
``libstamp.so`` raises ImportError (run ``python -m paper_2310_01775_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstamp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_01775_amd.build`")
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOSPACE, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
LAYOUT_AUTO, LAYOUT_BLOCKS, LAYOUT_PACKED = 0, 1, 2
STATUS_NONFINITE_COST, STATUS_NONFINITE_GRAD, STATUS_NONFINITE_PHI, STATUS_BAD_INDEX = 1, 2, 4, 8
MAX_BLOCKS, MAX_PUSHES, MODES = 4, 8, 4


class Scene(C.Structure):
    _fields_ = [("H", C.c_int32), ("M", C.c_int32), ("B", C.c_int32), ("T", C.c_int32),
                ("dt", C.c_float),
                ("half", C.c_float * 4), ("mass", C.c_float * 4), ("mu", C.c_float * 4),
                ("pose0", (C.c_float * 3) * 4), ("goal", C.c_float * 3), ("goal_tol", C.c_float),
                ("k_push", C.c_float), ("k_block", C.c_float), ("sp_beta", C.c_float),
                ("standoff", C.c_float), ("g", C.c_float), ("eps_v_scale", C.c_float),
                ("eps_r", C.c_float)]


class CostW(C.Structure):
    _fields_ = [("target", C.c_float), ("rot", C.c_float), ("traj", C.c_float), ("bound", C.c_float),
                ("o_max", C.c_float), ("d_max", C.c_float), ("traj_eps", C.c_float)]


KERNEL_PUSH = 0  # per action [a_k (4 logits), o_k, D_k]; d = 6K
KERNEL_POSE = 1  # [a_1..a_K, (x, y, phi)_1..K]; d = 7K


class StructKernel(C.Structure):
    _fields_ = [("layout", C.c_int32), ("K", C.c_int32), ("alpha_g", C.c_float), ("alpha_z", C.c_float),
                ("alpha_p", C.c_float), ("h_g", C.c_float), ("h_z", C.c_float), ("kappa", C.c_float)]


def struct_kernel(layout=KERNEL_PUSH, K=1, alpha_g=1.0, alpha_z=1.0, alpha_p=1.0, h_g=0.0, h_z=0.0,
                  kappa=1.0) -> StructKernel:
    """stamp_struct_kernel; h <= 0 selects the per-component median heuristic."""
    return StructKernel(int(layout), int(K), alpha_g, alpha_z, alpha_p, h_g, h_z, kappa)


class SolverCfg(C.Structure):
    _fields_ = [("iters", C.c_int32), ("t0", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("use_adam", C.c_int32),
                ("bandwidth", C.c_float), ("ckpt_every", C.c_int32), ("sgd_iters", C.c_int32),
                ("dsvgd", C.c_int32), ("per_phase", C.c_int32), ("classes", C.c_int32),
                ("kernel", C.POINTER(StructKernel))]


class Surrogate(C.Structure):
    _fields_ = [("iters", C.c_int32), ("n_in", C.c_int32), ("check_every", C.c_int32),
                ("max_log_err", C.c_float), ("phi_bf16", C.c_int32), ("reserved", C.c_int32),
                ("params", C.c_void_p), ("wbf16", C.c_void_p), ("enc", C.c_void_p)]


class SurrogateReport(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("fell_back", C.c_int32), ("checks", C.c_int32),
                ("log_err", C.c_float)]


_vp, _i32, _i64, _f32, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
_P = C.POINTER
_sig = {
    "stamp_create": (_i32, [_P(_vp), _i32]),
    "stamp_destroy": (None, [_vp]),
    "stamp_last_error": (C.c_char_p, [_vp]),
    "stamp_version": (C.c_char_p, []),
    "stamp_set_autotune": (_i32, [_vp, _i32]),
    "stamp_set_launch_shape": (_i32, [_vp, _i32, _i32, _i32]),
    "stamp_set_rollout_layout": (_i32, [_vp, _i32]),
    "stamp_tape_floats": (_sz, [_P(Scene), _i32, _i32]),
    "stamp_adj_workspace_bytes": (_sz, [_P(Scene), _i32, _i32]),
    "stamp_readout_workspace_bytes": (_sz, [_P(Scene), _i32]),
    "stamp_dsvgd_weights": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "stamp_svgd_step_weighted": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, C.c_float, _vp, _vp, _vp, _sz, _vp]),
    "stamp_svgd_bandwidth": (_i32, [_vp, _i32, _i32, _vp, _f32, _vp, _vp, _sz, _vp]),
    "stamp_svgd_direction": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "stamp_svgd_update": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _i32,
                                 _vp, _sz, _vp]),
    "stamp_svgd_step_structured": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _P(StructKernel), _vp, _vp, _vp, _sz,
                                          _vp]),
    "stamp_plan_readout": (_i32, [_vp, _P(Scene), _P(CostW), _i32, _vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "stamp_svgd_workspace_bytes": (_sz, [_i32, _i32]),
    "stamp_solve_workspace_bytes": (_sz, [_i32, _P(Scene), _P(_i32), _P(SolverCfg)]),
    "stamp_rollout_fwd": (_i32, [_vp, _P(Scene), _P(CostW), _i32, _vp, _vp, _vp, _sz, _i32, _vp, _vp]),
    "stamp_rollout_adj": (_i32, [_vp, _P(Scene), _P(CostW), _i32, _vp, _vp, _sz, _i32, _vp, _vp, _vp, _sz,
                                 _vp, _vp]),
    "stamp_rollout_adj_phases": (_i32, [_vp, _P(Scene), _P(CostW), _i32, _vp, _vp, _sz, _i32, _vp, _vp, _vp,
                                        _sz, _vp, _vp]),
    "stamp_svgd_step": (_i32, [_vp, _i32, _i32, _vp, _vp, _f32, _vp, _vp, _vp, _sz, _vp]),
    "stamp_svgd_step_bf16": (_i32, [_vp, _i32, _i32, _vp, _vp, _f32, _vp, _vp, _vp, _sz, _vp]),
    "stamp_svgd_step_noalloc": (_i32, [_vp, _i32, _i32, _vp, _vp, _f32, _vp, _vp, _vp]),
    "stamp_adam_step": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _i32, _vp]),
    "stamp_solve": (_i32, [_vp, _i32, _P(Scene), _P(CostW), _P(_i32), _P(SolverCfg), _vp, _vp, _vp, _vp,
                           _vp, _vp, _vp, _sz, _vp, _vp]),
    "stamp_mlp_prepare": (_i32, [_vp, _vp, _vp, _vp]),
    "stamp_mlp_standardize": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "stamp_mlp_label": (_i32, [_vp, _P(Scene), _P(CostW), _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "stamp_mlp_forward": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _P(CostW), _vp, _vp, _vp, _f32,
                                 _vp]),
    "stamp_mlp_train_workspace_bytes": (_sz, [_i32]),
    "stamp_mlp_train_step": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _i32, _f32, _f32,
                                    _f32, _f32, _vp, _vp, _vp, _sz, _vp]),
    "stamp_mlp_train_steps": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _i32,
                                     _P(_f32), _f32, _f32, _f32, _vp, _vp, _vp, _sz, _vp]),
    "stamp_solve_surrogate": (_i32, [_vp, _i32, _P(Scene), _P(CostW), _P(_i32), _P(SolverCfg), _P(Surrogate), _vp,
                                     _vp, _vp, _vp, _vp, _vp, _P(SurrogateReport), _vp, _sz, _vp, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = tuple(_sig)


class StampError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stamp error {code}: {msg}")
        self.code = code


def version() -> str:
    return _lib.stamp_version().decode()


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def make_scene(d: dict) -> Scene:
    """stamp_scene from a scene dict (keys as in workloads.make_scene)."""
    s = Scene()
    s.H, s.M, s.B, s.T = int(d["H"]), int(d.get("M", 4)), int(d["B"]), int(d["T"])
    s.dt = d["dt"]
    for b in range(s.B):
        s.half[b], s.mass[b], s.mu[b] = d["half"][b], d["mass"][b], d["mu"][b]
        for q in range(3):
            s.pose0[b][q] = d["pose0"][b][q]
    for q in range(3):
        s.goal[q] = d["goal"][q]
    for k in ("goal_tol", "k_push", "k_block", "sp_beta", "standoff", "g", "eps_v_scale", "eps_r"):
        setattr(s, k, d[k])
    return s


def make_cost(w: dict) -> CostW:
    c = CostW()
    for k, _ in CostW._fields_:
        setattr(c, k, w[k])
    return c


def make_cfg(iters, t0=0, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, use_adam=True,
             bandwidth=0.0, ckpt_every=0, sgd_iters=0, dsvgd=False, kernel=None, per_phase=False,
             classes=0) -> SolverCfg:
    """stamp_solver_cfg; kernel: a StructKernel (push layout) or None for the RBF kernel on theta;
    per_phase: the simulator iterations take the gradient of the per-phase split of the cost;
    classes > 1: the problems of a solve run in that many cost classes, cheapest first."""
    cfg = SolverCfg(int(iters), int(t0), lr, beta1, beta2, adam_eps, int(bool(use_adam)), bandwidth,
                    int(ckpt_every), int(sgd_iters), int(bool(dsvgd)), int(bool(per_phase)), int(classes))
    if kernel is not None:
        cfg.kernel = C.pointer(kernel)
        cfg._kernel_ref = kernel  # keeps the pointed-to struct alive with the cfg
    return cfg


def soa(theta_nd, device="cuda") -> torch.Tensor:
    """[N][d] host particles -> contiguous float32 [d][N] device tensor."""
    t = torch.as_tensor(np.asarray(theta_nd), dtype=torch.float32)
    return t.t().contiguous().to(device)


def aos(theta_dn: torch.Tensor) -> np.ndarray:
    """[d][N] device tensor -> [N][d] float64 numpy (host)."""
    return theta_dn.detach().to("cpu", torch.float64).t().contiguous().numpy()


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous CUDA/HIP tensors")
    # every array of the C ABI holds 4-byte (float32, int32) or narrower
    # elements: a float64 array (say one made from numpy without a dtype) would
    # be read as garbage
    if t.element_size() > 4:
        raise ValueError("the C ABI takes float32/int32 (or narrower) arrays, got %s" % t.dtype)
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# Surrogate network parameter vector (layout of include/stamp.h).
MLP_WIDTH, MLP_IN_PAD, MLP_PARAMS, MLP_BF16_WEIGHTS = 256, 64, 82817, 163840
_MLP_FIELDS = (("mu", (MLP_IN_PAD,)), ("inv_sigma", (MLP_IN_PAD,)), ("W1", (MLP_WIDTH, MLP_IN_PAD)),
               ("b1", (MLP_WIDTH,)), ("W2", (MLP_WIDTH, MLP_WIDTH)), ("b2", (MLP_WIDTH,)),
               ("w3", (MLP_WIDTH,)), ("b3", (1,)))


def pack_mlp(params: dict) -> np.ndarray:
    """Dict of arrays (W1 as [256][n_in], mu/inv_sigma [n_in]) -> the flat
    float32 parameter vector, inputs padded to 64 with zeros."""
    out = np.zeros(MLP_PARAMS, dtype=np.float32)
    off = 0
    for name, shape in _MLP_FIELDS:
        size = int(np.prod(shape))
        v = np.asarray(params[name], dtype=np.float32)
        blk = np.zeros(shape, dtype=np.float32)
        blk[tuple(slice(0, n) for n in v.shape)] = v
        out[off:off + size] = blk.ravel()
        off += size
    assert off == MLP_PARAMS
    return out


def unpack_mlp(flat, n_in: int) -> dict:
    """The flat parameter vector -> dict of float64 arrays cut to n_in inputs."""
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, shape in _MLP_FIELDS:
        size = int(np.prod(shape))
        v = flat[off:off + size].reshape(shape)
        if name in ("mu", "inv_sigma"):
            v = v[:n_in]
        elif name == "W1":
            v = v[:, :n_in]
        out[name] = v.copy()
        off += size
    return out


# ---------------------------------------------------------------------------
class Context:
    """One library context on a device (not thread-safe)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        rc = _lib.stamp_create(C.byref(h), int(device))
        if rc != OK:
            raise StampError(rc, "stamp_create failed")
        self._h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if self._h:
            _lib.stamp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_autotune(self, enable: bool):
        self._check(_lib.stamp_set_autotune(self._h, int(bool(enable))))

    def set_rollout_layout(self, layout: int):
        """stamp_set_rollout_layout: LAYOUT_AUTO, LAYOUT_BLOCKS or LAYOUT_PACKED."""
        self._check(_lib.stamp_set_rollout_layout(self._h, int(layout)))

    def set_launch_shape(self, roll_block=0, roll_grid=0, phi_rows=0):
        self._check(_lib.stamp_set_launch_shape(self._h, int(roll_block), int(roll_grid), int(phi_rows)))

    def _check(self, rc):
        if rc != OK:
            raise StampError(rc, _lib.stamp_last_error(self._h).decode())

    # -- sizing --------------------------------------------------------------
    @staticmethod
    def tape_floats(scene: Scene, N: int, ckpt_every: int = 0) -> int:
        return int(_lib.stamp_tape_floats(C.byref(scene), N, ckpt_every))

    @staticmethod
    def adj_workspace_bytes(scene: Scene, N: int, ckpt_every: int = 0) -> int:
        return int(_lib.stamp_adj_workspace_bytes(C.byref(scene), N, ckpt_every))

    @staticmethod
    def svgd_workspace_bytes(N: int, d: int) -> int:
        return int(_lib.stamp_svgd_workspace_bytes(N, d))

    @staticmethod
    def solve_workspace_bytes(scenes, Ns, cfg: SolverCfg) -> int:
        arr = (Scene * len(scenes))(*scenes)
        ns = (C.c_int32 * len(Ns))(*Ns)
        return int(_lib.stamp_solve_workspace_bytes(len(scenes), arr, ns, C.byref(cfg)))

    def _bytes(self, n):
        return torch.empty(max(int(n), 1), dtype=torch.uint8, device=self.device)

    def status_word(self):
        return torch.zeros(1, dtype=torch.int32, device=self.device)

    # -- hot path -------------------------------------------------------------
    @staticmethod
    def _particles(scene: Scene, theta: torch.Tensor) -> int:
        """Checks theta is float32 [6H][N] for this scene; returns N."""
        if theta.dtype != torch.float32 or theta.dim() != 2 or theta.shape[0] != 6 * int(scene.H):
            raise ValueError("theta must be float32 [6H][N] = [%d][N], got %s %s"
                             % (6 * int(scene.H), theta.dtype, tuple(theta.shape)))
        return int(theta.shape[1])

    @staticmethod
    def _vec(t, n: int, what: str):
        """Checks an optional float32 device array holds n floats."""
        if t is not None and (t.dtype != torch.float32 or t.numel() != n):
            raise ValueError("%s must be %d float32, got %s with %d elements" % (what, n, t.dtype, t.numel()))

    def _tape(self, scene: Scene, N: int, ckpt_every: int, tape):
        if tape is None:
            return 0
        need = self.tape_floats(scene, N, ckpt_every)
        if tape.dtype != torch.float32 or tape.numel() < need:
            raise ValueError("tape must hold >= %d float32 for ckpt_every=%d, got %s with %d elements"
                             % (need, ckpt_every, tape.dtype, tape.numel()))
        return tape.numel()

    def rollout_fwd(self, scene: Scene, w: CostW, theta: torch.Tensor, tape=None, ckpt_every: int = 0,
                    status=None, stream=None, cost=None):
        N = self._particles(scene, theta)
        if cost is None:
            cost = torch.empty(N, dtype=torch.float32, device=self.device)
        self._vec(cost, N, "cost")
        n_tape = self._tape(scene, N, ckpt_every, tape)
        self._check(_lib.stamp_rollout_fwd(self._h, C.byref(scene), C.byref(w), N, _ptr(theta), _ptr(cost),
                                           _ptr(tape), n_tape, ckpt_every, _ptr(status), _stream(stream)))
        return cost

    def dsvgd_weights(self, cost_relaxed, cost_discrete, weights=None, stream=None):
        """stamp_dsvgd_weights: importance weights [N] (mean 1) of Eq. (4)."""
        for t in (cost_relaxed, cost_discrete):
            if t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("costs must be contiguous float32")
        N = cost_relaxed.numel()
        if cost_discrete.numel() != N:
            raise ValueError("cost arrays differ in length")
        if weights is None:
            weights = torch.empty(N, dtype=torch.float32, device=self.device)
        self._check(_lib.stamp_dsvgd_weights(self._h, N, _ptr(cost_relaxed), _ptr(cost_discrete), _ptr(weights),
                                             _stream(stream)))
        return weights

    def svgd_step_weighted(self, theta, grad_logp, weights, bandwidth: float = 0.0, phi=None, h_out=None,
                           workspace=None, stream=None):
        d, N = theta.shape
        if weights.dtype != torch.float32 or weights.numel() != N or not weights.is_contiguous():
            raise ValueError("weights must be N contiguous float32")
        if phi is None:
            phi = torch.empty_like(theta)
        if workspace is None:
            workspace = self._bytes(self.svgd_workspace_bytes(N, d))
        self._check(_lib.stamp_svgd_step_weighted(self._h, N, d, _ptr(theta), _ptr(grad_logp), _ptr(weights),
                                                  float(bandwidth), _ptr(phi), _ptr(h_out), _ptr(workspace),
                                                  workspace.numel(), _stream(stream)))
        return phi

    def svgd_bandwidth(self, theta, bandwidth: float = 0.0, h_out=None, workspace=None, stream=None):
        """stamp_svgd_bandwidth: the first half of svgd_step; returns the workspace."""
        d, N = theta.shape
        if workspace is None:
            workspace = self._bytes(self.svgd_workspace_bytes(N, d))
        self._check(_lib.stamp_svgd_bandwidth(self._h, N, d, _ptr(theta), float(bandwidth), _ptr(h_out),
                                              _ptr(workspace), workspace.numel(), _stream(stream)))
        return workspace

    def svgd_direction(self, theta, grad_logp, workspace, weights=None, phi=None, stream=None):
        """stamp_svgd_direction: phi from the bandwidth the workspace holds."""
        d, N = theta.shape
        if phi is None:
            phi = torch.empty_like(theta)
        self._check(_lib.stamp_svgd_direction(self._h, N, d, _ptr(theta), _ptr(grad_logp), _ptr(weights), _ptr(phi),
                                              _ptr(workspace), workspace.numel(), _stream(stream)))
        return phi

    def svgd_update(self, theta, grad_logp, workspace, m, v, t: int, lr: float = 1e-3, beta1: float = 0.9,
                    beta2: float = 0.999, eps: float = 1e-8, use_adam: bool = True, weights=None, phi=None,
                    stream=None):
        """stamp_svgd_update: direction from the workspace's bandwidth, then the update of theta in place."""
        d, N = theta.shape
        self._check(_lib.stamp_svgd_update(self._h, N, d, _ptr(theta), _ptr(grad_logp), _ptr(weights), _ptr(phi),
                                           _ptr(m), _ptr(v), int(t), float(lr), float(beta1), float(beta2),
                                           float(eps), int(bool(use_adam)), _ptr(workspace), workspace.numel(),
                                           _stream(stream)))
        return theta

    def svgd_step_structured(self, theta, grad_logp, kernel: StructKernel, weights=None, phi=None, h_out=None,
                             workspace=None, stream=None):
        """stamp_svgd_step_structured: phi [d][N]; h_out (2 floats) receives (h_g, h_z)."""
        d, N = theta.shape
        for t in (theta, grad_logp) + ((weights,) if weights is not None else ()):
            if t.dtype != torch.float32:
                raise ValueError("theta, grad_logp and weights must be float32")
        if weights is not None and weights.numel() != N:
            raise ValueError("weights must hold N floats")
        if phi is None:
            phi = torch.empty_like(theta)
        if workspace is None:
            workspace = self._bytes(self.svgd_workspace_bytes(N, d))
        self._check(_lib.stamp_svgd_step_structured(self._h, N, d, _ptr(theta), _ptr(grad_logp), _ptr(weights),
                                                    C.byref(kernel), _ptr(phi), _ptr(h_out), _ptr(workspace),
                                                    workspace.numel(), _stream(stream)))
        return phi

    def plan_readout(self, scene: Scene, w: CostW, theta: torch.Tensor, modes=None, cost=None, workspace=None,
                     status=None, stream=None):
        """stamp_plan_readout: (modes [H][N] int32, cost [N] of the discrete plans)."""
        N = theta.shape[1]
        H = int(scene.H)
        if modes is None:
            modes = torch.empty((H, N), dtype=torch.int32, device=self.device)
        if cost is None:
            cost = torch.empty(N, dtype=torch.float32, device=self.device)
        if workspace is None:
            workspace = self._bytes(int(_lib.stamp_readout_workspace_bytes(C.byref(scene), N)))
        self._check(_lib.stamp_plan_readout(self._h, C.byref(scene), C.byref(w), N, _ptr(theta), _ptr(modes),
                                            _ptr(cost), _ptr(workspace), workspace.numel(), _ptr(status),
                                            _stream(stream)))
        return modes, cost

    def rollout_adj(self, scene: Scene, w: CostW, theta: torch.Tensor, tape: torch.Tensor,
                    ckpt_every: int = 0, cost_bar=None, grad=None, workspace=None, status=None, stream=None,
                    per_phase: bool = False):
        """stamp_rollout_adj (cost_bar * dC/dtheta), or with per_phase
        stamp_rollout_adj_phases (the gradient of the per-phase split)."""
        N = self._particles(scene, theta)
        if grad is None:
            grad = torch.empty_like(theta)
        self._vec(grad, theta.numel(), "grad")
        self._vec(cost_bar, N, "cost_bar")
        if tape is None:
            raise ValueError("the adjoint needs the forward's tape")
        n_tape = self._tape(scene, N, ckpt_every, tape)
        need = self.adj_workspace_bytes(scene, N, ckpt_every)
        if workspace is None and need:
            workspace = self._bytes(need)
        ws_bytes = workspace.numel() if workspace is not None else 0
        fn = _lib.stamp_rollout_adj_phases if per_phase else _lib.stamp_rollout_adj
        self._check(fn(self._h, C.byref(scene), C.byref(w), N, _ptr(theta), _ptr(tape), n_tape, ckpt_every,
                       _ptr(cost_bar), _ptr(grad), _ptr(workspace), ws_bytes, _ptr(status), _stream(stream)))
        return grad

    def svgd_step(self, theta: torch.Tensor, grad_logp: torch.Tensor, bandwidth: float = 0.0, phi=None,
                  h_out=None, workspace=None, stream=None):
        d, N = theta.shape
        if phi is None:
            phi = torch.empty_like(theta)
        if workspace is None:
            workspace = self._bytes(self.svgd_workspace_bytes(N, d))
        self._check(_lib.stamp_svgd_step(self._h, N, d, _ptr(theta), _ptr(grad_logp), float(bandwidth),
                                         _ptr(phi), _ptr(h_out), _ptr(workspace), workspace.numel(),
                                         _stream(stream)))
        return phi

    def svgd_step_noalloc(self, theta: torch.Tensor, grad_logp: torch.Tensor, bandwidth: float = 0.0, phi=None,
                          h_out=None, stream=None):
        """stamp_svgd_step_noalloc: the step without a workspace (the library's
        per-device scratch array; calls on one GPU must not overlap)."""
        d, N = theta.shape
        for t in (theta, grad_logp):
            if t.dtype != torch.float32 or t.shape != (d, N):
                raise ValueError("theta and grad_logp must be float32 [d][N]")
        if phi is None:
            phi = torch.empty_like(theta)
        self._check(_lib.stamp_svgd_step_noalloc(self._h, N, d, _ptr(theta), _ptr(grad_logp), float(bandwidth),
                                                 _ptr(phi), _ptr(h_out), _stream(stream)))
        return phi

    def svgd_step_bf16(self, theta: torch.Tensor, grad_logp: torch.Tensor, bandwidth: float = 0.0, phi=None,
                       h_out=None, workspace=None, stream=None):
        d, N = theta.shape
        if phi is None:
            phi = torch.empty_like(theta)
        if workspace is None:
            workspace = self._bytes(self.svgd_workspace_bytes(N, d))
        self._check(_lib.stamp_svgd_step_bf16(self._h, N, d, _ptr(theta), _ptr(grad_logp), float(bandwidth),
                                              _ptr(phi), _ptr(h_out), _ptr(workspace), workspace.numel(),
                                              _stream(stream)))
        return phi

    def adam_step(self, theta, phi, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, use_adam=True,
                  stream=None):
        self._check(_lib.stamp_adam_step(self._h, theta.numel(), _ptr(theta), _ptr(phi), _ptr(m), _ptr(v),
                                         int(t), lr, beta1, beta2, eps, int(bool(use_adam)), _stream(stream)))

    def solve(self, scenes, ws_, Ns, cfg: SolverCfg, theta, adam_m=None, adam_v=None, cost_out=None,
              modes_out=None, solve_time_us=None, workspace=None, status=None, stream=None):
        n = len(scenes)
        arr = (Scene * n)(*scenes)
        warr = (CostW * n)(*ws_)
        ns = (C.c_int32 * n)(*Ns)
        if cost_out is None:
            cost_out = torch.empty(sum(Ns), dtype=torch.float32, device=self.device)
        if workspace is None:
            workspace = self._bytes(self.solve_workspace_bytes(scenes, Ns, cfg))
        self._check(_lib.stamp_solve(self._h, n, arr, warr, ns, C.byref(cfg), _ptr(theta), _ptr(adam_m),
                                     _ptr(adam_v), _ptr(cost_out), _ptr(modes_out), _ptr(solve_time_us),
                                     _ptr(workspace), workspace.numel(), _ptr(status), _stream(stream)))
        return cost_out

    # -- learned cost surrogate -------------------------------------------------
    def mlp_weights(self):
        """An uninitialised buffer for the BF16 working copies."""
        return torch.empty(MLP_BF16_WEIGHTS, dtype=torch.bfloat16, device=self.device)

    @staticmethod
    def _mlp_buffers(params, wbf16, *moments):
        if params.dtype != torch.float32 or params.numel() < MLP_PARAMS:
            raise ValueError("params must hold %d float32" % MLP_PARAMS)
        if wbf16.dtype != torch.bfloat16 or wbf16.numel() < MLP_BF16_WEIGHTS:
            raise ValueError("wbf16 must hold %d bfloat16" % MLP_BF16_WEIGHTS)
        for t in moments:
            if t.dtype != torch.float32 or t.numel() < MLP_PARAMS:
                raise ValueError("Adam moments must hold %d float32" % MLP_PARAMS)

    def mlp_prepare(self, params: torch.Tensor, wbf16: torch.Tensor, stream=None):
        self._mlp_buffers(params, wbf16)
        self._check(_lib.stamp_mlp_prepare(self._h, _ptr(params), _ptr(wbf16), _stream(stream)))

    def mlp_standardize(self, params, x, cost=None, stream=None):
        """Set params' mu / inv_sigma from the rows of x [M][n_in] (and b3 from
        the mean target log(1 + cost) when cost [M] is given)."""
        if params.dtype != torch.float32 or params.numel() < MLP_PARAMS:
            raise ValueError("params must hold %d float32" % MLP_PARAMS)
        M, n_in = x.shape
        if cost is not None and tuple(cost.shape) != (M,):
            raise ValueError("cost must be [M]")
        self._check(_lib.stamp_mlp_standardize(self._h, M, n_in, _ptr(x), _ptr(cost), _ptr(params),
                                               _stream(stream)))

    def mlp_label(self, scene: Scene, w: CostW, theta, n_in: int, enc=None, x=None, cost=None, status=None,
                  stream=None):
        """Rollout part of the cost of theta [d][N] and the network inputs
        [N][n_in] = [theta_i, enc]; returns (x, cost)."""
        d, N = theta.shape
        if x is None:
            x = torch.empty((N, n_in), dtype=torch.float32, device=self.device)
        if cost is None:
            cost = torch.empty(N, dtype=torch.float32, device=self.device)
        if tuple(x.shape) != (N, n_in) or tuple(cost.shape) != (N,):
            raise ValueError("x must be [N][n_in] and cost [N]")
        if n_in > d and (enc is None or enc.numel() < n_in - d):
            raise ValueError("enc needs n_in - d floats")
        self._check(_lib.stamp_mlp_label(self._h, C.byref(scene), C.byref(w), N, _ptr(theta), n_in, _ptr(enc),
                                         _ptr(x), _ptr(cost), _ptr(status), _stream(stream)))
        return x, cost

    def mlp_forward(self, params, wbf16, x, n_in: int, d: int, x_layout: int = 0, enc=None, want_y=True,
                    want_cost=False, want_grad=False, grad_scale: float = 1.0, grad=None, w: CostW = None,
                    cost=None, stream=None):
        """x [M][n_in] (x_layout 0) or [d][M] (x_layout 1).  Returns (y, cost, grad)
        with None for what was not asked; grad is [d][M] (written into `grad`
        when given, which implies want_grad).  w adds the exact bound term."""
        self._mlp_buffers(params, wbf16)
        if x_layout == 1 and n_in > d and (enc is None or enc.numel() < n_in - d):
            raise ValueError("enc needs n_in - d = %d floats" % (n_in - d))
        M = x.shape[0] if x_layout == 0 else x.shape[1]
        if x.shape != ((M, n_in) if x_layout == 0 else (d, M)):
            raise ValueError("x has shape %s, expected %s" % (tuple(x.shape), (M, n_in) if x_layout == 0 else (d, M)))
        y = torch.empty(M, dtype=torch.float32, device=self.device) if want_y else None
        c = cost
        if c is None and want_cost:
            c = torch.empty(M, dtype=torch.float32, device=self.device)
        g = grad
        if g is None and want_grad:
            g = torch.empty((d, M), dtype=torch.float32, device=self.device)
        if g is not None and tuple(g.shape) != (d, M):
            raise ValueError("grad must be [d][M]")
        self._check(_lib.stamp_mlp_forward(self._h, M, n_in, d, _ptr(params), _ptr(wbf16), _ptr(x), int(x_layout),
                                           _ptr(enc), C.byref(w) if w is not None else None, _ptr(y), _ptr(c),
                                           _ptr(g), float(grad_scale), _stream(stream)))
        return y, c, g

    @staticmethod
    def mlp_train_workspace_bytes(M: int) -> int:
        return int(_lib.stamp_mlp_train_workspace_bytes(M))

    def mlp_train_step(self, params, wbf16, adam_m, adam_v, x, cost, t, idx=None, M=None, lr=1e-3, beta1=0.9,
                       beta2=0.999, eps=1e-8, loss=None, status=None, workspace=None, stream=None):
        """One Adam step on the minibatch rows idx (int32 [M]) of the dataset
        x [n_rows][n_in], cost [n_rows] (targets log(1 + cost)); without idx
        the first M rows (M defaults to n_rows)."""
        self._mlp_buffers(params, wbf16, adam_m, adam_v)
        n_rows, n_in = x.shape
        if tuple(cost.shape) != (n_rows,):
            raise ValueError("cost must be [n_rows]")
        if idx is not None:
            if idx.dtype != torch.int32:
                raise ValueError("idx must be int32")
            M = idx.numel()
        elif M is None:
            M = n_rows
        if workspace is None:
            workspace = self._bytes(self.mlp_train_workspace_bytes(M))
        self._check(_lib.stamp_mlp_train_step(self._h, M, n_in, _ptr(x), _ptr(cost), _ptr(idx), n_rows, _ptr(params),
                                              _ptr(wbf16), _ptr(adam_m), _ptr(adam_v), int(t), lr, beta1, beta2, eps,
                                              _ptr(loss), _ptr(status), _ptr(workspace), workspace.numel(),
                                              _stream(stream)))

    def mlp_train_steps(self, params, wbf16, adam_m, adam_v, x, cost, t0, idx, lr, beta1=0.9, beta2=0.999,
                        eps=1e-8, loss=None, status=None, workspace=None, stream=None):
        """len(lr) consecutive Adam steps t0+1.. in one call: step s on the rows
        idx[s] (int32 [n_steps][M]) with learning rate lr[s]; loss (float32
        [n_steps], optional) receives each step's loss before its update."""
        self._mlp_buffers(params, wbf16, adam_m, adam_v)
        n_rows, n_in = x.shape
        if tuple(cost.shape) != (n_rows,):
            raise ValueError("cost must be [n_rows]")
        if idx.dtype != torch.int32 or idx.dim() != 2 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int32 [n_steps][M] tensor")
        n_steps, M = idx.shape
        if len(lr) != n_steps:
            raise ValueError("one learning rate per step")
        if loss is not None and (loss.dtype != torch.float32 or loss.numel() < n_steps):
            raise ValueError("loss must hold n_steps float32")
        if workspace is None:
            workspace = self._bytes(self.mlp_train_workspace_bytes(M))
        lrs = (C.c_float * n_steps)(*[float(v) for v in lr])
        self._check(_lib.stamp_mlp_train_steps(self._h, n_steps, M, n_in, _ptr(x), _ptr(cost), _ptr(idx), n_rows,
                                               _ptr(params), _ptr(wbf16), _ptr(adam_m), _ptr(adam_v), int(t0), lrs,
                                               beta1, beta2, eps, _ptr(loss), _ptr(status), _ptr(workspace),
                                               workspace.numel(), _stream(stream)))

    def solve_surrogate(self, scenes, ws_, Ns, cfg: SolverCfg, sur_iters: int, params, wbf16, n_in: int, enc,
                        theta, adam_m=None, adam_v=None, check_every: int = 0, max_log_err: float = 0.0,
                        phi_bf16: bool = False, cost_out=None, modes_out=None, solve_time_us=None, workspace=None, status=None,
                        stream=None):
        """stamp_solve_surrogate: returns (cost_out, report)."""
        self._mlp_buffers(params, wbf16)
        n = len(scenes)
        arr = (Scene * n)(*scenes)
        warr = (CostW * n)(*ws_)
        ns = (C.c_int32 * n)(*Ns)
        if cost_out is None:
            cost_out = torch.empty(sum(Ns), dtype=torch.float32, device=self.device)
        if workspace is None:
            workspace = self._bytes(self.solve_workspace_bytes(scenes, Ns, cfg))
        need_enc = sum(max(0, n_in - 6 * sc.H) for sc in scenes)
        if need_enc and (enc is None or enc.numel() < need_enc):
            raise ValueError("enc needs %d floats" % need_enc)
        sur = Surrogate(int(sur_iters), int(n_in), int(check_every), float(max_log_err), int(bool(phi_bf16)), 0,
                        _ptr(params), _ptr(wbf16), _ptr(enc))
        rep = SurrogateReport()
        self._check(_lib.stamp_solve_surrogate(self._h, n, arr, warr, ns, C.byref(cfg), C.byref(sur), _ptr(theta),
                                               _ptr(adam_m), _ptr(adam_v), _ptr(cost_out), _ptr(modes_out),
                                               _ptr(solve_time_us), C.byref(rep), _ptr(workspace), workspace.numel(),
                                               _ptr(status), _stream(stream)))
        return cost_out, rep

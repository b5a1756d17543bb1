"""Benchmark of the STAMP SVGD hot path on one MI355X.

Default line -- the metric's own workload: SVGD particle-iterations/s of the
learned-surrogate form against the plain method at equal final cost, on the
N = 16384, B = 3, H = 5 (d = 30), T = 200 scene.  One step is one complete
300-iteration solve (Algorithm 1's SVGD phase with Adam) in the surrogate form:
the network's gradient drives iterations 0..239 (BF16 direction), the simulator
(rollout forward + adjoint, exact median, FP32 direction) iterations 240..299,
all in the library's HIP kernels, graph-replayed by stamp_solve_surrogate.
The plain method (300 simulator iterations) is timed the same way beside it.

value = N * 300 * steps / wall seconds of the timed surrogate-form solves
(inputs resident in HBM, synchronised on both sides).  The network is trained
by the library's own kernels first; that time is reported apart.  The
dominant kernel's duration comes from HIP events on the stream it is launched
on, around per-call launches of the same kernel at the same shape.
cpu_baseline times the FP64 oracle on bounded samples of each stage and
extrapolates to one solve.  --workload selects the other measurements.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SVGD particle-iters/s incl. sim fwd+adjoint; surrogate vs plain at equal cost"
UNIT = "particle-iters/s"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0    # MI355X published dense BF16 matrix peak


def rollout_bytes(N, d, B, T, H):
    """Algorithmic HBM bytes of one forward and one adjoint launch with the
    full tape.  Per particle: theta (4d), the tape -- the pre-step state of
    every step (T) plus the H phase-end states, 6 floats per block, for each of
    the 4 side sub-rollouts the phase mixture runs -- written by the forward
    and read once by the adjoint, and the output (cost 4 B; grad 4d)."""
    tape = (T + H) * 6 * B * 4 * 4
    return N * (4 * d + tape + 4), N * (4 * d + tape + 4 * d)


def rollout_bytes_single_trajectory(N, d, B, T):
    """The same count for one trajectory per particle (24 B (T+1) per block):
    the tape a rollout without the phase mixture would keep."""
    return N * (4 * d + 24 * B * (T + 1) + 4 * d)


def phi_flops(N, d):
    """Algorithmic flops of the SVGD contraction: the Gram distances (2d per
    pair) and K.[g - (2/h)x | 1] (2(d+1) per pair) over all N^2 pairs."""
    return N * N * (2 * d + 2 * (d + 1))


def split3_mfma_flops(N):
    """Matrix-core flops the split form of the FP32 direction (d <= 31)
    executes per launch: for each pair, six BF16 part products of the 32-wide
    Gram and six of the 32-column K.V, 2 flops per multiply-add."""
    npad = (N + 255) // 256 * 256
    return npad * npad * (6 * 2 * 32 + 6 * 2 * 32)


def mlp_flops(M, n_in, width=256):
    """Forward + input gradient of the 3-layer surrogate network per launch."""
    return M * 2 * 2 * (n_in * width + width * width + width)


PROFILE = os.path.join(ROOT, "profiles", "stages_n16384_counters.md")


def kernel_source_hash():
    """SHA-256 (first 16 hex digits) of every kernel source, *.hip then *.h in
    name order, with comments and blank lines left out (they change no
    kernel): the counters in PROFILE hold only while it matches."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_01775_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip"))) + sorted(glob.glob(os.path.join(csrc, "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(f).read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the plain-copy calibration),
    or None when the summary is missing or the kernel sources changed since."""
    if not os.path.exists(PROFILE):
        return None
    fields = {}
    for line in open(PROFILE):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256_16") != kernel_source_hash():
        return None
    v = fields.get(f"{kernel}_hbm_bytes_per_launch")
    return float(v) if v else None


def _host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def _oracle_stage_times(net_params, enc, scene, w, th, iters, s_iters):
    """Seconds per particle / row / call of each stage of the FP64 oracle on
    bounded samples of the N = 16384 workload, and the solve time they
    extrapolate to (s_iters surrogate iterations + the rest plain)."""
    import numpy as np

    from oracle import mlp, sim, svgd

    N, d = th.shape
    rng = np.random.default_rng(0)
    t = {}
    ns = 4096
    x = th[rng.choice(N, ns, replace=False)]
    t0 = time.perf_counter()
    sim.cost_and_grad(scene, w, x)
    t["sim_per_particle"] = (time.perf_counter() - t0) / ns
    nm = N
    t0 = time.perf_counter()
    mlp.surrogate_cost_and_grad(net_params, th[:nm], enc, w)
    t["mlp_per_particle"] = (time.perf_counter() - t0) / nm
    g = rng.standard_normal(th.shape) * 20.0
    nr = 8192
    t0 = time.perf_counter()
    svgd.svgd_phi_rows(th, g, 1.0, np.arange(nr))
    t["phi_per_row"] = (time.perf_counter() - t0) / nr
    nmed = N
    t0 = time.perf_counter()
    svgd.median_sqdist_blocked(th[:nmed])
    t["median_per_pair"] = (time.perf_counter() - t0) / (nmed * (nmed - 1) / 2)
    m = np.zeros_like(th)
    t0 = time.perf_counter()
    svgd.adam_step(th, g, m, m, 1, 1e-3)
    t["adam_per_call"] = time.perf_counter() - t0
    shared = N * t["phi_per_row"] + N * (N - 1) / 2 * t["median_per_pair"] + t["adam_per_call"]
    it_plain = N * t["sim_per_particle"] + shared
    it_sur = N * t["mlp_per_particle"] + shared
    t["solve_s"] = s_iters * it_sur + (iters - s_iters) * it_plain
    t["plain_solve_s"] = iters * it_plain
    return t


def cpu_baseline_surrogate(net_params, enc, scene, w, th, iters, s_iters):
    """The FP64 oracle as it stands, timed on bounded samples of every stage of
    the surrogate-form solve and extrapolated per iteration to N = 16384: the
    rollout + autodiff gradient on 4096 particles, the network's cost + input
    gradient on all N, the SVGD direction on 8192 rows against all N, the exact
    median over all pairs, Adam on all of theta; once on every host core and once on one."""
    import torch
    from threadpoolctl import threadpool_limits

    from oracle import mlp, sim

    model, avail = _host_cpu()
    torch.set_num_threads(avail)
    sim.cost_and_grad(scene, w, th[:2])  # first-use costs of torch and numpy stay out of the timing
    mlp.surrogate_cost_and_grad(net_params, th[:16], enc, w)
    t0 = time.perf_counter()
    allc = _oracle_stage_times(net_params, enc, scene, w, th, iters, s_iters)
    wall_all = time.perf_counter() - t0
    with threadpool_limits(1):
        torch.set_num_threads(1)
        t0 = time.perf_counter()
        one = _oracle_stage_times(net_params, enc, scene, w, th, iters, s_iters)
        wall_one = time.perf_counter() - t0
    torch.set_num_threads(avail)
    N = th.shape[0]
    return {"value": N * iters / allc["solve_s"], "unit": UNIT, "cores": avail, "kind": "oracle",
            "extrapolated": True, "value_1core": N * iters / one["solve_s"],
            "plain_value": N * iters / allc["plain_solve_s"], "cpu_model": model,
            "stage_seconds": {k: v for k, v in allc.items() if not k.endswith("solve_s")},
            "sample": f"FP64 oracle stages on bounded samples of the N={N}, B=3, H=5, T=200 workload "
                      f"(rollout+autodiff on 4096 particles, network on all, phi on 8192 rows x N, exact median "
                      f"over all pairs, Adam on all), extrapolated to a {iters}-iteration "
                      f"surrogate-form solve ({s_iters} network iterations); {wall_all:.1f} s on {avail} cores, "
                      f"{wall_one:.1f} s on 1 core"}


def cpu_baseline_plain(seconds_target=15.0):
    """The FP64 oracle (as it stands) on a bounded sample of the N = 1024,
    B = 3, H = 3 workload: whole SVGD iterations of rollout + autodiff
    gradient, median bandwidth, phi and Adam."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import sim, svgd

    _, avail = _host_cpu()
    torch.set_num_threads(avail)
    scene, w, th = W.config_problem(2)
    N = th.shape[0]
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    t0 = time.perf_counter()
    it = 0
    while True:
        _, dC = sim.cost_and_grad(scene, w, th)
        h = svgd.bandwidth(th)
        phi = svgd.svgd_phi(th, -dC, h)
        th, m, v = svgd.adam_step(th, phi, m, v, it + 1, 1e-3)
        it += 1
        el = time.perf_counter() - t0
        if el > seconds_target or it >= 20:
            break
    return {"value": N * it / el, "unit": UNIT, "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{it} SVGD iterations of the N={N}, B=3, H=3, T=200 workload in FP64 "
                      f"(torch CPU autodiff rollout + numpy SVGD), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5,
                    help="timed steps: 300-iteration solves (default workload) or iterations (plain)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="surrogate",
                    choices=["surrogate", "plain", "batched", "long", "refine", "structured", "surrogate-report",
                             "kernels"],
                    help="surrogate (default): the metric's workload, the surrogate form against the plain "
                         "method at N=16384; plain: per-call SVGD iterations at N=1024, B=3, H=3; batched: 64 "
                         "uneven problems in one graph-replayed solve; long: checkpointed and per-phase "
                         "differentiation at T=1000; refine: SVGD alone against SVGD followed by SGD refinement, "
                         "with the plan read-out; structured: the structured pusher kernel against the RBF "
                         "kernel; surrogate-report: the network's accuracy and both direction forms; kernels: "
                         "the default line's stage timings alone (for kernel traces and counters)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the particle set would shard by particle with one all-gather of "
              "[theta | grad] per iteration; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    fn = {"surrogate": bench_headline, "plain": bench_plain_line, "batched": bench_batched, "long": bench_long,
          "refine": bench_refine, "structured": bench_structured, "surrogate-report": bench_surrogate,
          "kernels": bench_kernels}
    return fn[args.workload](args)


def _time_launches(fn, reps=10, warm=2):
    """Mean ms of fn() over reps launches, each bracketed by HIP events on the
    current stream (the stream the library launches on)."""
    import numpy as np
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def stage_timings(ctx, sc, cw, theta0, params, wbf16, n_in, enc):
    """Per-call launches of each stage of the surrogate-form solve at its
    shape, timed with HIP events on the stream they run on (ms, mean of 10):
    the rollout forward and adjoint (the single-problem solve runs these very
    kernels), the exact FP32 bandwidth stage, the FP32 direction stage (V
    packing, the matrix-core contraction k_phi32, the reduce), the network's
    cost and input gradient, and the BF16 step."""
    import torch
    d, N = theta0.shape
    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")
    cost = torch.empty(N, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(theta0)
    minus = torch.full((N,), -1.0, device="cuda")
    sws = ctx._bytes(ctx.svgd_workspace_bytes(N, d))
    th = theta0.clone()
    ctx.rollout_fwd(sc, cw, th, tape=tape, cost=cost)
    ctx.rollout_adj(sc, cw, th, tape, cost_bar=minus, grad=grad)
    ms = {
        "rollout_fwd": _time_launches(lambda: ctx.rollout_fwd(sc, cw, th, tape=tape, cost=cost)),
        "rollout_adj": _time_launches(lambda: ctx.rollout_adj(sc, cw, th, tape, cost_bar=minus, grad=grad)),
        "bandwidth_fp32_exact": _time_launches(lambda: ctx.svgd_bandwidth(th, 0.0, workspace=sws)),
    }
    ctx.svgd_bandwidth(th, 0.0, workspace=sws)
    phi = torch.empty_like(th)
    ms["direction_fp32"] = _time_launches(lambda: ctx.svgd_direction(th, grad, sws, phi=phi))
    ms["mlp_infer"] = _time_launches(lambda: ctx.mlp_forward(params, wbf16, th, n_in, d, x_layout=1, enc=enc,
                                                             want_y=False, grad=grad, grad_scale=-1.0, w=cw))
    ms["step_bf16"] = _time_launches(lambda: ctx.svgd_step_bf16(th, grad, phi=phi, workspace=sws))
    # the BF16 step at a given bandwidth skips the sampled median: its operands,
    # the matrix-core contraction k_phi16 and the reduce
    h = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.svgd_step_bf16(th, grad, phi=phi, h_out=h, workspace=sws)
    torch.cuda.synchronize()
    hb = float(h.item())
    ms["direction_bf16"] = _time_launches(lambda: ctx.svgd_step_bf16(th, grad, bandwidth=hb, phi=phi, workspace=sws))
    return ms


def bench_kernels(args):
    """The stage timings of the default line alone (no training: the network
    takes its seeded initial weights, which time the same), so that a kernel
    trace of this command holds exactly the launches the line's roofline
    reads."""
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    torch.cuda.set_device(0)
    ctx = S.Context(0)
    scene, w, th0 = W.config_problem(5)
    H = int(scene["H"])
    n_in = 6 * H + W.SCENE_ENC
    params = torch.as_tensor(S.pack_mlp(W.mlp_init(n_in, seed=0)), device="cuda")
    wbf16 = ctx.mlp_weights()
    ctx.mlp_prepare(params, wbf16)
    enc = torch.as_tensor(W.scene_encoding(scene), dtype=torch.float32, device="cuda")
    ms = stage_timings(ctx, S.make_scene(scene), S.make_cost(w), S.soa(th0), params, wbf16, n_in, enc)
    ctx.close()
    print(json.dumps({"workload": "stage timings at N=16384, B=3, H=5 (d=30), T=200", "kernels_ms": ms}), flush=True)


def bench_headline(args):
    """The metric's workload: the surrogate form against the plain method at
    N = 16384, B = 3, H = 5, T = 200, 300 Adam SVGD iterations each; one
    step = one surrogate-form solve."""
    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    from paper_2310_01775_amd import surrogate as SG

    torch.cuda.set_device(0)
    ctx = S.Context(0)
    R = dict(W.SURROGATE_RECIPE)
    H = 5
    n_in = 6 * H + W.SCENE_ENC
    cw = S.make_cost(W.cost_weights())
    scenes = W.surrogate_dataset_scenes(max(R["random_scenes"], R["rounds"] * R["round_scenes"]))
    structs = [S.make_scene(sc) for sc in scenes]
    encs = [torch.as_tensor(W.scene_encoding(sc), dtype=torch.float32, device="cuda") for sc in scenes]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(R["seed"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net, ds, log, _ = SG.train_recipe(ctx, R, lambda p: (structs[p], cw, encs[p]),
                                      lambda p, n: S.soa(W.surrogate_training_plans(p, n, H)),
                                      lambda p, n: S.soa(W.make_particles(5, 1000 + p, n, H)),
                                      W.mlp_init(n_in, seed=R["seed"]), n_in, gen)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    scene, w, th0 = W.config_problem(5)
    N, d = th0.shape
    B, T = scene["B"], scene["T"]
    sc = S.make_scene(scene)
    enc = torch.as_tensor(W.scene_encoding(scene), dtype=torch.float32, device="cuda")
    iters, s_iters = W.CONFIGS[5].iters, int(round(W.CONFIGS[5].extra["surrogate_frac"] * W.CONFIGS[5].iters))
    lr = W.DEFAULT_ADAM["lr"]
    cfg = S.make_cfg(iters, lr=lr)
    work = ctx._bytes(ctx.solve_workspace_bytes([sc], [N], cfg))
    status = ctx.status_word()
    theta0 = S.soa(th0)

    def plain_solve():
        th = theta0.clone()
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        c = ctx.solve([sc], [cw], [N], cfg, th, m, v, workspace=work, status=status)
        return c, None

    def surrogate_solve():
        th = theta0.clone()
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        return ctx.solve_surrogate([sc], [cw], [N], cfg, s_iters, net.params, net.wbf16, n_in, enc, th, m, v,
                                   check_every=80, phi_bf16=True, workspace=work, status=status)

    def timed(fn, warm, steps):
        for _ in range(max(warm, 1)):  # the first solve tunes and captures
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, out

    wall_p, (cost_p, _) = timed(plain_solve, args.warmup, args.steps)
    wall_s, (cost_s, rep) = timed(surrogate_solve, args.warmup, args.steps)
    assert int(status.item()) == 0, "non-finite values during the benchmark"

    def stats(c):
        c = c.double()
        return {"mean": float(c.mean()), "median": float(c.median()), "p10": float(c.quantile(0.1))}

    value = N * iters * args.steps / wall_s
    plain_value = N * iters * args.steps / wall_p
    cs, cp = stats(cost_s), stats(cost_p)

    ms = stage_timings(ctx, sc, cw, theta0, net.params, net.wbf16, n_in, enc)
    # launches per surrogate-form solve: simulator iterations, network
    # iterations, simulator checks every 80 network iterations, final cost
    n_sim, n_net, n_chk = iters - s_iters, s_iters, s_iters // 80
    share = {"rollout_adj": n_sim * ms["rollout_adj"], "rollout_fwd": (n_sim + n_chk + 1) * ms["rollout_fwd"],
             "direction_fp32": n_sim * ms["direction_fp32"], "mlp_infer": (n_net + n_chk) * ms["mlp_infer"],
             "direction_bf16": n_net * ms["direction_bf16"],
             "bandwidth_bf16": n_net * max(ms["step_bf16"] - ms["direction_bf16"], 0.0)}
    def roof_for(dom):
        """The roofline object of one stage (its dominant kernel at this shape)."""
        by_f, by_a = rollout_bytes(N, d, B, T, H)
        if dom in ("rollout_adj", "rollout_fwd"):
            byts = by_a if dom == "rollout_adj" else by_f
            achieved = byts / (ms[dom] * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                    "kernel": "k_%s_packed<%d>" % (dom, B), "kernel_ms": ms[dom], "bytes_per_launch": byts}
            if dom == "rollout_adj":
                one = rollout_bytes_single_trajectory(N, d, B, T)
                roof["frac_single_trajectory_bytes"] = one / (ms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS
        elif dom == "mlp_infer":
            fl = mlp_flops(N, n_in)
            achieved = fl / (ms[dom] * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": measured_traffic("mlp_infer"), "kernel": "k_mlp_infer",
                    "kernel_ms": ms[dom]}
        else:  # a direction stage (the BF16 bandwidth stage, several small kernels, never leads)
            # both directions run on the BF16 matrix cores at d = 30: the FP32 one
            # in split form (three BF16 parts per operand), so its algorithmic
            # flops are priced against the BF16 peak too
            fl = phi_flops(N, d)
            achieved = fl / (ms[dom] * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": measured_traffic(dom), "kernel_ms": ms[dom],
                    "flops_per_launch": fl,
                    "kernel": ("k_phi3<2> (FP32 direction in split form on the BF16 matrix cores; the stage also holds "
                               "k_pack32_v and k_reduce32)" if dom == "direction_fp32" else
                               "k_phi16<32,32> (BF16 matrix cores; the stage also holds k_pack16_v and k_reduce16)")}
            if dom == "direction_fp32":
                ex = split3_mfma_flops(N)
                roof["executed_mfma_tflops"] = ex / (ms[dom] * 1e-3) / 1e12
                roof["executed_mfma_frac"] = roof["executed_mfma_tflops"] / MFMA_BF16_PEAK_TFLOPS
        return roof

    dom = max(share, key=share.get)
    roof = roof_for(dom)
    # every stage's own roofline beside it (the BF16 bandwidth stage is a few small kernels: none)
    stage_roofs = {k: roof_for(k) for k in share if k != "bandwidth_bf16"}

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": f"surrogate form vs plain STAMP SVGD: N={N} particles, B={B} blocks, H={H} pushes "
                               f"(d={d}), T={T} steps of dt={scene['dt']:.3f}, {iters} Adam SVGD iterations per "
                               f"solve (one step = one solve); surrogate form: the network's gradient (BF16 "
                               f"matrix cores) and the BF16 direction for iterations 0..{s_iters - 1}, the "
                               f"simulator (full-tape adjoint, exact median, FP32 direction) after",
                   "N": N, "d": d, "B": B, "H": H, "T": T, "iters": iters, "surrogate_iters": s_iters},
        "plain": {"value": plain_value, "ms_per_solve": wall_p * 1e3 / args.steps, "final_true_cost": cp},
        "surrogate": {"final_true_cost": cs, "surrogate_iters_run": rep.iters_run, "fell_back": rep.fell_back,
                      "handoff_log_error": rep.log_err},
        "speedup_vs_plain": value / plain_value,
        "equal_cost": {"surrogate_mean_le_plain_mean": cs["mean"] <= cp["mean"],
                       "surrogate_median_le_plain_median": cs["median"] <= cp["median"]},
        "training": {"rows": ds.n, "seconds": train_s, "steps": log.steps},
        "roofline": roof,
        "stage_rooflines": stage_roofs,
        "kernels_ms": ms,
        "kernel_ms_per_solve": share,
    }
    out["secondary"] = {"plain_n1024": plain_line_in_child()}
    if not args.no_cpu_baseline:
        from paper_2310_01775_amd import unpack_mlp
        params = unpack_mlp(net.params.cpu().numpy(), n_in)
        out["cpu_baseline"] = cpu_baseline_surrogate(params, W.scene_encoding(scene), scene, W.cost_weights(),
                                                     th0, iters, s_iters)
    ctx.close()
    print(json.dumps(out), flush=True)


def plain_line_in_child():
    """The per-call N = 1 024 line measured in a process of its own: after the
    surrogate-form solves this process's per-call launches run ~15 % slower
    (0.236 vs 0.205 ms per step), a state of the process, not of the
    workload."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "plain", "--steps", "100", "--warmup", "5",
           "--no-cpu-baseline"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError("the per-call line failed in its own process:\n" + r.stderr[-2000:])
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    out = json.loads(line)
    out["process"] = "own"
    return out


def bench_plain_line(args):
    """The per-call plain workload alone (N = 1024, B = 3, H = 3), as its own
    JSON line with the FP64 oracle beside it."""
    import paper_2310_01775_amd as S
    ctx = S.Context(0)
    out = bench_plain(args, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_plain(args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_plain(args, ctx):
    """Per-call SVGD iterations on the N = 1024, B = 3, H = 3 (d = 18), T = 200
    scene: bandwidth stage on a side stream beside rollout forward + adjoint,
    then direction + Adam in one pass; returns its measurements."""
    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    dev = torch.device("cuda", 0)
    scene, w, th = W.config_problem(2)
    N, d, B, T, H = th.shape[0], th.shape[1], scene["B"], scene["T"], scene["H"]
    sc, cw = S.make_scene(scene), S.make_cost(w)
    theta = S.soa(th)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device=dev)
    cost = torch.empty(N, dtype=torch.float32, device=dev)
    grad = torch.empty_like(theta)
    minus_one = torch.full((N,), -1.0, dtype=torch.float32, device=dev)
    sws = torch.empty(ctx.svgd_workspace_bytes(N, d), dtype=torch.uint8, device=dev)
    status = ctx.status_word()
    lr = W.DEFAULT_ADAM["lr"]

    # The bandwidth (exact median) depends on theta only: it runs on a side
    # stream beside the rollout, which leaves most SIMDs idle at this size;
    # the direction waits for it.  Both streams have the default priority.
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    ev_fork, ev_join = torch.cuda.Event(), torch.cuda.Event()

    def iteration(t, evs=None):
        ev_fork.record(main)
        side.wait_event(ev_fork)
        if evs:
            evs[4].record(side)
        ctx.svgd_bandwidth(theta, 0.0, workspace=sws, stream=side)
        ev_join.record(side)
        if evs:
            evs[5].record(side)
            evs[0].record()
        ctx.rollout_fwd(sc, cw, theta, tape=tape, cost=cost, status=status)
        if evs:
            evs[1].record()
        ctx.rollout_adj(sc, cw, theta, tape, cost_bar=minus_one, grad=grad, status=status)
        if evs:
            evs[2].record()
        main.wait_event(ev_join)
        ctx.svgd_update(theta, grad, sws, m, v, t, lr=lr)  # direction + Adam in one pass
        if evs:
            evs[3].record()

    for t in range(1, args.warmup + 1):
        iteration(t)
    torch.cuda.synchronize()
    # throughput without instrumentation (six timing events per step cost the
    # GPU timeline ~20 us), then the same number of steps with the events for
    # the per-kernel breakdown
    t0 = time.perf_counter()
    for k in range(args.steps):
        iteration(args.warmup + k + 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    for k in range(args.steps):
        iteration(args.warmup + args.steps + k + 1, events[k])
    torch.cuda.synchronize()
    assert int(status.item()) == 0, "non-finite values during the benchmark"
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    adj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    by_f, by_a = rollout_bytes(N, d, B, T, H)
    return {"metric": METRIC, "value": N * args.steps / wall, "unit": UNIT, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
            "config": {"workload": f"plain STAMP SVGD per call, FP32: N={N}, B={B}, H={H} (d={d}), T={T}, "
                                   f"full-tape adjoint, exact median beside the rollout, Adam",
                       "N": N, "d": d, "B": B, "H": H, "T": T},
            "kernels_ms": {"rollout_fwd": fwd_ms, "rollout_adj": adj_ms,
                           "direction+update": float(np.mean([e[2].elapsed_time(e[3]) for e in events])),
                           "bandwidth_beside_rollout": float(np.mean([e[4].elapsed_time(e[5]) for e in events]))},
            "rollout_adj_GBps": by_a / (adj_ms * 1e-3) / 1e9}


def bench_batched(args):
    """64 seeded problems, N ~ U{64..2048}, H ~ U{2..5}, B ~ U{1..4}, T=200,
    one stamp_solve call (batched stages, graph replay, autotuned shapes):
    once as one lockstep batch, and once class-scheduled (cfg.classes: the
    problems in cost classes, cheapest first, each class a batch of its own),
    where a problem's solve time is its class's end."""
    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W

    probs = W.batched_problems(4)
    ctx = S.Context(0)
    scenes = [S.make_scene(s) for s, _, _ in probs]
    ws_ = [S.make_cost(w) for _, w, _ in probs]
    Ns = [th.shape[0] for _, _, th in probs]
    flat = torch.cat([S.soa(th).reshape(-1) for _, _, th in probs]).contiguous()
    lr = W.DEFAULT_ADAM["lr"]
    total = sum(Ns)
    out = {"workload": "batched: 64 problems N~U{64..2048} H~U{2..5} B~U{1..4} T=200", "particles": total,
           "iters": args.steps}
    results = {}
    for name, classes in (("lockstep", 0), ("classes2", 2), ("classes4", 4), ("classes8", 8)):
        cfg = lambda iters: S.make_cfg(iters, lr=lr, classes=classes)
        work = torch.empty(ctx.solve_workspace_bytes(scenes, Ns, cfg(args.steps)), dtype=torch.uint8,
                           device="cuda")
        times = torch.zeros(len(probs), device="cuda")
        status = ctx.status_word()

        def run(iters, theta):
            m, v = torch.zeros_like(theta), torch.zeros_like(theta)
            return ctx.solve(scenes, ws_, Ns, cfg(iters), theta, m, v, solve_time_us=times, workspace=work,
                             status=status)

        # warm-up: the same solve, so that the autotuning and the capture of
        # every graph the timed call replays happen before it
        for _ in range(max(args.warmup, 1)):
            run(args.steps, flat.clone())
        torch.cuda.synchronize()
        theta = flat.clone()
        t0 = time.perf_counter()
        cost = run(args.steps, theta)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert int(status.item()) == 0
        tus = times.cpu().numpy()
        results[name] = (theta, cost)
        out[name] = {"wall_s": wall, "particle_iters_per_s": total * args.steps / wall,
                     "solve_time_us_p50": float(np.percentile(tus, 50)),
                     "solve_time_us_p99": float(np.percentile(tus, 99)),
                     "solve_time_us_mean": float(tus.mean())}
        del work
    out["classes_equal_lockstep"] = all(torch.equal(results["lockstep"][0], r[0]) and
                                        torch.equal(results["lockstep"][1], r[1]) for r in results.values())
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_long(args):
    """Checkpointed differentiation: 1 block, 5 pushes, T=1000 steps, N=4096;
    forward + adjoint time and the bytes kept between them, full tape vs
    32-step checkpoints."""
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    from paper_2310_01775_amd.autograd import rollout_cost, tape_bytes

    scene, w, th = W.config_problem(3)
    ctx = S.Context(0)
    sc, cw = S.make_scene(scene), S.make_cost(w)
    N = th.shape[0]
    out = {"workload": "1 block, 5 pushes (d=30), T=1000 steps of dt=0.001, N=4096", "N": N}
    for K in (0, 32):
        x = S.soa(th).requires_grad_(True)
        for _ in range(2):
            rollout_cost(x, ctx, sc, cw, K).sum().backward()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            x.grad = None
            rollout_cost(x, ctx, sc, cw, K).sum().backward()
        b.record()
        torch.cuda.synchronize()
        out[f"K{K}"] = {"fwd_bwd_ms": a.elapsed_time(b) / args.steps, "kept_bytes": tape_bytes(sc, N, K)}
    # the per-phase split of the cost: gradient size per push, full adjoint
    # against the split's (median over the particles of each push's gradient
    # norm), and the time of the split's adjoint
    theta = S.soa(th)
    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")
    ctx.rollout_fwd(sc, cw, theta, tape=tape)
    norms = {}
    for name, pp in (("full", False), ("per_phase", True)):
        g = ctx.rollout_adj(sc, cw, theta, tape, per_phase=pp)
        gg = g.double().view(int(scene["H"]), 6, N).norm(dim=1)
        norms[name] = [float(x) for x in gg.median(dim=1).values]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        ctx.rollout_adj(sc, cw, theta, tape, per_phase=True)
    b.record()
    torch.cuda.synchronize()
    out["grad_norm_median_per_push"] = norms
    out["per_phase_adj_ms"] = a.elapsed_time(b) / args.steps
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_surrogate(args):
    """The surrogate form against the plain method on the N=16384, B=3, H=5,
    T=200 scene: 300 SVGD iterations each, the surrogate form taking the
    network's gradient for the first 240 (simulator checks every 80).  The
    network is first trained by the library (2^20 labelled rollouts, two
    on-policy rounds); its training time is reported apart."""
    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    from paper_2310_01775_amd import surrogate as SG

    ctx = S.Context(0)
    R = dict(W.SURROGATE_RECIPE)
    H = 5
    n_in = 6 * H + W.SCENE_ENC
    cw = S.make_cost(W.cost_weights())
    scenes = W.surrogate_dataset_scenes(max(R["random_scenes"], R["rounds"] * R["round_scenes"]))
    structs = [S.make_scene(sc) for sc in scenes]
    encs = [torch.as_tensor(W.scene_encoding(sc), dtype=torch.float32, device="cuda") for sc in scenes]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(R["seed"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net, ds, log, reps = SG.train_recipe(ctx, R, lambda p: (structs[p], cw, encs[p]),
                                         lambda p, n: S.soa(W.surrogate_training_plans(p, n, H)),
                                         lambda p, n: S.soa(W.make_particles(5, 1000 + p, n, H)),
                                         W.mlp_init(n_in, seed=R["seed"]), n_in, gen)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    scene, _, th0 = W.config_problem(5)
    N = th0.shape[0]
    sc = S.make_scene(scene)
    enc = torch.as_tensor(W.scene_encoding(scene), dtype=torch.float32, device="cuda")
    iters, s_iters = 300, 240
    lr = W.DEFAULT_ADAM["lr"]
    work = ctx._bytes(ctx.solve_workspace_bytes([sc], [N], S.make_cfg(iters, lr=lr)))
    status = ctx.status_word()

    def plain():
        th = S.soa(th0)
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        torch.cuda.synchronize()
        t = time.perf_counter()
        c = ctx.solve([sc], [cw], [N], S.make_cfg(iters, lr=lr), th, m, v, workspace=work, status=status)
        torch.cuda.synchronize()
        return time.perf_counter() - t, c, None

    def surrogate(phi_bf16):
        th = S.soa(th0)
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        torch.cuda.synchronize()
        t = time.perf_counter()
        c, rep = ctx.solve_surrogate([sc], [cw], [N], S.make_cfg(iters, lr=lr), s_iters, net.params, net.wbf16,
                                     n_in, enc, th, m, v, check_every=80, phi_bf16=phi_bf16, workspace=work,
                                     status=status)
        torch.cuda.synchronize()
        return time.perf_counter() - t, c, rep

    def stats(c):
        c = c.double()
        return {"mean": float(c.mean()), "median": float(c.median()), "p10": float(c.quantile(0.1)),
                "min": float(c.min())}

    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device="cuda")

    def accuracy(th):
        """The network's cost and gradient against the simulator's (full
        cost, bound term included) on the particles th [d][N]."""
        c_true = ctx.rollout_fwd(sc, cw, th, tape=tape, status=status)
        g_true = ctx.rollout_adj(sc, cw, th, tape, status=status)
        _, c_sur, g_sur = ctx.mlp_forward(net.params, net.wbf16, th, n_in, 6 * H, x_layout=1, enc=enc,
                                          want_y=False, want_cost=True, want_grad=True, w=cw)
        ae = (c_sur.double() - c_true.double()).abs()
        rel = ae / c_true.double().abs().clamp_min(1e-3)
        gs, gt = g_sur.double(), g_true.double()
        cos = (gs * gt).sum(0) / (gs.norm(dim=0) * gt.norm(dim=0)).clamp_min(1e-30)
        return {"cost_abs_err_mean": float(ae.mean()), "cost_abs_err_median": float(ae.median()),
                "cost_rel_err_median": float(rel.median()), "grad_cosine_mean": float(cos.mean()),
                "grad_cosine_median": float(cos.median()), "true_cost_median": float(c_true.double().median())}

    def handoff(phi_bf16):
        """Accuracy on the particles the surrogate phase hands to the
        simulator (after its s_iters iterations; the solve is deterministic,
        so these are the timed run's particles at that point)."""
        th = S.soa(th0)
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        ctx.solve_surrogate([sc], [cw], [N], S.make_cfg(s_iters, lr=lr), s_iters, net.params, net.wbf16, n_in,
                            enc, th, m, v, check_every=80, phi_bf16=phi_bf16, workspace=work, status=status)
        return accuracy(th)

    out = {"workload": f"surrogate form vs plain: N={N}, B=3, H=5 (d=30), T=200 steps of dt=0.005, "
                       f"{iters} Adam SVGD iterations, surrogate for the first {s_iters}",
           "training": {"rows": ds.n, "seconds": train_s, "steps": log.steps,
                        "final_minibatch_loss": log.losses[-1][1]}}
    for name, fn in (("plain", plain), ("surrogate_bf16_phi", lambda: surrogate(True)),
                     ("surrogate_fp32_phi", lambda: surrogate(False))):
        fn()  # autotune, graph capture
        wall, c, rep = fn()
        out[name] = {"wall_s": wall, "particle_iters_per_s": N * iters / wall, "final_true_cost": stats(c)}
        if rep is not None:
            out[name]["surrogate_iters"] = rep.iters_run
            out[name]["fell_back"] = rep.fell_back
            out[name]["handoff_log_error"] = rep.log_err
    out["surrogate_accuracy"] = {"initial_particles": accuracy(S.soa(th0)),
                                 "handoff_bf16_phi": handoff(True), "handoff_fp32_phi": handoff(False)}
    assert int(status.item()) == 0
    for name in ("surrogate_bf16_phi", "surrogate_fp32_phi"):
        out[name]["speedup_vs_plain"] = out["plain"]["wall_s"] / out[name]["wall_s"]
        out[name]["median_cost_vs_plain"] = (out[name]["final_true_cost"]["median"] /
                                             out["plain"]["final_true_cost"]["median"])
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_refine(args):
    """Algorithm 1's two phases on the N=1024, B=3, H=3, T=200 scene: 300 SVGD
    iterations against 200 SVGD + 100 SGD refinement iterations (the paper's
    question whether refinement is needed), and the same with the importance
    weights of Eq. (4) in the SVGD phase; each one graph-replayed stamp_solve,
    then the plan read-out: the discrete plan of every particle, the cost of
    executing it, and the solutions (executed cost below the threshold) per
    plan."""
    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    from paper_2310_01775_amd import readout

    scene, w, th = W.config_problem(2)
    N = th.shape[0]
    ctx = S.Context(0)
    sc, cw = S.make_scene(scene), S.make_cost(w)
    lr = W.DEFAULT_ADAM["lr"]
    status = ctx.status_word()
    out = {"workload": f"refinement: N={N}, B=3, H=3 (d=18), T=200 steps of dt=0.005, 300 iterations, "
                       f"solutions = executed discrete-plan cost < {W.SOLUTION_COST}"}
    for name, (it, sgd, ds) in (("svgd300", (300, 0, False)), ("svgd200_sgd100", (200, 100, False)),
                                ("dsvgd200_sgd100", (200, 100, True))):
        cfg = S.make_cfg(it, lr=lr, sgd_iters=sgd, dsvgd=ds)
        work = ctx._bytes(ctx.solve_workspace_bytes([sc], [N], cfg))
        for rep in range(2):  # the first run tunes and captures
            theta = S.soa(th)
            m, v = torch.zeros_like(theta), torch.zeros_like(theta)
            torch.cuda.synchronize()
            t = time.perf_counter()
            cost = ctx.solve([sc], [cw], [N], cfg, theta, m, v, workspace=work, status=status)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
        c = cost.double()
        rd = readout.report(ctx, sc, cw, theta, W.SOLUTION_COST)
        out[name] = {"wall_s": wall, "particle_iters_per_s": N * (it + sgd) / wall,
                     "relaxed_cost_median": float(c.median()), "relaxed_cost_p10": float(c.quantile(0.1)),
                     "readout": rd}
    assert int(status.item()) == 0
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_structured(args):
    """The structured pusher kernel (Appendix E-C: per-action RBF terms on
    (o_k, D_k) and on softmax(a_k)) against the RBF kernel on theta: the SVGD
    step's time at N=1024, H=3 and N=16384, H=5 (median-heuristic bandwidths,
    HIP events around 20 steps), then 300 graph-replayed SVGD iterations with
    each kernel on the N=1024, B=3, H=3 scene and the plan read-out."""
    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W
    from paper_2310_01775_amd import readout

    ctx = S.Context(0)
    out = {"workload": "structured kernel vs RBF on theta: step time at N=1024/H=3 and N=16384/H=5; "
                       f"300-iteration solves at N=1024, B=3, H=3, solutions = executed cost < {W.SOLUTION_COST}"}
    for cfg_i in (2, 5):
        scene, w, th = W.config_problem(cfg_i)
        N, d = th.shape
        H = int(scene["H"])
        theta = S.soa(th)
        g = S.soa(np.random.default_rng(cfg_i).normal(0.0, 20.0, (N, d)))
        ws = ctx._bytes(ctx.svgd_workspace_bytes(N, d))
        phi = torch.empty_like(theta)
        kern = S.struct_kernel(S.KERNEL_PUSH, H)
        row = {}
        for name, fn in (("rbf_ms", lambda: ctx.svgd_step(theta, g, 0.0, phi=phi, workspace=ws)),
                         ("structured_ms", lambda: ctx.svgd_step_structured(theta, g, kern, phi=phi, workspace=ws))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(20):
                fn()
            b.record()
            torch.cuda.synchronize()
            row[name] = a.elapsed_time(b) / 20
        out[f"step_N{N}_H{H}"] = row
    scene, w, th = W.config_problem(2)
    N, H = th.shape[0], int(scene["H"])
    sc, cw = S.make_scene(scene), S.make_cost(w)
    status = ctx.status_word()
    for name, kern in (("rbf", None), ("structured", S.struct_kernel(S.KERNEL_PUSH, H))):
        cfg = S.make_cfg(300, lr=W.DEFAULT_ADAM["lr"], kernel=kern)
        work = ctx._bytes(ctx.solve_workspace_bytes([sc], [N], cfg))
        for rep in range(2):  # the first run tunes and captures
            theta = S.soa(th)
            m, v = torch.zeros_like(theta), torch.zeros_like(theta)
            torch.cuda.synchronize()
            t = time.perf_counter()
            cost = ctx.solve([sc], [cw], [N], cfg, theta, m, v, workspace=work, status=status)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
        c = cost.double()
        out[f"solve_{name}"] = {"wall_s": wall, "particle_iters_per_s": N * 300 / wall,
                                "relaxed_cost_median": float(c.median()),
                                "readout": readout.report(ctx, sc, cw, theta, W.SOLUTION_COST)}
    assert int(status.item()) == 0
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

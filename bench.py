"""Benchmark of the STAMP SVGD hot path on one MI355X.

One step = one SVGD iteration of Algorithm 1 over the whole particle set:
rollout forward (full tape) -> rollout adjoint (grad log rho) -> median
bandwidth -> SVGD direction (Eq. 1) -> Adam update, all in the library's HIP
kernels.  Workload: N=1024 particles, 3 blocks, 3 pushes (d=18), T=200 steps
of dt=0.005, seeded synthetic scene and particles.

Metric: particle-iterations/s = N * steps / wall seconds of the timed region
(inputs resident in HBM, synchronised on both sides).  The dominant kernel's
duration comes from HIP events recorded on the stream it is launched on.
cpu_baseline times the FP64 oracle on a bounded sample of the same workload.
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
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0


def rollout_flops_per_lane_step(B, adjoint=False):
    """Algorithmic FP32 operations of one sub-rollout step (one lane), counted
    from the forward step (friction 16/block, contact 26/pair, pusher 52,
    integrator 15/block, time scaling 8) and its reverse (which also recomputes
    the forward intermediates it needs)."""
    pairs = B * (B - 1) // 2
    if not adjoint:
        return 16 * B + 26 * pairs + 52 + 15 * B + 8
    return 12 * B + 36 * B + 54 * pairs + 119 + 8


def rollout_bytes(N, d, B, T, H):
    """Algorithmic HBM bytes of one forward (or adjoint) launch with the full
    tape: theta (4d per particle), the tape of (T+H) states of 6B floats for
    each of the 4 side lanes, and the per-particle output (cost, or 4d grad)."""
    tape = (T + H) * 6 * B * 4 * 4
    return N * (4 * d + tape), N * (4 * d + tape + 4 * d)


KERNEL_SOURCES = ["paper_2310_01775_amd/csrc/rollout.hip", "paper_2310_01775_amd/csrc/common.h"]
PROFILE = os.path.join(ROOT, "profiles", "rollout_n1024_counters.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
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


def cpu_baseline(seconds_target=15.0):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same
    workload: full N=1024 scene, a few iterations of rollout+autodiff gradient,
    median bandwidth, phi and Adam."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import sim, svgd

    threads = os.cpu_count() or 1
    torch.set_num_threads(threads)
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
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="plain", choices=["plain", "batched", "long", "surrogate", "refine",
                                                              "structured"],
                    help="plain: the metric's workload; batched: 64 uneven problems in one graph-replayed "
                         "solve; long: checkpointed differentiation (report only); surrogate: the learned "
                         "surrogate form against the plain method at N=16384 (report only); refine: SVGD "
                         "alone against SVGD followed by SGD refinement, with the plan read-out (report only); "
                         "structured: the structured pusher kernel against the RBF kernel (step time, and "
                         "solutions per plan after a solve; report only)")
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

    import numpy as np
    import torch

    import paper_2310_01775_amd as S
    import workloads as W

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "long":
        return bench_long(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "refine":
        return bench_refine(args)
    if args.workload == "structured":
        return bench_structured(args)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = W.CONFIGS[2]
    scene, w, th = W.config_problem(2)
    N, d, B, T, H = th.shape[0], th.shape[1], scene["B"], scene["T"], scene["H"]
    ctx = S.Context(0)
    sc, cw = S.make_scene(scene), S.make_cost(w)
    theta = S.soa(th)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    tape = torch.empty(ctx.tape_floats(sc, N, 0), dtype=torch.float32, device=dev)
    cost = torch.empty(N, dtype=torch.float32, device=dev)
    grad = torch.empty_like(theta)
    phi = torch.empty_like(theta)
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
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        iteration(args.warmup + k + 1, events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(status.item()) == 0, "non-finite values during the benchmark"

    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    adj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    svgd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in events]))
    bw_ms = float(np.mean([e[4].elapsed_time(e[5]) for e in events]))
    value = N * args.steps / wall
    fl_f = rollout_flops_per_lane_step(B) * 4 * N * T
    fl_a = rollout_flops_per_lane_step(B, True) * 4 * N * T
    by_f, by_a = rollout_bytes(N, d, B, T, H)
    dom = "rollout_adj" if adj_ms >= fwd_ms else "rollout_fwd"
    dom_ms = max(adj_ms, fwd_ms)
    dom_fl = fl_a if dom == "rollout_adj" else fl_f
    achieved = dom_fl / (dom_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"plain STAMP SVGD, FP32: N={N} particles, B={B} blocks, H={H} pushes "
                               f"(d={d}), T={T} steps of dt={scene['dt']:.3f}, full-tape adjoint, "
                               f"exact median bandwidth (on a side stream beside the rollout), Adam",
                   "N": N, "d": d, "B": B, "H": H, "T": T, "tape": "full"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": measured_traffic(dom),
                     "kernel": dom, "kernel_ms": dom_ms,
                     "hbm_GBps": (by_a if dom == "rollout_adj" else by_f) / (dom_ms * 1e-3) / 1e9},
        "kernels_ms": {"rollout_fwd": fwd_ms, "rollout_adj": adj_ms, "direction+update": svgd_ms,
                       "bandwidth_beside_rollout": bw_ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """64 seeded problems, N ~ U{64..2048}, H ~ U{2..5}, B ~ U{1..4}, T=200,
    one stamp_solve call (batched stages, graph replay, autotuned shapes)."""
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
    work = torch.empty(ctx.solve_workspace_bytes(scenes, Ns, S.make_cfg(args.steps, lr=lr)), dtype=torch.uint8,
                       device="cuda")
    times = torch.zeros(len(probs), device="cuda")
    status = ctx.status_word()

    def run(iters, theta):
        m, v = torch.zeros_like(theta), torch.zeros_like(theta)
        return ctx.solve(scenes, ws_, Ns, S.make_cfg(iters, lr=lr), theta, m, v, solve_time_us=times,
                         workspace=work, status=status)

    warm = flat.clone()
    run(max(args.warmup, 1), warm)  # autotune + graph instantiation
    torch.cuda.synchronize()
    theta = flat.clone()
    t0 = time.perf_counter()
    run(args.steps, theta)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(status.item()) == 0
    tus = times.cpu().numpy()
    total = sum(Ns)
    print(json.dumps({"workload": "batched: 64 problems N~U{64..2048} H~U{2..5} B~U{1..4} T=200",
                      "particles": total, "iters": args.steps, "wall_s": wall,
                      "particle_iters_per_s": total * args.steps / wall,
                      "solve_time_us_p50": float(np.percentile(tus, 50)),
                      "solve_time_us_p99": float(np.percentile(tus, 99))}), flush=True)
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

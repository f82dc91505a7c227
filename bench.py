#!/usr/bin/env python3
"""Throughput of one cost + exact-gradient evaluation (the whole hot path)
on one MI355X, in time-steps per second, on a seeded synthetic workload.

A "step" of this benchmark is one qoc_cost_grad_device call over the whole
control array: norms and (p, n), all N step exponentials, block products,
forward sweeps with penalties and fidelity, costate sweeps, and the exact
per-step derivative contracted into dC/du.  Inputs are resident in HBM
before the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config c4|c3|c2|c1|c5]

The default workload is the 9-spin chain (d=512, M=18, N=1000, S=8), the
largest single-GPU configuration of the metric's d = 16..512 range.

c5 (256 uneven instances): a step is one optimizer iteration (every
instance's cost + gradient and an Adam update), replayed from a HIP graph;
value = sum of N_i over the median iteration time.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cost+grad time-steps/sec vs plain FP64 GPU path at |ΔF|≤1e-6, d=16–512"
# Dense MFMA peaks.  bf16x3 executes three bf16 products per FP32-equivalent
# product, so its FP32-equivalent peak is the bf16 peak over 3.
PEAK = {"fp32": {"mfma": 157.3e12, "alu": 157.3e12 / 2}, "fp64": {"mfma": 78.6e12, "alu": 78.6e12},
        "bf16x3": {"mfma": 2.5e15 / 3, "alu": 157.3e12 / 2}}
BF3_PHASES = ("taylor", "blockprod")  # phases that run bf16x3 products (padded d % 64 == 0)
HBM_PEAK = 8.0e12


# HBM bytes per launch (read, written) of the kernel behind a timed phase,
# from two rocprofv3 PMC runs (FETCH_SIZE, WRITE_SIZE) scaled by the same
# counters on a 256 MiB device copy (x2.0 and x1.0 to four digits); the table, commands
# and calibration are in profiles/hbm_traffic_pmc.md.  FP32 chains; kernels
# changed since their counters were taken have no entry (traffic null).
TRAFFIC = {
    ("c2_transmon_cnot", "adjoint"): ("k_adjoint16", 15221088, 64064),
    ("c2_transmon_cnot", "taylor"): ("k_expm16", 615810, 18857632),
    ("c2_transmon_cnot", "bwd_blocks"): ("k_wB2", 2872874, 160384),
    ("c2_transmon_cnot", "fwd_replay"): ("k_wF3s", 9192707, 1184768),
    ("c2_transmon_cnot", "bwd_pairs"): ("k_wB3s", 5295042, 1024000),
    ("c4_spin_chain", "taylor"): ("k_stage_t", 7382338232, 2516582400),
    ("c3_transmon_cavity", "taylor"): ("k_stage64", 1933738424, 737280000),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_work(prob, info, phase, calls, precision, steps_timed=1):
    """(bound, algorithmic units per launch) for one timed kernel phase.

    Complex d x d x d product = 8 d^3 real flops; streaming one step
    propagator D_j = 8 d^2 bytes (FP32 planar).  True d, not the padding.
    """
    d, N, M, S = prob.d, prob.N, prob.M, prob.S
    p, n, L = info["p"], info["n"], info["block_len"]
    esz = 8 if precision == "fp64" else 4  # bf16x3 keeps FP32 storage
    if phase == "taylor":
        # batched path: every launch is one complex product per step (Horner
        # or Paterson-Stockmeyer stages, squarings); small-d path: one launch
        # runs the whole Horner chain, p - 1 + n products per step
        per_call = max(calls // max(steps_timed, 1), 1)
        G = 1 if per_call > 1 else p - 1 + n
        return "mfma", N * 8.0 * d ** 3 * G
    if phase == "blockprod":
        total = (N - info["n_blocks"]) * 8.0 * d ** 3
        return "mfma", total / max(calls // max(steps_timed, 1), 1)
    if phase in ("fwd_replay", "bwd_pairs"):
        return "hbm", N * 2.0 * d * d * esz
    if phase in ("fwd_blocks", "bwd_blocks"):
        return "hbm", info["n_blocks"] * 2.0 * d * d * esz
    if phase == "adjoint":
        f, r = 0.0, S
        for _ in range(n):
            f += 2 * 8.0 * d * d * min(r, d)
            r = min(2 * r, d)
        f += 2 * (p - 1) * 8.0 * d * d * r + 8.0 * d * d * p * r + 8.0 * d * d * M
        return "mfma", N * f
    if phase == "norm":
        return "alu", N * d * d * (M + 1) * 4.0
    if phase == "assemble":
        return "hbm", N * 2.0 * d * d * esz * 2
    return "hbm", 0.0


def path_work(prob, info):
    """Algorithmic real flops of one whole cost + gradient call, counted per
    time step as 3 G products of 8 d^3 (the G = p - 1 + n products of the
    step exponential and 2 G for its exact derivative), 24 d^2 S for the
    forward, replay and costate sweeps, 8 d^2 M for the gradient overlaps
    and 4 d^2 (M + 1) for the assembly, twice (true d).  The kernels execute
    fewer products than 3 G per step (Paterson-Stockmeyer Taylor stages and
    rank-S factored derivative products), so the whole-path fraction can
    exceed what the kernels' own MFMA counters show."""
    d, N, M, S = prob.d, prob.N, prob.M, prob.S
    G = info["p"] - 1 + info["n"]
    return N * (3 * G * 8.0 * d ** 3 + 24.0 * d * d * S + 8.0 * d * d * M
                + 2 * 4.0 * d * d * (M + 1))


def executed_work(prob, info, precision="fp32"):
    """Real flops the kernels execute as matrix products in one call: the
    Taylor stages (Paterson-Stockmeyer or Horner, as the library plans
    them), the squarings, the block products and the per-step derivative
    with factored cotangents (algorithmic_work's adjoint count)."""
    d, N = prob.d, prob.N
    pp, nn = info["p"], info["n"]
    G = ps_products(pp) + nn if info["d_pad"] > 48 else pp - 1 + nn
    f = N * 8.0 * d ** 3 * G + (N - info["n_blocks"]) * 8.0 * d ** 3
    _, fa = algorithmic_work(prob, info, "adjoint", 1, precision)
    return f + fa


def ps_products(p):
    """Products of the batched Taylor stage for order p: Paterson-Stockmeyer
    with block s in 2..4 when that beats the p - 1 of Horner (the rule of
    the library's host plan)."""
    best = p - 1
    for s in range(2, min(p, 4) + 1):
        Q, rem = divmod(p, s)
        best = min(best, (s - 1) + Q - (1 if rem == 0 else 0))
    return best


def fp64_torch_path(prob, dev, reps=2):
    """Plain FP64 GPU path: complex128 torch, batched matrix_exp, a
    sequential product loop and autograd (exact Frechet derivatives)."""
    import numpy as np
    import torch
    c128 = torch.complex128
    H0 = torch.tensor(prob.H0, dtype=c128, device=dev)
    Hk = torch.tensor(prob.Hk, dtype=c128, device=dev)
    psi0 = torch.tensor(prob.psi0.T.copy(), dtype=c128, device=dev)      # d x S
    psiT = torch.tensor(prob.psiT.T.copy(), dtype=c128, device=dev)
    w = torch.tensor(prob.w if prob.w is not None else np.zeros(prob.d), dtype=torch.float64,
                     device=dev)
    S = prob.S

    def run(u_np):
        u = torch.tensor(u_np, dtype=torch.float64, device=dev, requires_grad=True)
        H = H0 + torch.tensordot(u.to(c128).t().contiguous(), Hk, dims=1)
        U = torch.linalg.matrix_exp((-1j * prob.dt) * H)
        psi = psi0
        pen = torch.zeros((), dtype=torch.float64, device=dev)
        for j in range(prob.N):
            psi = U[j] @ psi
            if prob.w is not None:
                pen = pen + (w[:, None] * (psi.real ** 2 + psi.imag ** 2)).sum() / S
        ov = (psiT.conj() * psi).sum(dim=0)
        F = (ov.sum() / S).abs() ** 2 if prob.fid_mode == "coherent" else (ov.abs() ** 2).sum() / S
        C = prob.alpha_fid * (1 - F) + prob.alpha_pen * pen + prob.alpha_amp * (u ** 2).sum()
        if prob.N > 1:
            C = C + prob.alpha_var * ((u[:, 1:] - u[:, :-1]) ** 2).sum()
        C.backward()
        return float(C.detach()), float(F.detach()), u.grad.detach().cpu().numpy()

    run(prob.u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        C, F, g = run(prob.u)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return dict(value=prob.N / dt, unit="time-steps/s", ms_per_step=dt * 1e3, reps=reps,
                F=F, grad=g)


def quick_measure(prob, precision, args, tuned=None, segment_steps=0, propagation="matrix"):
    """ms per cost + gradient call of one workload and precision (device-
    resident inputs, args.steps timed calls after args.warmup), with its
    accuracy against the stored oracle outputs where they exist; with
    segment_steps, in the memory-lean mode (time segments)."""
    import numpy as np
    import torch
    from paper_1612_04929_amd import qoc
    from paper_1612_04929_amd import tune as qtune
    dev = torch.device("cuda:0")
    h = qoc.Problem(prob, precision=precision, device=0,
                    checkpoint_every=tuned["checkpoint_every"] if tuned else 0,
                    segment_steps=segment_steps, propagation=propagation)
    if tuned:
        qtune.apply(h, tuned)
    u = torch.from_numpy(np.ascontiguousarray(prob.u)).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    grad = torch.zeros(max(1, prob.M * prob.N), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    step = lambda: h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), st)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    info = h.info()
    h.close()
    r = dict(workload=prob.name, precision=precision, ms_per_step=ms, value=prob.N / (ms / 1e3),
             unit="time-steps/s", taylor_p=info["p"], taylor_n=info["n"],
             checkpoint_every=info["block_len"], bf16x3_classes=info["bf16x3_classes"],
             flags=info["flags"], segments=info["segments"], device_bytes=info["device_bytes"],
             propagation=propagation)
    golden = os.path.join(ROOT, "tests", "golden", f"{prob.name[:2]}_full_oracle.npz")
    if os.path.exists(golden):
        with np.load(golden) as z:
            g = grad[: prob.M * prob.N].cpu().numpy().reshape(prob.M, prob.N)
            r["accuracy_vs_oracle"] = dict(
                dF=abs((1 - float(out[1])) - float(z["F"])),
                grad_rel=float(np.linalg.norm(g - z["grad"]) / np.linalg.norm(z["grad"])),
                max_dc=float(np.max(np.abs(out[2:].cpu().numpy() - z["c"]))))
    log(f"[bench] {prob.name} {precision}: {ms:.3f} ms/call, {r['value']:.4g} time-steps/s")
    return r


def cpu_baseline(prob, seconds):
    """The FP64 oracle as it stands, on the host cores, on a bounded sample."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    # size the sample so that one call takes a few seconds at most
    probe = prob.with_steps(min(prob.N, 50))
    t0 = time.perf_counter()
    oracle.cost_grad(probe)
    per_step = (time.perf_counter() - t0) / probe.N
    n_sample = int(max(1, min(prob.N, (seconds / 3.0) / max(per_step, 1e-9))))
    sample = prob.with_steps(n_sample)
    runs, steps, t0 = 0, 0, time.perf_counter()
    ref = None
    while True:
        ref = oracle.cost_grad(sample)
        runs += 1
        steps += sample.N
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    return dict(value=steps / el, unit="time-steps/s", cores=int(cores), kind="oracle",
                sample=f"{runs} x oracle.cost_grad on the first {n_sample} of {prob.N} steps "
                       f"of {prob.name} ({el:.1f} s)"), (sample, ref)


def batch_work(probs, batch):
    """Algorithmic MFMA flops of one cost+grad over all instances (the
    counting of algorithmic_work: Taylor/squaring products, block products
    and the per-step derivative) and their sum over instances."""
    tot = 0.0
    for p, h in zip(probs, batch.handles):
        inf = h.info()
        d, N, M, S = p.d, p.N, p.M, p.S
        pp, nn = inf["p"], inf["n"]
        G = ps_products(pp) + nn if inf["d_pad"] > 48 else pp - 1 + nn
        f = N * 8.0 * d ** 3 * G + (N - inf["n_blocks"]) * 8.0 * d ** 3
        _, fa = algorithmic_work(p, inf, "adjoint", 1, "fp32")
        tot += f + fa
    return tot


def bench_batch(args):
    """Uneven batch: every instance's cost + gradient and an Adam update per
    iteration; graph replays vs eager multi-stream vs per-instance calls."""
    import numpy as np
    import torch

    import workloads
    from paper_1612_04929_amd.batch import Batch

    dev = torch.device("cuda:0")
    probs = workloads.config5()
    log(f"[bench] c5: {len(probs)} instances, d {min(p.d for p in probs)}..{max(p.d for p in probs)}, "
        f"sum N = {sum(p.N for p in probs)}, precision={args.precision}")
    t_tune = time.perf_counter()
    b = Batch(probs, precision=args.precision, streams=args.streams,
              tune_tiles=not args.no_tune)
    t_tune = time.perf_counter() - t_tune
    log(f"[bench] c5 tiles: {sum(1 for x in b.pads if x == 64)} of {len(probs)} instances on "
        f"64 x 64 tiles (set-up and tuning {t_tune:.1f} s)")
    res_acc = {}
    if not args.no_cpu_baseline:
        import oracle
        order = sorted(range(len(probs)), key=lambda i: probs[i].d ** 3 * probs[i].N)
        sample = order[:: max(1, len(order) // 6)][:6]
        worst_F, worst_g = 0.0, 0.0
        for i in sample:
            ref = oracle.cost_grad(probs[i])
            g = b.grad[i][: probs[i].M * probs[i].N].cpu().numpy().reshape(probs[i].M, probs[i].N)
            dF = abs((1 - float(b.out[i][1])) - ref["F"])
            gr = float(np.linalg.norm(g - ref["grad"]) / max(np.linalg.norm(ref["grad"]), 1e-300))
            worst_F, worst_g = max(worst_F, dF), max(worst_g, gr)
        res_acc = dict(instances=[f"{probs[i].name} d={probs[i].d} N={probs[i].N}" for i in sample],
                       max_dF=worst_F, max_grad_rel=worst_g)
        log(f"[bench] c5 accuracy sample: {res_acc}")

    def timed(fn, iters):
        st = torch.cuda.current_stream(dev)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(iters)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, e in evs:
            a.record(st)
            fn()
            e.record(st)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / iters
        ms = np.array([a.elapsed_time(e) for a, e in evs])
        return dict(p50_ms=float(np.percentile(ms, 50)), p99_ms=float(np.percentile(ms, 99)),
                    mean_ms=float(ms.mean()), wall_ms_per_iter=wall * 1e3, iters=iters,
                    ms=list(ms))

    iters = max(args.steps, 1)
    for _ in range(args.warmup):
        b.iteration(serial=True)
    serial = timed(lambda: b.iteration(serial=True), max(10, iters // 10))
    serial.pop("ms")
    log(f"[bench] c5 per-instance calls: {serial}")
    b.refresh()
    eager = timed(lambda: b.iteration(), max(10, iters // 10))
    eager.pop("ms")
    log(f"[bench] c5 multi-stream eager: {eager}")
    b.capture(warmup=args.warmup)
    # timed replays in chunks; between chunks (untimed) the fixed (p, n) of
    # instances whose theta_max has grown are re-chosen and the graph
    # re-captured
    chunk, ms_all, refreshes = 25, [], 0
    refreshes += b.refresh()
    done = 0
    while done < iters:
        k = min(chunk, iters - done)
        r = timed(b.replay, k)
        ms_all += r.pop("ms")
        done += k
        refreshes += b.refresh()
    ms_all = np.array(ms_all)
    graph = dict(p50_ms=float(np.percentile(ms_all, 50)), p99_ms=float(np.percentile(ms_all, 99)),
                 mean_ms=float(ms_all.mean()), iters=int(len(ms_all)))
    log(f"[bench] c5 graph replays: {graph}, pair refreshes {refreshes}")
    warn = b.taylor_warnings()
    flops = batch_work(probs, b)
    t = graph["p50_ms"] / 1e3
    value = b.total_steps / t
    peak = PEAK[args.precision]["mfma"]
    res = dict(metric=METRIC, value=value, unit="time-steps/s", n_gpus=1, steps=iters,
               warmup=args.warmup, ms_per_step=graph["p50_ms"], higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype=args.precision,
               data="synthetic (seeded generators)",
               config=dict(workload="c5_batched_uneven", instances=len(probs),
                           sum_N=b.total_steps, d_range=[min(p.d for p in probs),
                                                         max(p.d for p in probs)],
                           optimizer="Adam lr=1e-2 (qoc_adam_step kernel)", streams=len(b.streams),
                           precision=args.precision),
               roofline=dict(kernel="whole iteration (graph)", bound="mfma",
                             achieved=flops / t / 1e12, peak=peak / 1e12, unit="TFLOP/s",
                             frac=flops / t / peak, traffic=None),
               graph=graph, eager_multistream=eager, per_instance_calls=serial,
               tiles=dict(pad64=sum(1 for x in b.pads if x == 64), instances=len(probs),
                          tuned=not args.no_tune, setup_s=t_tune),
               speedup_graph_vs_per_instance=serial["p50_ms"] / graph["p50_ms"],
               taylor_pair_refreshes=refreshes, taylor_warnings_last_chunk=len(warn))
    if res_acc:
        res["accuracy_sample"] = res_acc
    b.close()
    print(json.dumps(res), flush=True)


def single_kernel_phases(info, sweep, precision="fp32"):
    """Phases of a cost + gradient call whose every timer brackets exactly
    one kernel launch: the norm (k_norm), the step assembly, each Taylor /
    Paterson-Stockmeyer / squaring stage, the sweeps that run as one kernel
    (not the per-step variant, which padded d >= 80 picks by default for
    the block sweeps), on the small path (padded d <= 32) the block-product
    tree, and at padded d 16 the per-step derivative kernel.  The cost phase
    (two kernels) and the tiled adjoint (a dozen) are not single kernels."""
    dp = info["d_pad"]
    ph = {"norm", "assemble", "taylor"}
    if dp <= 32:
        ph.add("blockprod")
    if dp == 16:
        ph.add("adjoint")
    chain = precision != "fp64" and 64 <= dp <= 128  # variant 4, the default from 64
    for name, v in zip(["fwd_blocks", "fwd_replay", "bwd_blocks", "bwd_pairs"], sweep):
        blocks = name in ("fwd_blocks", "bwd_blocks")
        auto_wide = v == 0 and not chain and (blocks or dp >= 256)
        if dp >= 80 and (v == 2 or auto_wide):
            continue
        ph.add(name)
    return ph


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-torch-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the bf16x3 and other-workload extra keys")
    ap.add_argument("--no-fp64-kernels", action="store_true",
                    help="skip timing this library's FP64-chain kernels")
    ap.add_argument("--streams", type=int, default=4, help="c5: streams per iteration")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the sweep autotuner (checkpoint interval, sweep variants)")
    ap.add_argument("--checkpoint-every", type=int, default=None,
                    help="fix the checkpoint interval instead of tuning it (with --sweep)")
    ap.add_argument("--sweep", default=None,
                    help="fix the four sweep variants, e.g. 1,1,1,1 (with --checkpoint-every)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the time-sharded design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1612_04929_amd import qoc

    if args.config == "c5":
        return bench_batch(args)
    dev = torch.device("cuda:0")
    prob = workloads.make_config(args.config)
    log(f"[bench] {prob.name}: d={prob.d} M={prob.M} N={prob.N} S={prob.S} "
        f"precision={args.precision}")
    from paper_1612_04929_amd import tune as qtune
    tuned = None
    if args.checkpoint_every is not None or args.sweep is not None:
        # a fixed configuration (e.g. the tuned one, for a profiler run
        # whose kernel averages should cover that configuration alone)
        sw = [int(x) for x in (args.sweep or "0,0,0,0").split(",")]
        if len(sw) != 4:
            ap.error("--sweep takes four comma-separated variants")
        tuned = dict(checkpoint_every=args.checkpoint_every or 0, sweep=sw, seconds=0.0,
                     table=[], fixed=True)
        from paper_1612_04929_amd import tune as qtune
    elif not args.no_tune:
        from paper_1612_04929_amd import tune as qtune
        tuned = qtune.tune(prob, precision=args.precision)
        log(f"[bench] tuned: L={tuned['checkpoint_every']} sweeps={tuned['sweep']} "
            f"({tuned['seconds']:.1f} s)")
    h = qoc.Problem(prob, precision=args.precision, device=0,
                    checkpoint_every=tuned["checkpoint_every"] if tuned else 0)
    if tuned:
        qtune.apply(h, tuned)
    u = torch.from_numpy(np.ascontiguousarray(prob.u)).to(dev)
    out = torch.zeros(2 + prob.N, dtype=torch.float64, device=dev)
    grad = torch.zeros(max(1, prob.M * prob.N), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step():
        h.cost_grad_device(u.data_ptr(), out.data_ptr(), grad.data_ptr(), stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region (value): no per-phase events, device-resident inputs
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # second pass of the same length with the library's per-phase HIP
    # events on the launch stream: per-kernel durations for the roofline
    # (the events cost a few microseconds each, so they stay out of `value`)
    h.profile_enable(True)
    h.profile_read(reset=True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_profiled = (time.perf_counter() - tp0) * 1e3 / args.steps
    prof = h.profile_read(reset=True)
    h.profile_enable(False)
    value = prob.N / (ms / 1e3)
    info = h.info()
    C_gpu = float(out[0].item())
    Cfid_gpu = float(out[1].item())
    g_gpu = grad[: prob.M * prob.N].cpu().numpy().reshape(prob.M, prob.N)
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step, {value:.4g} time-steps/s, info={info}")

    kernels = {}
    for ph, (tms, calls) in prof.items():
        if calls:
            kernels[ph] = dict(total_ms=tms / args.steps, launches=calls // args.steps,
                               avg_launch_ms=tms / calls)
    # the roofline kernel: the largest phase whose every timer brackets one
    # kernel launch (so its average is one kernel's average launch time)
    single = single_kernel_phases(info, tuned["sweep"] if tuned else [0, 0, 0, 0], args.precision)
    dom = max((k for k in kernels if k in single), key=lambda k: kernels[k]["total_ms"])
    bound, units = algorithmic_work(prob, info, dom, kernels[dom]["launches"] * args.steps,
                                    args.precision, args.steps)
    avg_s = kernels[dom]["avg_launch_ms"] / 1e3
    def peak_of(phase, b):
        prec = args.precision
        if prec == "bf16x3" and not (phase in BF3_PHASES and info["d_pad"] % 64 == 0):
            prec = "fp32"
        return PEAK[prec][b]

    if bound == "hbm":
        achieved, peak, unit = units / avg_s / 1e9, HBM_PEAK / 1e9, "GB/s"
    else:
        achieved, peak, unit = units / avg_s / 1e12, peak_of(dom, bound) / 1e12, "TFLOP/s"
    tr = TRAFFIC.get((prob.name, dom)) if args.precision == "fp32" else None
    # padded d <= 32 is latency-bound (launch and dependent-step latency, not
    # MFMA or HBM): the kernel's rate is reported without a fraction
    latency = info["d_pad"] <= 32
    roofline = dict(kernel=dom, bound="latency" if latency else bound, achieved=achieved,
                    peak=None if latency else peak, unit=unit,
                    frac=None if latency else achieved / peak,
                    traffic=(tr[1] + tr[2]) if tr else None)
    if tr:
        roofline["traffic_kernel"] = tr[0]
        roofline["traffic_read_bytes"] = tr[1]
        roofline["traffic_written_bytes"] = tr[2]
    for k, v in kernels.items():
        b, un = algorithmic_work(prob, info, k, v["launches"] * args.steps, args.precision,
                                 args.steps)
        s = v["avg_launch_ms"] / 1e3
        v["bound"] = b
        if b == "hbm":
            v["achieved_GBps"] = un / s / 1e9 if s > 0 else None
        else:
            v["achieved_TFLOPs"] = un / s / 1e12 if s > 0 else None

    res = dict(metric=METRIC, value=value, unit="time-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=args.precision, data="synthetic (seeded generators)",
               config=dict(workload=prob.name, d=prob.d, M=prob.M, N=prob.N, S=prob.S,
                           dt=prob.dt, precision=args.precision, taylor_p=info["p"],
                           taylor_n=info["n"], checkpoint_every=info["block_len"]),
               roofline=roofline)
    h.close()  # the comparators below allocate handles and tensors of their own
    golden = os.path.join(ROOT, "tests", "golden", f"{args.config}_full_oracle.npz")
    if os.path.exists(golden):
        # stored FP64 oracle outputs of the full workload (written by
        # tests/golden/make_golden.py, which calls only the oracle)
        with np.load(golden) as z:
            gref, Fref, Cref, cref = z["grad"], float(z["F"]), float(z["C"]), z["c"]
        c_gpu = out[2:].cpu().numpy()
        res["accuracy_vs_oracle"] = dict(
            source=os.path.relpath(golden, ROOT), dF=abs((1 - Cfid_gpu) - Fref),
            dC=abs(C_gpu - Cref), max_dc=float(np.max(np.abs(c_gpu - cref))),
            grad_rel=float(np.linalg.norm(g_gpu - gref) / np.linalg.norm(gref)))
    if not args.no_cpu_baseline:
        cb, (sample, ref) = cpu_baseline(prob, args.cpu_seconds)
        res["cpu_baseline"] = cb
        if sample.N == prob.N and "accuracy_vs_oracle" not in res:
            gref = ref["grad"]
            res["accuracy_vs_oracle"] = dict(
                source="oracle.cost_grad (live)",
                dF=abs((1 - Cfid_gpu) - ref["F"]), dC=abs(C_gpu - ref["C"]),
                max_dc=float(np.max(np.abs(out[2:].cpu().numpy() - ref["c"]))),
                grad_rel=float(np.linalg.norm(g_gpu - gref) / np.linalg.norm(gref)))
    if not args.no_fp64_kernels and args.precision != "fp64":
        # secondary comparator: this library's own kernels with FP64 chains
        # (FP64 MFMA), which separates the algorithmic gain from the precision gain
        h64 = qoc.Problem(prob, precision="fp64", device=0,
                          checkpoint_every=tuned["checkpoint_every"] if tuned else 0)
        g64 = torch.zeros_like(grad)
        o64 = torch.zeros_like(out)
        run64 = lambda: h64.cost_grad_device(u.data_ptr(), o64.data_ptr(), g64.data_ptr(), stream)
        run64()
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            run64()
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t0) / reps
        h64.close()
        res["fp64_own_kernels"] = dict(value=prob.N / t64, unit="time-steps/s",
                                       ms_per_step=t64 * 1e3, reps=reps)
        golden64 = os.path.join(ROOT, "tests", "golden", f"{args.config}_full_oracle.npz")
        if os.path.exists(golden64):
            with np.load(golden64) as z:
                g = g64[: prob.M * prob.N].cpu().numpy().reshape(prob.M, prob.N)
                res["fp64_own_kernels"]["accuracy_vs_oracle"] = dict(
                    dF=abs((1 - float(o64[1])) - float(z["F"])),
                    grad_rel=float(np.linalg.norm(g - z["grad"]) / np.linalg.norm(z["grad"])),
                    max_dc=float(np.max(np.abs(o64[2:].cpu().numpy() - z["c"]))))
    if not args.no_extras:
        # the same call in the other precision and on the other workloads of
        # the metric's range (tuned the same way), as extra keys
        if args.precision == "fp32":
            res["bf16x3"] = quick_measure(prob, "bf16x3", args, tuned)
        if info["d_pad"] >= 64:
            # memory-lean mode: four time segments, every stack a quarter
            # as long, the exponentials formed twice
            torch.cuda.empty_cache()
            r = quick_measure(prob, args.precision, args, tuned, segment_steps=-(-prob.N // 4))
            r["whole_horizon_device_bytes"] = info["device_bytes"]
            r["whole_horizon_ms_per_step"] = ms
            res["memory_lean_4_segments"] = r
        if args.precision != "bf16x3" and prob.S * 8 <= prob.d:
            # the state-mode action form (matrix-vector products, no U_j) on
            # the same workload: it pays where S << d and H_j is sparse
            torch.cuda.empty_cache()
            try:
                r = quick_measure(prob, args.precision, args, None, propagation="action")
                r["matrix_path_ms_per_step"] = ms
                res["action_form"] = r
            except qoc.QocError as e:
                res["action_form"] = dict(unsupported=str(e))
        for name in [c for c in ("c2", "c3") if c != args.config]:
            q = workloads.make_config(name)
            tq = None if args.no_tune else qtune.tune(q, precision=args.precision)
            res.setdefault("other_workloads", {})[name] = quick_measure(q, args.precision, args, tq)
            if name == "c3":
                # the transmon-cavity workload's stated checkpoint interval, 71
                t71 = dict(checkpoint_every=71, sweep=tq["sweep"] if tq else [0, 0, 0, 0])
                res["other_workloads"]["c3_checkpoint_71"] = quick_measure(q, args.precision,
                                                                            args, t71)
                if args.precision == "fp32":
                    # the transmon-cavity workload in the other two precisions,
                    # each with its error against the stored oracle outputs
                    for prec in ("bf16x3", "fp64"):
                        res["other_workloads"][f"c3_{prec}"] = quick_measure(q, prec, args, tq)
    if not args.no_torch_baseline:
        tb = fp64_torch_path(prob, dev)
        g64 = tb.pop("grad")
        tb["dF_vs_this"] = abs(tb.pop("F") - (1 - Cfid_gpu))
        tb["grad_rel_vs_this"] = float(np.linalg.norm(g64 - g_gpu) / np.linalg.norm(g64))
        res["fp64_gpu_path"] = tb
        res["speedup_vs_fp64_gpu_path"] = value / tb["value"]
        torch.cuda.empty_cache()
    # whole call against the MFMA peak: the per-step algorithmic count
    # (3 G products) and the products the kernels execute
    pk = PEAK["fp64" if args.precision == "fp64" else "fp32"]["mfma"]
    wa, we = path_work(prob, info), executed_work(prob, info, args.precision)
    res["path_roofline"] = dict(
        algorithmic_flops=wa, executed_flops=we, ms=ms,
        achieved_algorithmic_TFLOPs=wa / (ms / 1e3) / 1e12,
        achieved_executed_TFLOPs=we / (ms / 1e3) / 1e12, peak_TFLOPs=pk / 1e12,
        frac_algorithmic=None if latency else wa / (ms / 1e3) / pk,
        frac_executed=None if latency else we / (ms / 1e3) / pk)
    res["kernels"] = kernels
    res["ms_per_step_with_phase_events"] = ms_profiled
    if tuned:
        res["tuning"] = dict(checkpoint_every=tuned["checkpoint_every"], sweep=tuned["sweep"],
                             seconds=tuned["seconds"], fixed=bool(tuned.get("fixed")),
                             candidates={r["L"]: round(r["ms"], 4) for r in tuned["table"]})
    res["diagnostics"] = dict(theta_max=info["theta_max"], norm_drift=info["norm_drift"],
                              n_blocks=info["n_blocks"], d_pad=info["d_pad"],
                              device_bytes=info["device_bytes"])
    h.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

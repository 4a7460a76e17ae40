"""Benchmark of the per-time-step hot path on one MI355X.

A "step" is one full time step of eq. (4): ionic update and ion term, right-hand
side, and the two-level additive Schwarz PCG to relative residual 1e-10 from
x0 = U^k -- all in libpdg's HIP kernels.  Workload (default): 3-D cube [0, 10 mm]^3,
40^3 cubes agglomerated into ~8,000 polyhedra, p = 2 (~80k dofs), two tissue
regions (conductivity 1:3), 64 subdomains of uneven size (+-40 %) with a P1
coarse space on them, planar stimulus, plain FP64.

``--workload cfg4`` runs the batching form instead: 64 independent systems
(~1.05M dofs, p = 1..4) in one context per degree, each on its own stream,
stepped together (pdg_step_batch) with PCG chunks replayed as captured graphs.
``cfg3`` is the precision form (64^3 cubes, p = 3, FP32 Schwarz solves, FP64
CG), ``cfg5`` the learned initial guess (trained here on the GPU, evaluated on
held-out steps), ``table1`` the paper's Table-1 experiment (2-D grey/white
square, iterations and condition numbers per fine/coarse mesh pair) and
``fig2`` a 4000-step run of its p = 4 problem.

Prints one JSON line: the metric, time per step, iterations, a roofline record
for the dominant kernel and the oracle's CPU baseline.  Inputs are resident in
HBM before the timed region starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time per CN step & MDoF/s at relres 1e-10; PCG iters; % HBM roofline vs FP64"
# Inside a timed region one Schwarz launch in TIMING_PERIOD carries dispatch
# events.  Each timed launch adds about 6.5 us to its PCG iteration (timing
# every launch would add 6 % to a step of the default workload); one in 32
# adds about 0.2 %.
TIMING_PERIOD = 32


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256[:16] of the kernel source and its header (kernels.hip, kernels.h)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2512_19536_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload_tag, n_launch_bytes):
    """HBM bytes per Schwarz-apply launch from the committed counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"schwarz_apply_{workload_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(problem, n_steps=1):
    """The FP64 oracle (as it stands) on the host cores: setup untimed, then
    `n_steps` time steps timed."""
    from oracle.monodomain import Monodomain
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = cores
    t0 = time.perf_counter()
    md = Monodomain(problem)
    t_setup = time.perf_counter() - t0
    U, Up, Y = md.initial_state()
    t0 = time.perf_counter()
    iters = []
    for _ in range(n_steps):
        U, Up, Y, info = md.step(U, Up, Y)
        iters.append(info.iters)
    dt = (time.perf_counter() - t0) / n_steps
    return {
        "value": problem.n_dof / dt / 1e6,
        "unit": "MDoF/s",
        "cores": int(min(cores, blas_threads)),
        "kind": "oracle",
        "sample": f"first {n_steps} CN step(s) of the same workload (oracle setup {t_setup:.1f} s untimed); "
                  f"s/step {dt:.2f}, PCG iters {iters}; scipy.sparse SpMV single-threaded, dense "
                  f"Cholesky solves on {blas_threads} BLAS threads of {cores} host cores",
    }


def cpu_baseline_batch(batch, min_dofs=40000):
    """The oracle on a bounded sample of the batch: the first systems (in
    generation order) up to `min_dofs` dofs, one CN step each, setup untimed."""
    from oracle.monodomain import Monodomain
    cores = len(os.sched_getaffinity(0))
    picked, tot = [], 0
    for i, q in enumerate(batch.systems):
        picked.append(i)
        tot += q.n_dof
        if tot >= min_dofs:
            break
    t_step, iters = 0.0, []
    for i in picked:
        md = Monodomain(batch.systems[i])
        U, Up, Y = md.initial_state()
        t0 = time.perf_counter()
        U, Up, Y, info = md.step(U, Up, Y)
        t_step += time.perf_counter() - t0
        iters.append(info.iters)
    return {
        "value": tot / t_step / 1e6,
        "unit": "MDoF/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"first CN step of batch systems {picked} ({tot} dofs, FP64 Schwarz, setup untimed), "
                  f"{t_step:.1f} s, PCG iters {iters}",
    }


def bench_batch(args, steps=None, emit=True, graph=None):
    import numpy as np
    import torch

    from paper_2512_19536_amd import _lib
    from paper_2512_19536_amd.solver import BatchSolver
    from pdg_inputs import problems

    t0 = time.perf_counter()
    batch = problems.cfg4()
    log(f"[bench] workload cfg4: {len(batch.systems)} systems, {batch.n_dof} dofs, degrees "
        f"{ {p: len(ix) for p, (_, ix) in batch.groups.items()} }; inputs {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    graph = args.graph if graph is None else graph
    opts = {_lib.PDG_OPT_GRAPH: graph, _lib.PDG_OPT_CHUNK: args.chunk}
    bs = BatchSolver(batch, device="cuda:0", options=opts)
    torch.cuda.synchronize()
    log(f"[bench] library setup {time.perf_counter() - t0:.1f} s")
    n_steps = args.steps if steps is None else steps
    U, Up, Y = bs.initial_state()
    tol, maxit = 1e-10, 5000
    for k in range(args.warmup):
        infos = bs.step(U, Up, Y, tol, maxit)
        log(f"[bench] warmup step {k}: iters per degree {[i['iters'] for i in infos]}")

    def timed_steps():
        torch.cuda.synchronize()
        it = []
        t0 = time.perf_counter()
        for k in range(n_steps):
            infos = bs.step(U, Up, Y, tol, maxit)
            it.append([i["iters"] for i in infos])
        torch.cuda.synchronize()
        return it, (time.perf_counter() - t0) * 1e3 / n_steps

    tune = None
    if args.autotune:
        # every degree context tunes its own split; the steps are timed with
        # the default split first, then with the chosen one
        _, ms_default = timed_steps()
        tune = {"per_context": []}
        for ci, c in enumerate(bs.ctxs):
            res = c.autotune(reps=args.tune_reps)
            tune["per_context"].append(dict(res, p=bs.problems[ci].p))
            log(f"[bench] autotune p={bs.problems[ci].p}: {res}")
        bs.step(U, Up, Y, tol, maxit)  # first step on the new splits (graphs recaptured; untimed)
        tune["ms_per_step_default"] = round(ms_default, 4)
    iters, ms_step = timed_steps()
    if tune:
        tune["ms_per_step_tuned"] = round(ms_step, 4)
        log(f"[bench] default split {tune['ms_per_step_default']:.3f} ms/step, tuned {ms_step:.3f} ms/step")
    sys_iters = [bs.system_info(i)["iters"] for i in range(len(batch.systems))]
    log(f"[bench] {n_steps} steps: {ms_step:.3f} ms/step; max iters per degree {iters[-1]}; "
        f"system iters last step min {min(sys_iters)} max {max(sys_iters)}")
    # kernel timing of the Schwarz apply: one step per context, contexts one after the other
    launches, tot_ms, tot_bytes = 0, 0.0, 0.0
    for ci, c in enumerate(bs.ctxs):
        c.set_option(_lib.PDG_OPT_KERNEL_TIMING, 1)
        c.kernel_timing()
        c.step(U[ci], Up[ci], Y[ci], None, tol, maxit)
        n, ms, by = c.kernel_timing()
        c.set_option(_lib.PDG_OPT_KERNEL_TIMING, 0)
        launches += n
        tot_ms += ms
        tot_bytes += n * by
        log(f"[bench] p={bs.problems[ci].p}: schwarz apply {n} launches, avg {ms / max(n, 1) * 1e3:.1f} us, "
            f"{by / 1e6:.1f} MB -> {by / (ms / max(n, 1) * 1e-3) / 1e9 if n else 0:.0f} GB/s")
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    # the SpMV moves the most bytes in this workload (the p = 3, 4 matrices):
    # each context's SpMV on its own, HIP events on the context's stream
    sp_ms, sp_bytes, sp_launches, sp_ctx = 0.0, 0.0, 0, []
    for ci, c in enumerate(bs.ctxs):
        _, nd_c, n_dof_c, nnzb = c.get_sizes()
        by = nnzb * nd_c * nd_c * 8 + 2 * n_dof_c * 8
        x = U[ci]
        y = torch.empty_like(x)
        reps = 10
        with torch.cuda.stream(c.stream):
            c.spmv(x, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(c.stream)
            for _ in range(reps):
                c.spmv(x, y)
            e1.record(c.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        sp_ms += ms
        sp_bytes += reps * by
        sp_launches += reps
        sp_ctx.append({"p": bs.problems[ci].p, "avg_us": round(ms / reps * 1e3, 1), "bytes": int(by),
                       "gb_s": round(by / (ms / reps * 1e-3) / 1e9, 1)})
        log(f"[bench] p={bs.problems[ci].p}: spmv {ms / reps * 1e3:.1f} us, {by / 1e6:.1f} MB -> "
            f"{by / (ms / reps * 1e-3) / 1e9:.0f} GB/s")
    sp_gbs = sp_bytes / (sp_ms * 1e-3) / 1e9 if sp_ms > 0 else 0.0
    cpu = None
    if emit and not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle ...")
        cpu = cpu_baseline_batch(batch)
        log(f"[bench] cpu baseline: {cpu['value']:.4f} MDoF/s")
    out = {
        "metric": METRIC,
        "value": round(batch.n_dof / (ms_step * 1e-3) / 1e6, 3),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32-schwarz",
        "data": "synthetic",
        "config": {
            "workload": (f"cfg4: batch of {len(batch.systems)} independent 3-D polytopal problems, "
                         f"{batch.n_dof} dofs in total (2k-60k each, p=1..4), ~250-dof subdomains + P1 coarse "
                         f"per system, Schwarz f32/f32, relres 1e-10, one context per degree on its own stream, "
                         f"graph replay {'on' if graph else 'off'}"),
            "n_dof": batch.n_dof, "n_systems": len(batch.systems),
        },
        "pcg_iters": {"max_per_step": int(np.max(iters)), "systems_last_step": {"min": min(sys_iters),
                                                                                 "max": max(sys_iters)}},
        "autotune": tune,
        "roofline": {
            "kernel": "k_spmv (element-block SpMV), each degree context on its own",
            "bound": "hbm",
            "achieved": round(sp_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(sp_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes_per_launch": int(sp_bytes / max(sp_launches, 1)),
            "avg_launch_us": round(sp_ms / max(sp_launches, 1) * 1e3, 2),
            "per_context": sp_ctx,
        },
        "schwarz_roofline": {
            "kernel": "k_schwarz (local + coarse inverse-tile products), all degree contexts",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes_per_launch": int(tot_bytes / max(launches, 1)),
            "avg_launch_us": round(tot_ms / max(launches, 1) * 1e3, 2),
        },
        "cpu_baseline": cpu,
    }
    del bs
    torch.cuda.empty_cache()
    if emit:
        print(json.dumps(out), flush=True)
    return out


def bench_learned(args):
    """Learned initial guess on the cfg2 mesh: 20 training trajectories x 100
    steps generated by the method, training on the GPU, 5 held-out trajectories
    x 100 steps evaluated against plain PCG from U^k and against linear
    extrapolation.  The timed steps are the held-out learned-guess steps
    (features, inference, guess choice and PCG)."""
    import numpy as np
    import torch

    from paper_2512_19536_amd import learned
    from pdg_inputs import problems

    t0 = time.perf_counter()
    train_p, test_p = problems.cfg5(n_steps=args.traj_steps)
    if args.train_trajs:
        train_p = train_p[:args.train_trajs]
    if args.test_trajs:
        test_p = test_p[:args.test_trajs]
    pr0 = test_p[0]
    log(f"[bench] workload cfg5: {len(train_p)} training + {len(test_p)} held-out trajectories x "
        f"{args.traj_steps} steps on {pr0.n_elem} elements, {pr0.n_dof} dofs; inputs {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    trajs = [learned.generate(q, args.traj_steps, log=log) for q in train_p]
    t_gen = time.perf_counter() - t0
    n_elem, nd = pr0.n_elem, pr0.nd
    blk = learned.row_block(n_elem)
    net = learned.Mlp(nd=nd, max_rows=args.batch_steps * blk)
    learned.fit_normalisation(net, trajs, n_samples=64, seed=0)
    net.init_params(0)
    hist, t_train = learned.train(net, trajs, epochs=args.epochs, batch_steps=args.batch_steps, lr=args.lr, seed=0,
                                  log=log)
    # matrix-core throughput of training: timed train steps on a fixed batch
    rows, n_valid = learned.load_batch(net, trajs, [(0, k) for k in range(args.batch_steps)])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 50
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        net.train_step(rows, n_valid, 1e-12)
    ev1.record()
    torch.cuda.synchronize()
    ms_train_step = ev0.elapsed_time(ev1) / reps
    W = learned.WIDTH
    macs = learned.N_IN * W + 2 * W * W + W * learned.N_OUT
    flops = rows * 2 * (2 * macs + (2 * W * W + W * learned.N_OUT))
    tflops = flops / (ms_train_step * 1e-3) / 1e12
    step_bytes = mlp_train_step_bytes(rows)
    mlp_gbs = step_bytes / (ms_train_step * 1e-3) / 1e9
    log(f"[bench] training: {t_train:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}; train step {ms_train_step:.3f} ms "
        f"({rows} rows, {tflops:.1f} TFLOP/s BF16, {step_bytes / 1e6:.0f} MB moved -> {mlp_gbs:.0f} GB/s)")
    recs = [learned.evaluate(net, q, args.traj_steps, log=log) for q in test_p]
    n_l = sum(r["schwarz_timing"][0] for r in recs)
    t_l = sum(r["schwarz_timing"][1] for r in recs)
    by_l = sum(r["schwarz_timing"][0] * r["schwarz_timing"][2] for r in recs)
    sw_gbs = by_l / (t_l * 1e-3) / 1e9 if t_l > 0 else 0.0
    for r in recs:
        del r["schwarz_timing"]
    cat = {k: np.concatenate([r[k] for r in recs]) for k in recs[0]}
    ms = {k: float(np.mean(cat["t_" + k])) for k in ("plain", "extrap", "learned")}
    it = {k: float(np.mean(cat[k])) for k in ("plain", "extrap", "learned")}
    used = float(np.mean(np.asarray(cat["used"]) > 0))
    log(f"[bench] held-out {len(cat['plain'])} steps: iters plain {it['plain']:.2f} extrap {it['extrap']:.2f} "
        f"learned {it['learned']:.2f}; ms/step plain {ms['plain']:.3f} extrap {ms['extrap']:.3f} learned "
        f"{ms['learned']:.3f}; guess used {used:.2f}; max rel diff {float(np.max(cat['diff'])):.1e}")
    out = {
        "metric": METRIC,
        "value": round(pr0.n_dof / (ms["learned"] * 1e-3) / 1e6, 3),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": int(len(cat["plain"])),
        "warmup": 0,
        "ms_per_step": round(ms["learned"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32-schwarz+bf16-mlp",
        "data": "synthetic",
        "config": {
            "workload": (f"cfg5: learned initial guess on the cfg2 mesh ({pr0.n_dof} dofs, p=2, 64 subdomains, "
                         f"FP32 Schwarz), {len(train_p)}x{args.traj_steps} training steps, "
                         f"{len(test_p)}x{args.traj_steps} held-out steps, MLP 96-256-256-256-32 BF16"),
            "n_dof": pr0.n_dof,
        },
        "learned": {
            "iters_mean": it, "ms_per_step": ms,
            "iteration_reduction_vs_plain": round(1.0 - it["learned"] / it["plain"], 4),
            "iteration_reduction_vs_extrap": round(1.0 - it["learned"] / it["extrap"], 4),
            "guess_used_fraction": used, "max_rel_diff_vs_plain": float(np.max(cat["diff"])),
            "training": {"epochs": args.epochs, "seconds": round(t_train, 2), "loss_first": hist[0],
                         "loss_last": hist[-1], "data_generation_s": round(t_gen, 1),
                         "train_step_ms": round(ms_train_step, 4), "rows_per_step": rows},
        },
        "roofline": {
            "kernel": "k_schwarz (FP32 local + coarse inverse-tile products) in the held-out steps",
            "bound": "hbm",
            "achieved": round(sw_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(sw_gbs / HBM_PEAK_GBS, 4),
            "traffic": None,
            "avg_launch_us": round(t_l / max(n_l, 1) * 1e3, 2),
            "algorithmic_bytes_per_launch": int(by_l / max(n_l, 1)),
            "fits_in_256MB_MALL": bool(by_l / max(n_l, 1) < 256e6),
        },
        "mlp_training_roofline": {
            "kernel": "one training step (BF16 MFMA layer products, loss, bias gradients, split sums, Adam)",
            "bound": "hbm",
            "achieved": round(mlp_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(mlp_gbs / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_step": int(step_bytes),
            "mfma_tflops": round(tflops, 2),
            "mfma_frac_of_2.5_pflops": round(tflops / 2500.0, 5),
            "arithmetic_intensity_flop_per_byte": round(flops / step_bytes, 1),
        },
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def mlp_train_step_bytes(rows, split_rows=1024):
    """Algorithmic HBM bytes of one training step of the 96-256-256-256-32 MLP
    on `rows` samples: every product reads its operands once and writes its
    outputs (bf16 activations and gradients with their transposed copies,
    fp32 last-layer output and split partials), plus the loss, bias-gradient,
    split-sum and Adam passes.  At 52 flop/byte the step sits far below the
    BF16 ridge point (2.5 PFLOP/s / 8 TB/s = 312 flop/byte): HBM bounds it."""
    from paper_2512_19536_amd import learned
    dims = [learned.N_IN, learned.WIDTH, learned.WIDTH, learned.WIDTH, learned.N_OUT]
    bf, f4 = 2, 4
    splits = -(-rows // split_rows)
    b = 0
    for l in range(4):
        K, N = dims[l], dims[l + 1]
        b += rows * K * bf + N * K * bf                                  # forward operands
        b += rows * N * (2 * bf if l < 3 else f4)                        # H and H^T, or Y
    n_out = dims[-1]
    b += rows * n_out * (2 * f4 + 2 * bf) + rows * 4                     # loss: Y, T -> dY, dY^T; row weights
    for l in range(3, -1, -1):
        K, N = dims[l], dims[l + 1]
        b += N * rows * bf + K * rows * bf + splits * N * K * f4         # weight gradient: dY^T, H^T -> partials
        b += splits * N * K * f4 + N * K * f4                            # split sums
        b += N * rows * bf + N * f4                                      # bias gradient
        if l > 0:
            b += rows * N * bf + K * N * bf + rows * K * bf + rows * K * 2 * bf  # data gradient with ReLU mask
    n_par = sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(4))
    b += n_par * (4 * f4 + 3 * f4) + 2 * n_par * bf                      # Adam: theta, m, v, grad -> theta, m, v; bf16 copies
    return b


def _mesh_h(mesh):
    """Largest element diameter (max vertex-vertex distance over the cells)."""
    import numpy as np
    h = 0.0
    for e in range(mesh.n_elem):
        v = mesh.cell_geom[mesh.cell_ptr[e]:mesh.cell_ptr[e + 1]].reshape(-1, mesh.dim)
        d = np.sqrt(((v[:, None, :] - v[None, :, :]) ** 2).sum(-1)).max()
        h = max(h, float(d))
    return h


def bench_table1(args):
    """The paper's Table-1 experiment (Section 5) on the library: per fine mesh
    N_h, degree p = q and coarse size H = k h, the mean PCG iterations per time
    step and the Lanczos condition-number estimate (mean over the steps' solves
    and that of the last step);
    plus the unpreconditioned CG rows (B = I).  Prints one line per cell, a
    markdown table beside the paper's numbers, and one JSON line."""
    import numpy as np
    import torch

    from paper_2512_19536_amd import _lib, from_problem, initial_state
    from paper_2512_19536_amd._lib import PdgError
    from pdg_inputs import problems

    dev = "cuda:0"
    with open(os.path.join(ROOT, "tests", "golden", "table1_paper.json")) as f:
        paper = json.load(f)
    ps = [int(v) for v in args.t1_p.split(",")]
    nhs = [int(v) for v in args.t1_nh.split(",")]
    ks = [int(v) for v in args.t1_h.split(",")]
    cells, dofs_steps, solve_s = [], 0, 0.0

    def run(pr, n_steps, precond):
        nonlocal dofs_steps, solve_s
        t0 = time.perf_counter()
        stream = torch.cuda.Stream(device=dev)
        opts = {_lib.PDG_OPT_GRAPH: 1, _lib.PDG_OPT_CHUNK: 16, _lib.PDG_OPT_LANCZOS_CAP: 1 << 15}
        ctx = from_problem(pr, device=dev, options=opts, stream=stream)
        if not precond:
            ctx.set_option(_lib.PDG_OPT_PRECONDITIONER, 0)
        t_setup = time.perf_counter() - t0
        U, Up, Y = initial_state(ctx, pr)
        torch.cuda.synchronize()
        iters, kappas = [], []
        dt = 0.0
        for k in range(n_steps):
            t0 = time.perf_counter()
            info = ctx.step(U, Up, Y, None, pr.tol, 40000)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            iters.append(info["iters"])
            kappas.append(ctx.lanczos()[0])  # outside the timed part
        dofs_steps += pr.n_dof * n_steps
        solve_s += dt
        # kappa from one solve with a seeded random right-hand side (all
        # eigenvectors present, so the extreme Ritz values converge) from x0 = 0
        gen = torch.Generator(device=dev).manual_seed(pr.n_dof)
        b = torch.randn(pr.n_dof, dtype=torch.float64, device=dev, generator=gen)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()  # b and x come from torch's stream; the solve runs on the context's
        info_r = ctx.solve(b, x, pr.tol, 40000)
        kappa_r = ctx.lanczos()[0]
        del ctx
        torch.cuda.empty_cache()
        return {"iters_mean": float(np.mean(iters)), "iters_first": iters[0], "iters_last": iters[-1],
                "kappa_mean": float(np.mean(kappas)), "kappa_last_step": kappas[-1],
                "kappa_random_rhs": kappa_r, "iters_random_rhs": info_r["iters"],
                "ms_per_step": dt * 1e3 / n_steps, "setup_s": round(t_setup, 2)}

    for p in ps:
        for ci, nh in enumerate(nhs):
            col = problems.TABLE1_NH.index(nh) if nh in problems.TABLE1_NH else None
            h = None
            for k in ks + [0]:
                t0 = time.perf_counter()
                pr = problems.table1_problem(nh, p, k if k else ks[-1], n_steps=args.t1_steps)
                if h is None:
                    h = _mesh_h(pr.mesh)
                row = f"H={k}h" if k else "CG"
                cell = {"p": p, "N_h": nh, "h": round(h, 4), "row": row, "n_dof": pr.n_dof,
                        "n_coarse": int(pr.elem_coarse.max()) + 1 if k else 0,
                        "coarse_dofs": (int(pr.elem_coarse.max()) + 1) * pr.nd if k else 0}
                if col is not None and row in paper[f"p{p}"]:
                    kp, ip = paper[f"p{p}"][row][col]
                    cell["paper"] = {"kappa": kp, "iters": ip}
                try:
                    cell.update(run(pr, args.t1_steps if k else args.t1_cg_steps, precond=bool(k)))
                except PdgError as e:
                    cell["error"] = str(e)
                cells.append(cell)
                log(f"[table1] p={p} N_h={nh} {row}: " + json.dumps({kk: v for kk, v in cell.items()
                                                                    if kk not in ("p", "N_h", "row")})
                    + f" ({time.perf_counter() - t0:.1f} s)")
    # markdown summary: ours (paper)
    lines = []
    for p in ps:
        lines.append(f"p = q = {p}: kappa estimate (mean over steps) [from a random right-hand side] / "
                     f"mean iterations per step, this library (paper)")
        lines.append("| row | " + " | ".join(f"N_h={nh}" for nh in nhs) + " |")
        lines.append("|---|" + "---|" * len(nhs))
        for row in [f"H={k}h" for k in ks] + ["CG"]:
            out = []
            for nh in nhs:
                c = next(c for c in cells if c["p"] == p and c["N_h"] == nh and c["row"] == row)
                if "error" in c:
                    out.append("n/a")
                    continue
                txt = f"{c['kappa_mean']:.4g} [{c['kappa_random_rhs']:.4g}] / {c['iters_mean']:.1f}"
                if "paper" in c:
                    txt += f" ({c['paper']['kappa']:.4g} / {c['paper']['iters']})"
                out.append(txt)
            lines.append(f"| {row} | " + " | ".join(out) + " |")
        lines.append("")
    log("\n".join(lines))
    if args.t1_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.t1_out)), exist_ok=True)
        with open(args.t1_out, "w") as f:
            json.dump({"cells": cells, "markdown": lines, "steps": args.t1_steps, "cg_steps": args.t1_cg_steps,
                       "chi_cm": problems.TABLE1_CHI_CM}, f, indent=1)
    out = {
        "metric": "Table-1 experiment: mean PCG iterations per step and Lanczos kappa per (N_h, H, p) cell",
        "value": round(dofs_steps / solve_s / 1e6, 3) if solve_s else None,
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": args.t1_steps,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"table1: 2-D grey/white square, N_h in {nhs}, p = q in {ps}, H = {ks} h, "
                                f"one subdomain per element + q = p coarse, dt 2.5 us, relres 1e-9, "
                                f"{args.t1_steps} steps per cell ({args.t1_cg_steps} for CG)")},
        "cells": cells,
    }
    print(json.dumps(out), flush=True)


def bench_fig2(args):
    """Long run of the Table-1 problem (Section 5, Fig. 2 setting): N_h = 4096,
    p = q = 4, T = 10 ms (4000 steps of 2.5 us), coarse agglomerates H = 4h.
    Reports iterations over time and, at t = 2, 4.8 and 8.4 ms, the element
    means of the potential (min, max, depolarised area, an ASCII map).  The
    ionic constants are not the paper's, so the pictures are qualitative."""
    import numpy as np
    import torch

    from paper_2512_19536_amd import _lib, from_problem, initial_state
    from pdg_inputs import problems

    dev = "cuda:0"
    n_steps = args.fig2_steps
    pr = problems.table1_problem(args.fig2_nh, args.fig2_p, args.fig2_h, n_steps=n_steps, chi_cm=args.fig2_chi_cm)
    log(f"[fig2] {pr.name}: {pr.n_elem} elements, {pr.n_dof} dofs, {int(pr.elem_coarse.max()) + 1} agglomerates")
    stream = torch.cuda.Stream(device=dev)
    ctx = from_problem(pr, device=dev, options={_lib.PDG_OPT_GRAPH: 1, _lib.PDG_OPT_CHUNK: 16}, stream=stream)
    U, Up, Y = initial_state(ctx, pr)
    n, nd = pr.n_elem, pr.nd
    # element means: (1, u)_K / |K| with the coefficients c1 of the constant 1
    _, _, _, mass = ctx.get_matrix()
    with torch.cuda.stream(stream):
        c1 = torch.empty(n * nd, dtype=torch.float64, device=dev)
        ctx.project_p0(torch.ones(1, n, dtype=torch.float64, device=dev), c1)
    stream.synchronize()
    M = torch.tensor(mass, device=dev)
    w = torch.bmm(M, c1.view(n, nd, 1)).view(n, nd)
    vol = (w * c1.view(n, nd)).sum(1)
    cen = pr.mesh.element_centroid()
    gx, gy = 48, 24
    cell = np.clip((np.floor(cen[:, 0] * gx)).astype(int), 0, gx - 1) + gx * np.clip(
        (np.floor((1.0 - cen[:, 1]) * gy)).astype(int), 0, gy - 1)
    snaps_at = {int(round(t / (pr.dt))): t for t in (2.0, 4.8, 8.4)}
    snaps, iters, t0 = [], [], time.perf_counter()
    for k in range(1, n_steps + 1):
        info = ctx.step(U, Up, Y, None, pr.tol, 20000)
        iters.append(info["iters"])
        if k in snaps_at:
            mean = ((w * U.view(n, nd)).sum(1) / vol).cpu().numpy()
            ascii_rows = []
            for r in range(gy):
                row = ""
                for c in range(gx):
                    v = mean[cell == r * gx + c]
                    u = float(v.mean()) if len(v) else float("nan")
                    row += " " if not np.isfinite(u) else ".:-=+*#%@"[int(np.clip((u + 80.0) / 100.0 * 9, 0, 8))]
                ascii_rows.append(row)
            area = float(vol.cpu().numpy()[mean > -40.0].sum())
            snaps.append({"t_ms": snaps_at[k], "step": k, "u_min": float(mean.min()), "u_max": float(mean.max()),
                          "depolarised_area_u_gt_-40mV": area, "map": ascii_rows})
            log(f"[fig2] t = {snaps_at[k]} ms: u in [{mean.min():.1f}, {mean.max():.1f}] mV, area above -40 mV "
                f"{area:.4f}\n" + "\n".join(ascii_rows))
        if k % 250 == 0:
            log(f"[fig2] step {k}: mean iterations of the last 250 steps {np.mean(iters[-250:]):.1f}, "
                f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if args.fig2_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.fig2_out)), exist_ok=True)
        with open(args.fig2_out, "w") as f:
            json.dump({"problem": pr.name, "iters": iters, "snapshots": snaps}, f)
    out = {
        "metric": "long run (T = 10 ms) of the Table-1 problem: iterations over time, potential snapshots",
        "value": round(pr.n_dof * n_steps / dt / 1e6, 3),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": 0,
        "ms_per_step": round(dt * 1e3 / n_steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{pr.name}: {pr.n_dof} dofs, q = p coarse on H = {args.fig2_h}h agglomerates, "
                               f"chi_m C_m = {pr.chi_m * pr.c_m:g}, relres 1e-9, {n_steps} steps of 2.5 us, "
                               f"graph replay"},
        "pcg_iters": {"mean": float(np.mean(iters)), "first": iters[0], "last": iters[-1],
                      "mean_per_1000_steps": [float(np.mean(iters[i:i + 1000])) for i in range(0, n_steps, 1000)]},
        "snapshots": [{k: v for k, v in sn.items() if k != "map"} for sn in snaps],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "table1", "fig2"])
    ap.add_argument("--t1-p", default="1,4", help="table1: degrees p = q")
    ap.add_argument("--t1-nh", default="512,1024,2048,4096", help="table1: fine mesh sizes N_h")
    ap.add_argument("--t1-h", default="2,4,8,16", help="table1: coarse sizes H / h")
    ap.add_argument("--t1-steps", type=int, default=100, help="table1: time steps per preconditioned cell")
    ap.add_argument("--t1-cg-steps", type=int, default=10, help="table1: time steps per unpreconditioned cell")
    ap.add_argument("--t1-out", default=None, help="table1: JSON file for the cells")
    ap.add_argument("--fig2-steps", type=int, default=4000, help="fig2: time steps (4000 = 10 ms)")
    ap.add_argument("--fig2-nh", type=int, default=4096, help="fig2: fine mesh size N_h")
    ap.add_argument("--fig2-p", type=int, default=4, help="fig2: degree p = q")
    ap.add_argument("--fig2-h", type=int, default=4, help="fig2: coarse size H / h")
    ap.add_argument("--fig2-out", default=None, help="fig2: JSON file for iterations and snapshots")
    ap.add_argument("--fig2-chi-cm", type=float, default=None,
                    help="fig2: chi_m C_m (default: the Table-1 calibration)")
    ap.add_argument("--epochs", type=int, default=60, help="cfg5: training epochs")
    ap.add_argument("--batch-steps", type=int, default=4, help="cfg5: time steps per training batch")
    ap.add_argument("--lr", type=float, default=3e-3, help="cfg5: peak learning rate")
    ap.add_argument("--traj-steps", type=int, default=100, help="cfg5: steps per trajectory")
    ap.add_argument("--train-trajs", type=int, default=0, help="cfg5: use only the first N training trajectories")
    ap.add_argument("--test-trajs", type=int, default=0, help="cfg5: use only the first N held-out trajectories")
    ap.add_argument("--graph", type=int, default=None, help="replay PCG chunks as captured graphs (0/1)")
    ap.add_argument("--chunk", type=int, default=4, help="PCG iterations between host polls")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the autotuner (by default the steps are timed before and after it)")
    ap.add_argument("--tune-reps", type=int, default=20, help="PCG iterations per autotuner candidate")
    ap.add_argument("--no-forms", action="store_true",
                    help="cfg2: skip the compact cfg3 (precision) and cfg4 (batch) records")
    ap.add_argument("--form-steps", type=int, default=5, help="timed steps of the compact form records")
    ap.add_argument("--local-prec", default=None, choices=["f64", "f32", "bf16"])
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle time steps in the CPU baseline (about 7 s each at cfg2)")
    ap.add_argument("--item-kb", type=int, default=None, help="Schwarz work-item size (KiB of tiles)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mb", type=int, default=1024)
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="precision form: steps also taken with FP64 Schwarz solves to report the error")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this benchmark runs on one GPU only; a multi-GPU run is not provided "
              "(the path would shard by subdomain, with one halo exchange per SpMV and an "
              "all-reduce of the coarse residual).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "cfg4":
        if args.graph is None:
            args.graph = 1
        return bench_batch(args)
    if args.workload == "cfg5":
        return bench_learned(args)
    if args.workload == "table1":
        return bench_table1(args)
    if args.workload == "fig2":
        return bench_fig2(args)
    if args.graph is None:
        args.graph = 0
    out = bench_single(args, args.workload, args.local_prec, args.steps, args.warmup, args.graph,
                       cpu=not args.no_cpu_baseline, compare_steps=args.compare_steps)
    if args.workload == "cfg2" and not args.no_forms:
        # the precision and batching forms, compact, beside the headline
        out["forms"] = {
            "precision_cfg3": form_record(bench_single(args, "cfg3", "f32", args.form_steps, 1, 0, cpu=False,
                                                       compare_steps=2, also_bf16=True)),
            "batch_cfg4": form_record(bench_batch(args, steps=args.form_steps, emit=False, graph=1)),
        }
    print(json.dumps(out), flush=True)


def form_record(r):
    """The figures of a form's run kept in the headline line."""
    keep = ("value", "unit", "ms_per_step", "ms_per_step_median", "dtype", "config", "pcg_iters",
            "precision_form_error", "oracle_error_step0", "bf16", "autotune", "roofline", "schwarz_roofline")
    return {k: r[k] for k in keep if k in r}


def oracle_fixture_error(name, u0, u1):
    """Error of the first step against the FP64 oracle's stored first step of
    the same workload (tests/golden/<name>_step1.json, sampled entries), or
    None where no such record exists."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}_step1.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        fx = json.load(f)
    idx = np.asarray(fx["idx"])
    U1o, U0o = np.asarray(fx["U1"]), np.asarray(fx["U0"])
    a, a0 = u1.cpu().numpy()[idx], u0.cpu().numpy()[idx]
    # both sides project the same per-element constants, each in its own code
    if np.abs(a0 - U0o).max() > 1e-12 * np.abs(U0o).max():
        return {"error": "initial state differs from the stored one"}
    return {"rel_l2_sampled": float(np.linalg.norm(a - U1o) / np.linalg.norm(U1o)),
            "rel_l2_of_change_sampled": float(np.linalg.norm(a - U1o) / np.linalg.norm(U1o - U0o)),
            "oracle_iters": fx["iters"], "samples": int(len(idx))}


def bench_single(args, workload, local_prec, n_steps, n_warmup, graph, cpu=True, compare_steps=0, also_bf16=False):
    """One workload in one context: `n_warmup` untimed steps from the initial
    state (the first is checked against the oracle's stored first step where
    one exists), the autotuner (unless disabled) with `n_steps` steps timed
    before and after it, the Schwarz roofline, the device-copy ceiling, the
    precision form's error against FP64 Schwarz solves and the CPU baseline."""
    import numpy as np
    import torch

    from paper_2512_19536_amd import _lib, from_problem, initial_state
    from pdg_inputs import problems

    dev = "cuda:0"
    t0 = time.perf_counter()
    pr = problems.BUILDERS[workload]()
    if local_prec:
        pr.local_prec = local_prec
        pr.coarse_prec = "f64" if local_prec == "f64" else "f32"
    log(f"[bench] workload {pr.name}: {pr.n_elem} elements, p={pr.p}, {pr.n_dof} dofs, "
        f"{pr.n_sub} subdomains, Schwarz {pr.local_prec}/{pr.coarse_prec}; inputs {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    opts = {_lib.PDG_OPT_CHUNK: args.chunk}
    if args.item_kb:
        opts[_lib.PDG_OPT_SCHWARZ_ITEM_KB] = args.item_kb
    stream = None
    if graph:
        opts[_lib.PDG_OPT_GRAPH] = 1
        stream = torch.cuda.Stream(device=dev)
    ctx = from_problem(pr, device=dev, options=opts, stream=stream)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"[bench] library setup (assembly, Schwarz inverses, upload) {t_setup:.1f} s")
    U, Up, Y = initial_state(ctx, pr)
    stream = ctx.stream
    oracle_err = None
    for k in range(n_warmup):
        u0 = U.clone() if k == 0 else None
        info = ctx.step(U, Up, Y, None, pr.tol, pr.maxit)
        log(f"[bench] warmup step {k}: iters {info['iters']}"
            + (f", {info['local_fp32']} subdomains stored in FP32" if pr.local_prec == "bf16" else ""))
        if k == 0:
            torch.cuda.synchronize()
            oracle_err = oracle_fixture_error(pr.name, u0, U)
            if oracle_err:
                log(f"[bench] step 0 against the oracle's stored step: {oracle_err}")

    def timed_steps():
        # Schwarz kernel timed with HIP events inside the timed region; with
        # graph replay (no per-launch events possible) in two extra steps after
        if not graph:
            ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, TIMING_PERIOD)
        ctx.kernel_timing()  # reset
        torch.cuda.synchronize()
        iters = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_steps + 1)]
        for k in range(n_steps):
            ev[k].record(stream)
            info = ctx.step(U, Up, Y, None, pr.tol, pr.maxit)
            iters.append(info["iters"])
        ev[n_steps].record(stream)
        torch.cuda.synchronize()
        ms_steps = [ev[k].elapsed_time(ev[k + 1]) for k in range(n_steps)]
        if graph:
            ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, 1)
            for _ in range(2):
                ctx.step(U, Up, Y, None, pr.tol, pr.maxit)
        n_launch, k_ms, k_bytes = ctx.kernel_timing()
        ctx.set_option(_lib.PDG_OPT_KERNEL_TIMING, 0)
        return iters, ms_steps, n_launch, k_ms, k_bytes

    tune = None
    if args.autotune:
        iters0, ms0, _, _, _ = timed_steps()
        res = ctx.autotune(reps=args.tune_reps)
        log(f"[bench] autotune: {res}")
        ctx.step(U, Up, Y, None, pr.tol, pr.maxit)  # first step on the new split (untimed)
        tune = dict(res, ms_per_step_default=round(float(np.mean(ms0)), 4),
                    pcg_iters_default=float(np.mean(iters0)))
    iters, ms_steps, n_launch, k_ms, k_bytes = timed_steps()
    ms_step = float(np.mean(ms_steps))
    if tune:
        tune["ms_per_step_tuned"] = round(ms_step, 4)
        log(f"[bench] default split {tune['ms_per_step_default']:.3f} ms/step, tuned {ms_step:.3f} ms/step")
    log(f"[bench] {n_steps} steps: {ms_step:.3f} ms/step, iters {iters}")
    k_avg_ms = k_ms / max(n_launch, 1)
    achieved = k_bytes / (k_avg_ms * 1e-3) / 1e9 if n_launch else 0.0
    log(f"[bench] schwarz apply: {n_launch} launches, avg {k_avg_ms * 1e3:.1f} us, {k_bytes / 1e6:.1f} MB "
        f"-> {achieved:.0f} GB/s")

    # plain copy of known size, for calibrating HBM byte counters in profiles,
    # then timed: the copy ceiling (bytes read + written per second) on this machine
    nb = args.copy_calibration_mb * (1 << 20)
    src = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(3):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * nb * 3 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    log(f"[bench] device copy of {nb >> 20} MiB: {copy_gbs:.0f} GB/s (read + write)")
    del src, dst

    # precision form: error per step against the same steps taken with FP64
    # Schwarz solves (the FP64 path is the one checked against the oracle);
    # with also_bf16, BF16-stored local solves take the same steps too
    prec_err, bf16 = None, None
    if pr.local_prec != "f64" and compare_steps > 0:
        log(f"[bench] precision form: {compare_steps} steps beside an FP64-Schwarz context")
        ref = from_problem(pr, device=dev, local_prec="f64", coarse_prec="f64",
                           options={_lib.PDG_OPT_TRUE_RESIDUAL: 1})
        alt = None
        if also_bf16:
            t0 = time.perf_counter()
            alt = from_problem(pr, device=dev, local_prec="bf16", coarse_prec="f32",
                               options={_lib.PDG_OPT_TRUE_RESIDUAL: 1})
            torch.cuda.synchronize()
            log(f"[bench] BF16-store setup {time.perf_counter() - t0:.1f} s")
            bf16 = {"steps": []}
        ctx.set_option(_lib.PDG_OPT_TRUE_RESIDUAL, 1)
        prec_err = []
        for k in range(compare_steps):
            u2, up2, y2 = U.clone(), Up.clone(), Y.clone()
            u3, up3, y3 = U.clone(), Up.clone(), Y.clone()
            i_lo = ctx.step(U, Up, Y, None, pr.tol, pr.maxit)
            i_hi = ref.step(u2, up2, y2, None, pr.tol, pr.maxit)
            torch.cuda.synchronize()
            err = float((U - u2).norm() / u2.norm())
            prec_err.append({"step": k, "rel_l2_vs_f64": err, "iters": i_lo["iters"], "iters_f64": i_hi["iters"],
                             "true_relres": i_lo["true_relres"]})
            log(f"[bench]   step {k}: rel L2 vs FP64 {err:.2e}, iters {i_lo['iters']} (FP64 {i_hi['iters']}), "
                f"true relres {i_lo['true_relres']:.2e}")
            if alt is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(alt.stream)
                i_b = alt.step(u3, up3, y3, None, pr.tol, pr.maxit)
                e1.record(alt.stream)
                torch.cuda.synchronize()
                err_b = float((u3 - u2).norm() / u2.norm())
                bf16["steps"].append({"step": k, "rel_l2_vs_f64": err_b, "iters": i_b["iters"],
                                      "true_relres": i_b["true_relres"], "ms": round(e0.elapsed_time(e1), 3)})
                bf16["local_fp32"] = i_b["local_fp32"]
                log(f"[bench]   BF16 store: rel L2 vs FP64 {err_b:.2e}, iters {i_b['iters']}, true relres "
                    f"{i_b['true_relres']:.2e}, {i_b['local_fp32']} subdomains in FP32, {e0.elapsed_time(e1):.2f} ms")
        ctx.set_option(_lib.PDG_OPT_TRUE_RESIDUAL, 0)
        del ref, alt
        torch.cuda.empty_cache()

    tag = pr.name + ("" if pr.local_prec == "f64" else "_" + pr.local_prec)
    traffic = traffic_from_profiles(tag, k_bytes)
    roof = {
        "kernel": "k_schwarz (local + coarse inverse-tile products)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": int(k_bytes),
        "avg_launch_us": round(k_avg_ms * 1e3, 2),
        "copy_ceiling_gb_s": round(copy_gbs, 1),
        "frac_of_copy_ceiling": round(achieved / copy_gbs, 4) if copy_gbs > 0 else None,
        "fits_in_256MB_MALL": bool(k_bytes < 256e6),
    }
    cpu_rec = None
    if cpu:
        log("[bench] cpu baseline: oracle ...")
        cpu_rec = cpu_baseline(pr, args.cpu_steps)
        log(f"[bench] cpu baseline: {cpu_rec['value']:.4f} MDoF/s")
    dtype = {"f64": "f64", "f32": "f64+f32-schwarz", "bf16": "f64+bf16-schwarz"}[pr.local_prec]
    return {
        "metric": METRIC,
        "value": round(pr.n_dof / (ms_step * 1e-3) / 1e6, 3),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": n_warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"{pr.name}: {'3-D' if pr.mesh.dim == 3 else '2-D'} polytopal mesh, {pr.n_elem} elements, "
                         f"p={pr.p}, {pr.n_dof} dofs, {pr.n_sub} subdomains + P1 coarse, "
                         f"Schwarz {pr.local_prec}/{pr.coarse_prec}, relres {pr.tol:g}"
                         f"{', graph replay' if graph else ''}"),
            "n_dof": pr.n_dof, "n_elem": pr.n_elem, "p": pr.p, "n_sub": pr.n_sub,
        },
        "pcg_iters": {"mean": float(np.mean(iters)), "min": int(min(iters)), "max": int(max(iters))},
        "ms_per_step_median": round(float(np.median(ms_steps)), 4),
        "setup_s": round(t_setup, 1),
        "oracle_error_step0": oracle_err,
        "precision_form_error": prec_err,
        "bf16": bf16,
        "autotune": tune,
        "roofline": roof,
        "cpu_baseline": cpu_rec,
    }

if __name__ == "__main__":
    main()

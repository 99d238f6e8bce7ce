"""Throughput of the NLPR fusion ADMM on one MI355X.

One step = one whole solve of the hot path on one synthetic scene already resident in HBM:
guide weights, initial values and `iters` ADMM iterations (X-update by FFT, blur, P1/P2/dual
update, the fused Q/Sigma sweep, right-hand-side assembly).  The default workload is the
512 x 512 x 128-band HS+MS scene (4-band MS guide, 9x9 blur, d = 4, patch 5x5, window 11x11,
100 iterations).

Prints one JSON line: pixel*band*iteration/s over the timed steps, the roofline of the
dominant kernel (the sweep, timed with HIP events on the solve's stream inside the timed
region) and the FP64 oracle's throughput on a bounded sample (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
SWEEP_SRC = os.path.join(ROOT, "paper_2210_04184_amd", "csrc", "sweep.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_c3_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_name(spec) -> str:
    kind = {"c1": "pansharpening", "c2": "hs+pan", "c3": "hs+ms"}.get(spec.name, spec.name)
    return (f"{kind} {spec.p}x{spec.q}x{spec.L}, Lh={spec.Lh}, d={spec.d}, "
            f"blur {2 * spec.blur_radius + 1}x{2 * spec.blur_radius + 1}, patch "
            f"{2 * spec.K + 1}x{2 * spec.K + 1}, window {2 * spec.Sw + 1}x{2 * spec.Sw + 1}, "
            f"{spec.iters} iterations")


def sweep_bytes_per_launch(spec, npairs: int) -> int:
    """HBM bytes of one sweep launch were Sigma' stored densely: Sigma' read + write (8 B per
    pair, patch offset, pixel and band), X read and C write (8 B per pixel and band),
    thresholds mu read once (4 B per pair and pixel)."""
    npatch = (2 * spec.K + 1) ** 2
    n = spec.p * spec.q
    return (8 * npairs * npatch + 8) * n * spec.L + 4 * npairs * n


def coded_sweep_bytes(spec, npairs: int, lx: int, counts):
    """Algorithmic HBM bytes of each sweep launch of a solve with the coded Sigma' (one code
    byte per float4 item, and 16 B per open item): launch t reads the codes and open items
    launch t-1 wrote (nothing for t = 0) and writes its own, plus X read, C write and mu read
    once.  counts[t] = open items written by launch t (nlpr_sweep_counts)."""
    npatch = (2 * spec.K + 1) ** 2
    n = spec.p * spec.q
    items = npairs * npatch * n * lx // 4
    fixed = 8 * n * lx + 4 * npairs * n
    out = []
    for t, c in enumerate(counts):
        rd = (items + 16 * counts[t - 1]) if t > 0 else 0
        out.append(fixed + rd + items + 16 * c)
    return out


def sweep_shape_stream(plan, ws, spec, lx: int, reps: int = 3):
    """GB/s of the library's sweep-shaped reference stream (nlpr_stream_chunks) over the
    solve's own dual-state region, run after the timed solves (it overwrites Sigma'): one
    chunk per (tile, band) workgroup of the sweep, holding the Sigma' that workgroup streams,
    a step of the 2K+1 planes of one patch row, and the sweep's LDS per workgroup.  The rate
    is the ceiling of the sweep's access pattern on the same footprint."""
    import torch
    from paper_2210_04184_amd import nlpr
    inf = plan.info()
    off, nbytes = plan.region(nlpr.REGION_SIGMA)
    nchunks = lx * inf.ntiles
    chunk, kw = nbytes // nchunks, 2 * spec.K + 1
    if chunk == 0 or chunk % (4096 * kw):
        return None
    rows, q = inf.tile_rows, spec.q
    lds = 4 * ((rows + 2 * spec.K) * q + 2 * (rows + inf.halo_rows) * q)
    run = lambda: nlpr.stream_chunks(ws, chunk, nchunks, lx, kw, lds, offset=off)
    run()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        run()
    e.record()
    torch.cuda.synchronize()
    return round(2 * chunk * nchunks * reps / (s.elapsed_time(e) * 1e-3) / 1e9, 1)


def sweep_kernel_sha() -> str:
    """sha256 of the sweep kernel's source text (between its begin / end markers)."""
    import hashlib
    with open(SWEEP_SRC) as f:
        src = f.read()
    a = src.index("// ---- sweep kernel begin")
    b = src.index("// ---- sweep kernel end")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def measured_traffic(config: str):
    """The committed rocprofv3 counter record of the sweep (HBM bytes per launch of the
    profiled launches, and their ratio to the algorithmic bytes of the same launches), if it
    was taken on the current sweep source and workload; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        sha = sweep_kernel_sha()
    except (OSError, ValueError):
        return None
    if rec.get("sweep_source_sha256") != sha or rec.get("config") != config:
        return None
    return rec


def hbm_reference(gib: float):
    """Plain torch copy and in-place negation, and the library's reference stream (in-place,
    one 16-byte non-temporal load and store per thread, the sweep's access pattern), over
    `gib` GiB buffers, event-timed on the current stream: the practical HBM ceilings for a
    streaming read+write, and the copy kernel of known size whose FETCH_SIZE / WRITE_SIZE
    counters calibrate the traffic figures."""
    import torch
    n = int(gib * 1024 ** 3) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    out = {}
    from paper_2210_04184_amd import nlpr
    for name, fn in (("copy", lambda: y.copy_(x)), ("inplace_rmw", lambda: x.neg_()),
                     ("inplace_rmw_nt16", lambda: nlpr.stream_rmw(x))):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(3):
            fn()
        e.record()
        torch.cuda.synchronize()
        out[name + "_GBs"] = round(2 * 4 * n * 3 / (s.elapsed_time(e) * 1e-3) / 1e9, 1)
    out["bytes_each_way"] = 4 * n
    del x, y
    torch.cuda.empty_cache()
    return out


def host_cores() -> int:
    """Cores this process may use (its CPU affinity), at most 16: the host share one GPU
    comes with."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model() -> dict:
    """Model name, family / model / stepping numbers and clock of the first host CPU, as
    /proc/cpuinfo gives them (a virtual machine may shorten the name)."""
    keys = {"model name": "cpu", "cpu family": "family", "model": "model",
            "stepping": "stepping", "cpu MHz": "mhz"}
    out = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if not ln.strip():
                    break                       # first processor only
                k, _, v = ln.partition(":")
                k = k.strip()
                if k in keys:
                    out[keys[k]] = v.strip()
    except OSError:
        pass
    return out


def cpu_baseline(seconds_target: float = 12.0):
    """The FP64 oracle on a sample of the same workload: a 32 x 32 scene with all 128 bands
    of the HS+MS workload, its 4-band guide, 9x9 blur, decimation 4, patch 5x5 and window
    11x11, drawn by the same generator; ADMM iterations until ``seconds_target`` has passed,
    once on every usable host core (the oracle's (shift, patch offset) loops on a thread
    pool, results bit-identical to one thread) and once on one thread."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import nlpr_oracle as o

    spec = synth.config("c3", p=32, q=32, iters=1)
    sc = synth.make_scene(spec)
    pr = o.Problem.from_scene(sc)
    Yl, Yh = sc.Yl.astype(np.float64), sc.Yh.astype(np.float64)

    def timed(workers):
        with threadpool_limits(1), ThreadPoolExecutor(max_workers=workers) as pool:
            t0 = time.perf_counter()
            iters = 0
            X, st = o.initial_state(Yl, pr)
            den = o.denominator(pr.p, pr.q, pr.b, pr.window, pr.K)
            mu = pr.lam * o.weights(Yh, pr.window, pr.K, pr.h) / pr.rho
            F = o.p2_matrix(pr)
            while True:
                X, st = o.admm_step(st, Yl, Yh, pr, den, mu, F, pool if workers > 1 else None)
                iters += 1
                if time.perf_counter() - t0 >= seconds_target:
                    break
            return iters, time.perf_counter() - t0

    cores = host_cores()
    it_n, dt_n = timed(cores)
    it_1, dt_1 = timed(1)
    pb = spec.p * spec.q * spec.L
    return {"value": pb * it_n / dt_n, "unit": "pixel*band*iter/s", "cores": cores,
            "kind": "oracle",
            "host": {**cpu_model(), "cpu_count": os.cpu_count(), "cores_used": cores},
            "one_thread_value": pb * it_1 / dt_1,
            "sample": f"literal FP64 oracle, 32x32x128 bands, Lh=4, 9x9 blur, d=4, patch 5x5, "
                      f"window 11x11: {it_n} iterations incl. weights/setup in {dt_n:.1f} s on "
                      f"{cores} threads; {it_1} in {dt_1:.1f} s on 1 thread"}


def run_batch(args):
    """The 48-scene workload: every stage one launch over all scenes, the whole solve one HIP
    graph; compared with the same scenes solved one after another (one plan each, also
    graph-captured) on the same GPU."""
    import numpy as np
    import torch

    import synth
    from paper_2210_04184_amd import nlpr

    iters = args.iters if args.iters is not None else 100
    specs = synth.batch_specs(48, iters=iters)
    log(f"[bench] generating 48 scenes")
    scenes = [synth.make_scene(s) for s in specs]
    Yls = [torch.from_numpy(s.Yl).cuda() for s in scenes]
    Yhs = [torch.from_numpy(s.Yh).cuda() for s in scenes]
    batch = nlpr.Batch.from_scenes(scenes, flags=nlpr.GRAPH)
    ws = batch.alloc_workspace()
    Zs = [torch.empty((s.spec.L, s.spec.p, s.spec.q), device="cuda") for s in scenes]
    log(f"[bench] batch workspace {batch.workspace_bytes / 1e9:.1f} GB")
    for i in range(args.warmup):
        batch.solve(Yls, Yhs, Zs=Zs, ws=ws)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        batch.solve(Yls, Yhs, Zs=Zs, ws=ws)
        torch.cuda.synchronize()
        log(f"[bench] batched step {i + 1} done at {time.perf_counter() - t0:.2f} s")
    elapsed = time.perf_counter() - t0
    finite = all(bool(torch.isfinite(z).all().item()) for z in Zs)
    Zb = [z.clone() for z in Zs]
    del ws
    torch.cuda.empty_cache()
    # sequential: one plan per scene, solved one after another
    plans = [nlpr.Plan.from_scene(sc, flags=nlpr.GRAPH) for sc in scenes]
    wsz = max(p.workspace_bytes for p in plans)
    ws1 = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    for p, yl, yh, z in zip(plans, Yls, Yhs, Zs):      # warm-up: graph capture per plan
        p.solve(yl, yh, Z=z, ws=ws1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        for p, yl, yh, z in zip(plans, Yls, Yhs, Zs):
            p.solve(yl, yh, Z=z, ws=ws1)
        torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    same = all(torch.equal(a, b) for a, b in zip(Zb, Zs))
    pbi = sum(s.p * s.q * s.L for s in specs) * iters
    npairs = [(2 * s.Sw + 1) ** 2 // 2 for s in specs]
    sweep_bytes = sum((8 * n * (2 * s.K + 1) ** 2 + 8) * s.p * s.q * s.L + 4 * n * s.p * s.q
                      for n, s in zip(npairs, specs))
    out = {
        "metric": "ADMM pixel*band*iter/s (+ % HBM roofline) at <=1e-4 rel. RMSE vs FP64 oracle",
        "value": pbi * args.steps / elapsed, "unit": "pixel*band*iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"48 scenes, sizes 128^2..512^2, 4..128 bands, d 4/8, PAN or "
                               f"4-band MS guide, patch 3x3, window 3x3, {iters} iterations",
                   "seed": 1000, "scenes": len(specs)},
        "sequential_pbi_per_s": pbi * args.steps / seq,
        "batched_over_sequential": seq / elapsed,
        "batched_equals_sequential": same, "finite": finite,
        "sweep_bytes_per_iteration": sweep_bytes,
        "sweep_bound_GBs_if_all_time_in_sweep": sweep_bytes * iters * args.steps / elapsed / 1e9,
    }
    print(json.dumps(out), flush=True)


def run_grad(args):
    """The differentiated workload: 256 x 256 x 31 bands, 3-band guide, 7x7 blur, d = 4,
    patch and window 3x3, 20 unrolled iterations, loss = mean squared error to the ground
    truth.  One step = forward with checkpoints + reverse pass (gradients with respect to
    Y_l, Y_h, lambda_2, rho); compared with the plain solve of the same scene."""
    import numpy as np
    import torch

    import synth
    from paper_2210_04184_amd import nlpr

    spec = synth.config("c5")
    if args.iters is not None:
        spec = spec.replace(iters=args.iters)
    sc = synth.make_scene(spec)
    Yl = torch.from_numpy(sc.Yl).cuda()
    Yh = torch.from_numpy(sc.Yh).cuda()
    Zt = torch.from_numpy(sc.Z).cuda()
    plan = nlpr.Plan.from_scene(sc)
    ckb, gwsb = plan.grad_sizes()
    ws = plan.alloc_workspace()
    ck = torch.empty(ckb, dtype=torch.uint8, device="cuda")
    gws = torch.empty(gwsb, dtype=torch.uint8, device="cuda")
    Z = torch.empty((spec.L, spec.p, spec.q), device="cuda")
    log(f"[bench] checkpoints {ckb / 1e9:.2f} GB, gradient workspace {gwsb / 1e9:.2f} GB")

    def grad_step():
        plan.forward(Yl, Yh, Z=Z, ws=ws, ck=ck)
        dZ = (2.0 * (Z.double() - Zt) / Z.numel()).float()
        return plan.backward(Yl, Yh, dZ, ws, ck, gws=gws)

    def timed(fn, n):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    t_grad = timed(grad_step, args.steps)
    t_fwd = timed(lambda: plan.forward(Yl, Yh, Z=Z, ws=ws, ck=ck), args.steps)
    t_solve = timed(lambda: plan.solve(Yl, Yh, Z=Z, ws=ws), args.steps)
    dYl, dYh, ds = grad_step()
    torch.cuda.synchronize()
    # untimed check of the scalar gradients: central differences of the loss over plain
    # solves at a relative step of 1e-3 (the loss is piecewise smooth; 1e-2 agreement)
    def loss_at(**over):
        Zs, _ = nlpr.Plan.from_scene(sc, **over).solve(Yl, Yh)
        return float(torch.mean((Zs.double() - Zt) ** 2))
    fd = {}
    for i, (name, val) in enumerate((("lam", spec.lam), ("rho", spec.rho))):
        h = 1e-3 * val
        d = (loss_at(**{name: val + h}) - loss_at(**{name: val - h})) / (2 * h)
        fd[name] = {"reverse": float(ds[i]), "central_difference": d,
                    "rel_err": abs(float(ds[i]) - d) / max(abs(d), 1e-300)}
    pbi = spec.p * spec.q * spec.L * spec.iters
    out = {
        "metric": "ADMM pixel*band*iter/s (+ % HBM roofline) at <=1e-4 rel. RMSE vs FP64 oracle",
        "value": pbi / t_grad, "unit": "pixel*band*iter/s (forward + reverse)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_grad * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"differentiated: {spec.p}x{spec.q}x{spec.L}, Lh={spec.Lh}, "
                               f"d={spec.d}, blur {2 * spec.blur_radius + 1}x"
                               f"{2 * spec.blur_radius + 1}, patch 3x3, window 3x3, "
                               f"{spec.iters} unrolled iterations, MSE loss",
                   "seed": spec.seed},
        "forward_with_checkpoints_ms": t_fwd * 1e3,
        "reverse_ms": (t_grad - t_fwd) * 1e3,
        "plain_solve_ms": t_solve * 1e3,
        "gradient_step_over_plain_solve": t_grad / t_solve,
        "checkpoint_bytes": ckb, "gradient_workspace_bytes": gwsb,
        "grads_finite": bool(torch.isfinite(dYl).all() and torch.isfinite(dYh).all()),
        "dlambda_drho": [float(x) for x in ds.cpu()],
        "fd_check": fd,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--iters", type=int, default=None, help="override the iteration count")
    ap.add_argument("--bands", type=int, default=None,
                    help="override the band count (e.g. 16: one GPU's share of the 128-band "
                         "scene split over 8 GPUs by bands)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 3x3 plain-solve leg of the default run")
    ap.add_argument("--subspace", type=int, default=0,
                    help="Ls > 0: solve for Z = X E with E the Ls leading right singular "
                         "vectors of Y_l")
    ap.add_argument("--graph", action="store_true",
                    help="solve through one captured HIP graph (stage timers off): the form "
                         "for small, launch-bound scenes")
    ap.add_argument("--fused", action="store_true",
                    help="the splitting with S inside the X-update (no P1)")
    ap.add_argument("--monitor", type=int, default=0,
                    help="record the objective and residuals every N iterations (0 = off; "
                         "the default run keeps it off)")
    ap.add_argument("--calib-gib", type=float, default=4.0,
                    help="size of the reference copy (0 = skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU only: the solve of one scene is "
                          "not split across GPUs; run with --gpus 1"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2210_04184_amd import nlpr

    if args.config == "c4":
        return run_batch(args)
    if args.config == "c5":
        return run_grad(args)
    spec = synth.config(args.config)
    if args.iters is not None:
        spec = spec.replace(iters=args.iters)
    if args.bands is not None:
        spec = spec.replace(L=args.bands)
    ref = hbm_reference(args.calib_gib) if args.calib_gib > 0 else None
    if ref:
        log(f"[bench] reference streams: {ref}")
    res = measure_solve(spec, args.steps, args.warmup, subspace=args.subspace, graph=args.graph,
                        fused=args.fused, monitor=args.monitor, shape_stream=ref is not None,
                        traffic_key=None if (args.subspace or args.bands) else args.config)
    if ref and res["sweep_shape_stream_GBs"]:
        ref["sweep_shape_stream_GBs"] = res["sweep_shape_stream_GBs"]
    out = {
        "metric": "ADMM pixel*band*iter/s (+ % HBM roofline) at <=1e-4 rel. RMSE vs FP64 oracle",
        "value": res["value"], "unit": "pixel*band*iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_name(spec) + (f", subspace Ls={args.subspace}"
                                                      if args.subspace else "")
                   + (", fused-S X-update" if args.fused else "")
                   + (", one HIP graph" if args.graph else ""),
                   "p": spec.p, "q": spec.q, "L": spec.L, "Ls": args.subspace or spec.L,
                   "Lh": spec.Lh, "d": spec.d, "blur": 2 * spec.blur_radius + 1,
                   "patch": 2 * spec.K + 1, "window": 2 * spec.Sw + 1, "iters": spec.iters,
                   "lambda": spec.lam, "rho": spec.rho, "seed": spec.seed},
        "roofline": res["roofline"],
        "loop_pbi_per_s": res["loop_pbi_per_s"],
        "loop": res["loop"],
        "stages": res["stages"], "finite": res["finite"], "hbm_reference": ref,
    }
    if args.monitor:
        out["monitor"] = res["monitor"]
    if args.config == "c3" and not (args.subspace or args.bands or args.fused or args.graph
                                    or args.iters is not None) and not args.no_small:
        # the paper's own window and patch (3x3 / 3x3) on the differentiated workload's
        # scene, plain solve: the same measurement at a small dual state
        c5 = synth.config("c5")
        log(f"[bench] 3x3 leg: {workload_name(c5)}")
        r5 = measure_solve(c5, 10, 2, shape_stream=ref is not None)
        out["w3p3_plain_solve"] = {
            "workload": workload_name(c5), "pbi_per_s": r5["value"],
            "ms_per_solve": r5["ms_per_step"], "loop": r5["loop"], "roofline": r5["roofline"],
            "stages": r5["stages"], "finite": r5["finite"]}
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def measure_solve(spec, steps, warmup, subspace=0, graph=False, fused=False, monitor=0,
                  shape_stream=False, traffic_key=None):
    """Solve one synthetic scene `warmup` + `steps` times with the inputs resident in HBM: the
    timed region, on a plan without stage timers (an event recorded between two launches
    costs a short kernel several microseconds).  Then, unless the solve runs as one graph,
    solve it again on a plan with HIP events around every stage launch for the per-stage
    times, the sweep's launch duration and open-item counts (the roofline), the loop's HBM
    fraction and the sweep-shaped reference stream."""
    import numpy as np
    import torch

    import synth
    from paper_2210_04184_amd import nlpr

    log(f"[bench] generating {workload_name(spec)}")
    sc = synth.make_scene(spec)
    dev = torch.device("cuda:0")
    Yl = torch.from_numpy(sc.Yl).to(dev)
    Yh = torch.from_numpy(sc.Yh).to(dev)
    E = None
    if subspace:
        M = sc.Yl.reshape(spec.L, -1).T.astype(np.float64)
        E = np.ascontiguousarray(np.linalg.svd(M, full_matrices=False)[2][:subspace],
                                 dtype=np.float32)
    form = nlpr.FUSED_S if fused else 0
    plan = nlpr.Plan.from_scene(sc, flags=(nlpr.GRAPH if graph else 0) | form, E=E,
                                monitor_every=monitor)
    npairs = len(plan.half_window())
    ws = plan.alloc_workspace()
    Z = torch.empty((spec.L, spec.p, spec.q), dtype=torch.float32, device=dev)
    log(f"[bench] workspace {plan.workspace_bytes / 1e9:.1f} GB; warmup {warmup}")
    for i in range(warmup):
        plan.solve(Yl, Yh, Z=Z, ws=ws)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_s = []
    for i in range(steps):
        t1 = time.perf_counter()
        plan.solve(Yl, Yh, Z=Z, ws=ws)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t1)
        log(f"[bench] step {i + 1} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    finite = bool(torch.isfinite(Z).all().item())
    mon = ([dict(zip(nlpr.MON_FIELDS, map(float, r))) for r in plan.monitor()]
           if monitor else None)
    plan.close()
    value = spec.p * spec.q * spec.L * spec.iters * steps / elapsed
    lx = subspace or spec.L

    # stage timers: per-stage HIP events, the sweep's open-item counts
    stages, counts, shape_gbs, prof_steps = {}, [], None, 0
    if not graph:
        prof_steps = max(1, min(steps, 3))
        tplan = nlpr.Plan.from_scene(sc, flags=nlpr.TIMING | form, E=E)
        tplan.solve(Yl, Yh, Z=Z, ws=ws)
        torch.cuda.synchronize()
        for st in nlpr.STAGE_NAMES:
            tplan.stage_time(st, reset=True)
        for i in range(prof_steps):
            tplan.solve(Yl, Yh, Z=Z, ws=ws)
            torch.cuda.synchronize()
        log(f"[bench] {prof_steps} solves with stage timers done")
        for st, name in nlpr.STAGE_NAMES.items():
            ms, n = tplan.stage_time(st)
            if n:
                stages[name] = {"ms_total": round(ms, 3), "launches": n,
                                "ms_avg": round(ms / n, 4)}
        counts = tplan.sweep_counts() if npairs else []
        if shape_stream and npairs:
            shape_gbs = sweep_shape_stream(tplan, ws, spec, lx)
        tplan.close()
    sw = stages.get("sweep")
    roof = None
    sweep_bytes = coded_sweep_bytes(spec, npairs, lx, counts) if counts else []
    if sw and len(sweep_bytes) > 1:
        # the timed "sweep" launches are iterations 2 .. T of every solve (the first sweep of a
        # solve, which reads no state, is timed as "sweep_first")
        bytes_launch = sum(sweep_bytes[1:]) / len(sweep_bytes[1:])
        achieved = bytes_launch / (sw["ms_avg"] * 1e-3) / 1e9
        dense = sweep_bytes_per_launch(spec.replace(L=lx), npairs)
        items = npairs * (2 * spec.K + 1) ** 2 * spec.p * spec.q * lx // 4
        roof = {"bound": "hbm", "kernel": "sweep_kernel", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": round(bytes_launch),
                "ms_per_launch": sw["ms_avg"],
                "open_item_fraction": round(sum(counts[1:]) / len(counts[1:]) / items, 4),
                "dense_format_bytes_per_launch": dense,
                "dense_format_equivalent_GBs": round(dense / (sw["ms_avg"] * 1e-3) / 1e9, 1),
                "frac_of_sweep_shape_stream": round(achieved / shape_gbs, 4) if shape_gbs else None}
    tr = measured_traffic(traffic_key) if (traffic_key and roof) else None
    if tr:
        roof["traffic"] = tr["hbm_bytes_per_launch"]
        roof["traffic_launches"] = tr.get("launches")
        roof["traffic_over_algorithmic"] = tr.get("traffic_over_algorithmic")
    # the iterations alone: the timed solve's wall time less the weights and start (their
    # event times from the profiled solves).  Bytes of an iteration = the sweep's (coded
    # Sigma', X, C, mu) + 16 dense FP32 touches of the other stages (X, BX, C, Lambda1,
    # Lambda2, W1, W2, FFT in/out) per pixel and band; also against the bytes the dual state
    # would move stored densely (8 N_pairs |P| + 64 B per pixel, band and iteration)
    loop = None
    if prof_steps:
        setup_ms = sum(stages[k]["ms_total"] for k in ("weights", "init") if k in stages)
        setup_ms /= prof_steps
        events_ms = sum(v["ms_total"] for k, v in stages.items()
                        if k not in ("weights", "init")) / prof_steps
        loop_ms = elapsed / steps * 1e3 - setup_ms          # per solve
        pbi = spec.p * spec.q * lx * spec.iters
        loop_bytes_pbi = 8 * npairs * (2 * spec.K + 1) ** 2 + 64
        dense_gbs = loop_bytes_pbi * pbi / (loop_ms * 1e-3) / 1e9
        loop = {"t_loop_ms_per_solve": round(loop_ms, 3),
                "t_total_ms_per_solve": round(elapsed / steps * 1e3, 3),
                "t_setup_ms_per_solve": round(setup_ms, 3),
                "t_stage_events_ms_per_solve": round(events_ms, 3),
                "step_ms_median": round(sorted(step_s)[len(step_s) // 2] * 1e3, 3),
                "dense_format_bytes_per_pbi": loop_bytes_pbi,
                "dense_format_equivalent_GBs": round(dense_gbs, 1),
                "dense_format_hbm_frac": round(dense_gbs / HBM_PEAK_GBS, 4)}
        if sweep_bytes:
            coded = sum(sweep_bytes) + 64 * pbi
            gbs = coded / (loop_ms * 1e-3) / 1e9
            loop.update({"bytes_per_solve": coded, "achieved_GBs": round(gbs, 1),
                         "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
    res = {"value": value, "ms_per_step": elapsed / steps * 1e3, "roofline": roof,
           "loop_pbi_per_s": spec.p * spec.q * spec.L * spec.iters / (loop["t_loop_ms_per_solve"]
                                                                     * 1e-3) if loop else None,
           "loop": loop, "stages": stages, "finite": finite,
           "sweep_shape_stream_GBs": shape_gbs}
    if monitor:
        res["monitor"] = mon
    del ws, Z, Yl, Yh
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()

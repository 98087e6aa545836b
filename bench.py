"""Benchmark of the fused MLP + DROP reconstruction path on one MI355X.

Workload (default): the head-sized single-GPU share of a full scan, a
256x256x64 grid of 1 mm voxels, ellipsoidal phantom with 10 spherical
inserts, 5*10^7 protons over 360 projection angles sorted by angle, 4 mm slab
of v_in and t_in, DROP block 6400, lambda 0.1, FP32 RSP volume, 8 sweeps (one
reconstruction).  One step is one DROP sweep over all protons: for every
block, each proton's most likely path is traced, a_i.x and ||a_i||^2
computed, and the D-weighted back-projection committed.  Inputs are resident
in HBM before the timed region starts.  --config 2 runs the 10^7-proton
200x200x32 cylinder scan (block 3200, 12 sweeps) instead.

Prints one JSON line:  value = proton-iterations/s, a roofline object for the
dominant kernel (the block kernel) and the CPU oracle baseline measured on a
bounded sample of the same scan.

    python bench.py [--gpus 1] [--steps 8] [--warmup 1] [--no-cpu-baseline]

Two more workloads, each printing its own JSON line:
    --config 4   precision form: 2*10^7 protons on the 200x200x32 scan, 8
                 sweeps with FP32, FP16 and BF16 chords; RSP error of each
                 against an FP64 run (FP64 value type and chords) and speed
                 relative to the FP32-chord run.
    --config 5   differentiation form: 2*10^7 protons on the 256x256x64 scan,
                 20 steps of TV-regularised gradient descent (forward +
                 backward projection per step); loss curve and pass rates.
    --config bsweep  block-size variants on the 10^7-proton 200x200x32 scan
                 (B = 3200, 32000, 320000): time per sweep and insert RSP
                 error after each of 4 sweeps.
    --config alg1  the multi-region split (Algorithm 1) of the 10^7-proton
                 200x200x32 scan into two overlapping z regions, run one after
                 the other on this GPU, against the single-volume solve: insert
                 RSP error after every sweep, per-region time.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BYTES_PER_PROTON = 40.0        # proton record: 9 float32 fields + b_i
BYTES_PER_NONZERO = 8.0        # x_j gather (4 B) + back-projected contribution (4 B)
RSP_FLOOR = 0.05               # RSP errors are relative to max(|x_oracle|, RSP_FLOOR)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources each profiled kernel is built from: its counters stay valid while
# these files are unchanged.
KERNEL_SOURCES = {
    "k_drop": ("pct_internal.h", "pct_path.hpp", "pct_kernels.hip"),
    "fbp": ("pct_internal.h", "pct_fbp.hip"),
}


def kernel_sources_digest(kernel: str = "k_drop") -> str:
    """sha256 over the HIP sources a profiled kernel is built from (the
    traffic counters are valid only for the kernels they were taken on)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1802_01070_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update(name.encode())
        h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of the block kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload and kernel, or None when
    the kernel sources changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None, f"no counter summary for {kernel} on {workload}"
    t = json.load(open(p))
    if t.get("workload") != workload:
        return None, "counters taken on another workload"
    if t.get("sources_sha256") != kernel_sources_digest():
        return None, "kernel sources changed since the counters were taken"
    return float(t["hbm_bytes_per_launch"]), os.path.relpath(p, ROOT)


def measured_fbp_traffic(workload: str, kernels):
    """HBM bytes per launch of FBP kernels (one name, or the kernels of a step
    summed) from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or
    None when the sources changed since."""
    p = os.path.join(ROOT, "profiles", "traffic_fbp_cyl200.json")
    if not os.path.exists(p):
        return None, "no counter summary"
    t = json.load(open(p))
    if t.get("workload") != workload:
        return None, "counters taken on another workload"
    if t.get("sources_sha256") != kernel_sources_digest("fbp"):
        return None, "kernel sources changed since the counters were taken"
    total = 0.0
    for kernel in ([kernels] if isinstance(kernels, str) else kernels):
        k = t.get("kernels", {}).get(kernel)
        if k is None:
            return None, f"no counters for {kernel}"
        total += float(k["hbm_bytes_per_launch"])
    return total, os.path.relpath(p, ROOT)


def count_nonzeros(api, plan, pr, chunk=1 << 20):
    """Sum over protons of the path's merged (voxel, chord) pieces, from the
    trace kernel (max_nnz = 1: only the lengths are kept)."""
    import torch
    total = 0
    for lo in range(0, pr.n, chunk):
        cnt = min(chunk, pr.n - lo)
        _, _, nnz = api.pct_mlp_trace(plan, pr, lo, cnt, max_nnz=1)
        total += int(nnz.to(torch.int64).sum())
    api.pct_device_status(plan, reset=True)   # rows longer than 1 raise the overflow bit: expected here
    return total


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(sc, cfg, x_gpu_sample, n_blocks, hull=0.0, mode="none"):
    """FP64 oracle on the first n_blocks blocks of one sweep (from x0 = 1):
    throughput on the host cores and the RSP error of the GPU result on the
    same sample."""
    import oracle
    oracle.build(force=False)
    oracle.set_hull(hull or None)
    m = min(sc.m, n_blocks * cfg.block)
    sub = sc.subset(0, m)
    t0 = time.perf_counter()
    ref = oracle.drop(sc.grid, sc.mlp, sub.protons, sub.b, 1.0, block=cfg.block, lam=cfg.lam, n_iter=1, mode=mode)
    dt = time.perf_counter() - t0
    err = np.abs(x_gpu_sample - ref) / np.maximum(np.abs(ref), RSP_FLOOR)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": m / dt, "unit": "proton-iterations/s", "cores": threads, "kind": "oracle",
        "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
        "sample": f"first {n_blocks} blocks ({m} protons) of one sweep of the same scan, FP64 C oracle, "
                  f"{dt:.1f} s" + ("" if mode == "none" else f", chords rounded to {mode}"),
    }, float(err.max()), float(err.mean())


def sweep_roofline(ms_per_sweep, T, m, sum_nnz, kernel):
    """Roofline entry of the block kernel from the time of whole sweeps: the
    sweep's stream carries the T block launches and two small kernels."""
    k_ms = ms_per_sweep / T
    nbytes = (BYTES_PER_PROTON * m + BYTES_PER_NONZERO * sum_nnz) / T
    gbs = nbytes / (k_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": None, "traffic_source": "counters taken on the FP32 head-scan headline run only",
            "kernel": kernel, "kernel_avg_us": k_ms * 1e3,
            "kernel_avg_us_how": "sweeps timed with HIP events on the sweep's stream / block launches",
            "algorithmic_bytes_per_launch": nbytes}


def time_events(fn, reps=1):
    """Mean ms of fn() on the current stream, bracketed by HIP events."""
    import torch
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    z.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(z) / reps


def parallel_sweep_ceiling(api, plan, pr, x):
    """One forward projection (with ||a_i||^2) and one back projection over all
    protons with no block sequencing: the rate the same walk reaches when every
    proton is independent."""
    import torch
    r = torch.ones(pr.n, dtype=x.dtype, device=x.device)
    g = torch.zeros_like(x)
    api.pct_forward(plan, pr, x, with_norm=True)
    api.pct_backproject(plan, pr, r, g)
    f_ms = time_events(lambda: api.pct_forward(plan, pr, x, with_norm=True), reps=2)
    b_ms = time_events(lambda: api.pct_backproject(plan, pr, r, g), reps=2)
    log(f"[bench] parallel sweep: forward {f_ms:.1f} ms, back projection {b_ms:.1f} ms")
    return {"forward_ms": f_ms, "backproject_ms": b_ms,
            "protons_per_s_forward_plus_back": pr.n / ((f_ms + b_ms) * 1e-3)}


def rsp_error(x, ref, touched):
    import torch
    d = (x.double() - ref.double()).abs() / ref.double().abs().clamp_min(RSP_FLOOR)
    d = d[touched]
    return float(d.max()), float(d.mean())


def run_precision(args):
    """Precision form on the 2*10^7-proton 200x200x32 scan."""
    import torch
    from paper_1802_01070_amd import api, synth
    cfg = synth.WORKLOADS[4]
    m = args.protons or cfg.m
    log(f"[bench] generating {cfg.name}: {m} protons")
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    pr = api.Protons(sc.protons, dev)
    b = torch.from_numpy(sc.b).to(dev)
    pr, b = api.pct_order_blocks(plan, pr, b, cfg.block)       # as the headline run does
    n_iter = cfg.n_iter
    runs = {}
    for name, dtype, chord in (("f64", torch.float64, "f64"), ("f32", torch.float32, "f32"),
                               ("f16", torch.float32, "f16"), ("bf16", torch.float32, "bf16")):
        x = torch.ones(sc.grid.nvox, dtype=dtype, device=dev)
        api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, chord=chord)  # warm-up
        x.fill_(1.0)
        ms = time_events(lambda: api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam,
                                                      n_iter=n_iter, chord=chord))
        bits = api.pct_device_status(plan)
        log(f"[bench] {name} chords: {ms:.0f} ms for {n_iter} sweeps (status {bits:#x})")
        runs[name] = (x, ms, bits)
    # stored rows: traced once (timed), then the same sweeps read from HBM
    stored = {}
    for name in ("f32", "f16", "bf16"):
        box = {}
        build_ms = time_events(lambda: box.setdefault("rows", api.Rows(plan, pr, name)))
        rows = box["rows"]
        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
        api.pct_drop_iterate_rows(plan, rows, b, x, block=cfg.block, lam=cfg.lam, n_iter=1)   # warm-up
        x.fill_(1.0)
        ms = time_events(lambda: api.pct_drop_iterate_rows(plan, rows, b, x, block=cfg.block, lam=cfg.lam,
                                                           n_iter=n_iter))
        bits = api.pct_device_status(plan)
        log(f"[bench] stored {name} rows: build {build_ms:.0f} ms, {ms:.0f} ms for {n_iter} sweeps, "
            f"{rows.nbytes / 2**30:.1f} GiB (status {bits:#x})")
        stored[name] = (x, ms, build_ms, rows.nbytes, bits)
        del rows, box
        torch.cuda.empty_cache()
    ref = runs["f64"][0]
    # voxels crossed by at least one row: A^T 1 > 0
    cover = api.pct_backproject(plan, pr, torch.ones(pr.n, dtype=torch.float32, device=dev))
    touched = cover > 0
    table = {}
    for name in ("f32", "f16", "bf16"):
        x, ms, bits = runs[name]
        emax, emean = rsp_error(x, ref, touched)
        table[name] = {"ms_per_reconstruction": ms, "rsp_err_max": emax, "rsp_err_mean": emean,
                       "speedup_vs_f32_chords": runs["f32"][1] / ms, "status": bits}
    for name in ("f32", "f16", "bf16"):
        x, ms, build_ms, nbytes, bits = stored[name]
        emax, emean = rsp_error(x, ref, touched)
        table["stored_" + name] = {"ms_per_reconstruction": ms, "build_ms": build_ms, "row_bytes": nbytes,
                                   "rsp_err_max": emax, "rsp_err_mean": emean,
                                   "speedup_vs_f32_chords": runs["f32"][1] / ms,
                                   "speedup_incl_build_vs_f32_chords": runs["f32"][1] / (ms + build_ms),
                                   "status": bits}
    f16_ms = runs["f16"][1]
    sum_nnz = count_nonzeros(api, plan, pr)
    T = (m + cfg.block - 1) // cfg.block
    roof = sweep_roofline(f16_ms / n_iter, T, m, sum_nnz,
                          "block step of the binned schedule with FP16 chords (k_drop_bin + k_slab_commit; "
                          "chords rounded as traced)")
    roof["nonzeros_per_proton"] = sum_nnz / m
    cpu = None
    cpu_err = None
    if not args.no_cpu_baseline:
        nb = min(args.cpu_blocks, T)
        xs = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
        api.pct_drop_iterate(plan, pr, b, xs, block=cfg.block, lam=cfg.lam, n_iter=1, block_end=nb, chord="f16")
        torch.cuda.synchronize()
        log(f"[bench] CPU oracle baseline on {nb} blocks (FP16 chords) ...")
        cpu, emax, emean = cpu_baseline(sc, cfg, xs.double().cpu().numpy(), nb, mode="f16")
        cpu_err = {"sample": f"first {nb} blocks of one sweep, FP16 chords on both sides", "max": emax,
                   "mean": emean}
    out = {
        "metric": "proton-iterations/sec (fused MLP+DROP, FP16 chords) at 1 GPU",
        "value": m * n_iter / (f16_ms * 1e-3),
        "unit": "proton-iterations/s",
        "n_gpus": 1, "steps": n_iter, "warmup": 1, "ms_per_step": f16_ms / n_iter,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f16 chords)",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} grid, {m} protons, "
                               f"{cfg.n_angles} angles, DROP block {cfg.block}, lambda {cfg.lam}, {n_iter} sweeps; "
                               "chords rounded to FP16/BF16 as computed, FP32 iterate and accumulation, FP64 "
                               "a_i.x and ||a_i||^2",
                   "reference": "same scan, FP64 iterate and FP64 chords on the GPU",
                   "touched_voxels": int(touched.sum())},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rsp_err_vs_fp64_oracle": cpu_err,
        "precision": table,
    }
    print(json.dumps(out), flush=True)


def run_gradient(args):
    """Differentiation form on the 2*10^7-proton 256x256x64 scan."""
    import torch
    from paper_1802_01070_amd import api, synth
    cfg = synth.WORKLOADS[5]
    m = args.protons or cfg.m
    log(f"[bench] generating {cfg.name}: {m} protons")
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    pr = api.Protons(sc.protons, dev)
    b = torch.from_numpy(sc.b).to(dev)
    beta, eps, n_steps = 1e-3, 1e-3, cfg.n_iter
    x0 = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
    r = torch.ones(pr.n, dtype=torch.float32, device=dev)
    g = torch.zeros_like(x0)
    api.pct_forward(plan, pr, x0)
    api.pct_backproject(plan, pr, r, g)
    f_ms = time_events(lambda: api.pct_forward(plan, pr, x0), reps=3)
    b_ms = time_events(lambda: api.pct_backproject(plan, pr, r, g), reps=3)
    v0 = torch.from_numpy(synth.power_start(sc.grid.nvox, cfg.seed)).to(dev, torch.float32)
    t0 = time.perf_counter()
    lam_max = api.power_iteration(plan, pr, v0, 20)
    t_power = time.perf_counter() - t0
    eta = 1.0 / (lam_max + 12.0 * beta / eps)
    box = {}

    def gd():
        box["res"] = api.tv_gradient_descent(plan, pr, b, x0, beta, eps, n_steps, eta=eta)

    gd_ms = time_events(gd)
    x, losses, _ = box["res"]
    bits = api.pct_device_status(plan)
    log(f"[bench] forward {f_ms:.1f} ms, back projection {b_ms:.1f} ms, GD {gd_ms:.0f} ms; "
        f"loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    sum_nnz = count_nonzeros(api, plan, pr)
    # dominant kernel: k_backproject (one lane per proton: 9 record fields and
    # r_i in, 40 B; pieces pre-summed per workgroup in LDS, one FP32 atomic per distinct voxel)
    bp_bytes = BYTES_PER_PROTON * m + 4.0 * sum_nnz
    bp_gbs = bp_bytes / (b_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": bp_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": bp_gbs / HBM_PEAK_GBS,
            "traffic": None, "traffic_source": "no counter run on this workload",
            "kernel": "k_backproject (A^T r: MLP trace per proton, pieces pre-summed per workgroup in LDS, one FP32 atomic per distinct voxel)",
            "kernel_avg_us": b_ms * 1e3, "kernel_avg_us_how": "HIP events on the stream, mean of 3 launches",
            "algorithmic_bytes_per_launch": bp_bytes, "nonzeros_per_proton": sum_nnz / m,
            "forward_kernel_avg_us": f_ms * 1e3,
            "forward_GBps": (BYTES_PER_PROTON * m + 4.0 * sum_nnz) / (f_ms * 1e-3) / 1e9}
    cpu = None
    cpu_err = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        ms_ = min(m, 400_000)
        sub = sc.subset(0, ms_)
        xt = np.ones(sc.grid.nvox)
        rt = np.ones(ms_)
        log(f"[bench] CPU oracle baseline: forward + back projection of {ms_} protons ...")
        t1 = time.perf_counter()
        y_ref = oracle.forward(sc.grid, sc.mlp, sub.protons, xt)
        oracle.backproject(sc.grid, sc.mlp, sub.protons, rt)
        dt = time.perf_counter() - t1
        y_gpu = api.pct_forward(plan, api.Protons(sub.protons, dev), x0)
        y_gpu = (y_gpu[0] if isinstance(y_gpu, tuple) else y_gpu).double().cpu().numpy()
        yr = np.asarray(y_ref[0] if isinstance(y_ref, tuple) else y_ref, dtype=np.float64)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": ms_ / dt, "unit": "proton-iterations/s", "cores": threads, "kind": "oracle",
               "sample": f"forward A.x and back projection A^T r of the first {ms_} protons, FP64 C oracle, "
                         f"{dt:.1f} s (one gradient step per proton)"}
        rel = np.abs(y_gpu - yr) / np.maximum(np.abs(yr), 1.0)
        cpu_err = {"sample": f"A.1 of the first {ms_} protons", "max": float(rel.max()), "mean": float(rel.mean())}
    out = {
        "metric": "proton-iterations/sec (TV-regularised gradient descent, forward+backward) at 1 GPU",
        "value": m * n_steps / (gd_ms * 1e-3),
        "unit": "proton-iterations/s",
        "n_gpus": 1, "steps": n_steps, "warmup": 1, "ms_per_step": gd_ms / n_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} grid, {m} protons, "
                               f"{cfg.n_angles} angles, sorted by (angle, slab, t_in); {n_steps} gradient steps on "
                               f"1/2||Ax-b||^2 + {beta} TV_eps (eps {eps}), step 1/(lambda_max + 12 beta/eps)",
                   "beta": beta, "eps": eps},
        "forward_protons_per_s": m / (f_ms * 1e-3),
        "backward_protons_per_s": m / (b_ms * 1e-3),
        "power_iteration": {"lambda_max": lam_max, "steps": 20, "seconds": t_power},
        "eta": eta,
        "loss_curve": losses,
        "status": bits,
        "roofline": roof,
        "cpu_baseline": cpu,
        "forward_err_vs_fp64_oracle": cpu_err,
    }
    print(json.dumps(out), flush=True)


def insert_errors(sc, x):
    """Per insert: mean RSP over voxels whose centre lies at least 1.5 mm
    inside it, and its relative error (%) against the insert's true RSP."""
    import torch
    g = sc.grid
    xs = g.origin[0] + (np.arange(g.nx) + 0.5) * g.pitch[0]
    ys = g.origin[1] + (np.arange(g.ny) + 0.5) * g.pitch[1]
    X, Y = np.meshgrid(xs, ys)
    xv = x.double().cpu().numpy().reshape(g.nz, g.ny, g.nx)
    out = []
    for s in sc.phantom.inserts:
        r = np.hypot(X - s.centre[0], Y - s.centre[1])
        mask = r < s.axes[0] - 1.5
        mean = float(xv[:, mask].mean())
        out.append({"true": s.rsp, "mean": mean, "err_pct": 100.0 * (mean - s.rsp) / s.rsp})
    return out


def run_block_sizes(args):
    """Block-size variants of the plain method on the 10^7-proton scan."""
    import torch
    from paper_1802_01070_amd import api, synth
    cfg = synth.WORKLOADS[2]
    m = args.protons or cfg.m
    log(f"[bench] generating {cfg.name}: {m} protons")
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    pr0 = api.Protons(sc.protons, dev)
    b0 = torch.from_numpy(sc.b).to(dev)
    n_sweeps = 4
    variants = []
    for B in (3200, 32000, 320000):
        pr, b = api.pct_order_blocks(plan, pr0, b0, min(B, 8192)) if B <= 8192 else (pr0, b0)
        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
        api.pct_drop_iterate(plan, pr, b, x, block=B, lam=cfg.lam, n_iter=1)       # warm-up (records the graph)
        x.fill_(1.0)
        sweeps = []
        for k in range(n_sweeps):
            ms = time_events(lambda: api.pct_drop_iterate(plan, pr, b, x, block=B, lam=cfg.lam, n_iter=1))
            sweeps.append({"sweep": k + 1, "ms": ms, "inserts": insert_errors(sc, x)})
        bits = api.pct_device_status(plan)
        log(f"[bench] B={B}: {[round(s['ms'], 1) for s in sweeps]} ms per sweep, status {bits:#x}")
        variants.append({"block": B, "blocks_per_sweep": (m + B - 1) // B, "sweeps": sweeps, "status": bits})
    best = min(variants, key=lambda v: np.mean([s["ms"] for s in v["sweeps"]]))
    ms = float(np.mean([s["ms"] for s in best["sweeps"]]))
    out = {
        "metric": "proton-iterations/sec (fused MLP+DROP, block-size variants) at 1 GPU",
        "value": m / (ms * 1e-3), "unit": "proton-iterations/s", "n_gpus": 1, "steps": n_sweeps, "warmup": 1,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} grid, {m} protons, "
                               f"lambda {cfg.lam}, DROP block 3200 / 32000 / 320000 (value: the fastest, "
                               f"B={best['block']})"},
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


def run_regions(args):
    """Algorithm 1 on the 10^7-proton 200x200x32 scan against the single-volume
    solve, sweep by sweep."""
    import torch
    from paper_1802_01070_amd import api, synth
    cfg = synth.WORKLOADS[2]
    m = args.protons or cfg.m
    n_sweeps = args.steps if args.steps != 12 else 6
    log(f"[bench] generating {cfg.name}: {m} protons")
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    pr = api.Protons(sc.protons, dev)
    b = torch.from_numpy(sc.b).to(dev)
    hist = api.pct_slice_span_histogram(plan, pr)
    halo = api.overlap_halo(hist, 0.96)
    cov = (torch.cumsum(hist.double(), 0) / hist.sum()).cpu().numpy()
    n_regions = 2
    # single volume
    x1 = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
    api.pct_drop_iterate(plan, pr, b, x1, block=cfg.block, lam=cfg.lam, n_iter=1)   # warm-up
    x1.fill_(1.0)
    single = []
    for k in range(n_sweeps):
        ms = time_events(lambda: api.pct_drop_iterate(plan, pr, b, x1, block=cfg.block, lam=cfg.lam, n_iter=1))
        single.append({"sweep": k + 1, "ms": ms, "inserts": insert_errors(sc, x1)})
        log(f"[bench] single volume sweep {k + 1}: {ms:.0f} ms")
    # two regions, one after the other on this GPU
    x2 = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    state = None
    lay = api.pct_region_layout(sc.grid.nz, n_regions, halo)
    split = []
    for k in range(n_sweeps):
        torch.cuda.synchronize()
        if state is None:
            state = api.region_drop(plan, pr, b, x2, n_regions, halo, cfg.block, cfg.lam, 0)
            for reg in state:     # warm-up sweep (records the graph), then back to x0 = 1
                api.pct_drop_iterate(reg["plan"], reg["protons"], reg["b"], reg["x"], cfg.block, cfg.lam, 1)
                reg["x"].fill_(1.0)
        per_region = []
        for reg in state:
            per_region.append(time_events(lambda: api.pct_drop_iterate(reg["plan"], reg["protons"], reg["b"],
                                                                          reg["x"], cfg.block, cfg.lam, 1)))
        api.region_drop(plan, pr, b, x2, n_regions, halo, cfg.block, cfg.lam, 0, regions=state)
        split.append({"sweep": k + 1, "ms_per_region": per_region, "inserts": insert_errors(sc, x2)})
        log(f"[bench] two regions sweep {k + 1}: {per_region} ms")
    torch.cuda.synchronize()
    diff = (x1.double() - x2.double()).abs()
    out = {
        "metric": "proton-iterations/sec (Algorithm 1, two z regions, max over regions) at 1 GPU",
        "value": m * n_sweeps / (max(sum(r["ms_per_region"][i] for r in split) for i in range(n_regions)) * 1e-3),
        "unit": "proton-iterations/s",
        "n_gpus": 1, "steps": n_sweeps, "warmup": 1,
        "ms_per_step": float(np.mean([max(r["ms_per_region"]) for r in split])),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} grid, {m} protons, "
                               f"{cfg.n_angles} angles, DROP block {cfg.block}, lambda {cfg.lam}; {n_regions} z "
                               f"regions with {halo} slices of halo (96% coverage), regions run one after the "
                               "other; value = the rate a region-per-GPU run would reach (slowest region)",
                   "layout": lay, "region_protons": [reg["protons"].n for reg in state]},
        "coverage_by_span": [float(c) for c in cov[:12]],
        "single_volume": single,
        "regions": split,
        "max_abs_diff_split_vs_single": float(diff.max()),
    }
    print(json.dumps(out), flush=True)


FBP_FLOPS_PER_VOXEL_ANGLE = 12.0   # t (2 mul, 1 add), s (1 sub, 1 mul, 1 sub), w (1 sub), value (1 sub, 2 mul, 1 add), sum (1 add)
FBP_BIN_BYTES_PER_PROTON = 36.0    # t_in, t_out, v_in, v_out, gantry, b (24 B) + bin sum and count update (12 B)


def run_fbp(args):
    """FBP initial iterate (Section I) on the 10^7-proton scan: time of the
    image (binning, ramp filter, back-projection), its kernels, and DROP
    sweeps started from it against x0 = 1."""
    import torch
    from paper_1802_01070_amd import api, synth
    cfg = synth.WORKLOADS[2]
    m = args.protons or cfg.m
    log(f"[bench] generating {cfg.name}: {m} protons")
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    pr = api.Protons(sc.protons, dev)
    b = torch.from_numpy(sc.b).to(dev)
    geom = api.FbpGeom.for_grid(sc.grid, cfg.n_angles)
    ws = api.FbpWorkspace(plan, geom)
    x = torch.empty(sc.grid.nvox, dtype=torch.float32, device=dev)
    for _ in range(max(1, args.warmup)):
        api.pct_fbp(plan, pr, b, geom, x=x, ws=ws)
    steps = args.steps
    ms = time_events(lambda: api.pct_fbp(plan, pr, b, geom, x=x, ws=ws), reps=steps) / 1.0
    # the three steps on their own (HIP events on the stream they run on)
    box = {}
    # 20 repetitions each: the device work (0.1-0.3 ms per call) outlasts the host's enqueue
    t_sino = time_events(lambda: box.__setitem__("s", api.pct_fbp_sinogram(plan, pr, b, geom, ws=ws)), reps=20)
    t_filt = time_events(lambda: box.__setitem__("q", api.pct_fbp_filter(plan, box["s"][0], geom)), reps=20)
    t_bp = time_events(lambda: box.__setitem__("x", api.pct_fbp_backproject(plan, box["q"], geom)), reps=20)
    nb = sc.grid.nz * geom.n_angles * geom.n_t
    log(f"[bench] FBP image {ms:.3f} ms (sinogram {t_sino:.3f}, filter {t_filt:.3f}, back-projection {t_bp:.3f})")
    bp_flops = float(sc.grid.nvox) * geom.n_angles * FBP_FLOPS_PER_VOXEL_ANGLE
    bin_bytes = FBP_BIN_BYTES_PER_PROTON * m
    stages = {"sinogram_ms": t_sino, "filter_ms": t_filt, "backproject_ms": t_bp}
    if t_bp >= t_sino:
        roof = {"bound": "alu", "achieved": bp_flops / (t_bp * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                "kernel": "k_fbp_backproject_tiled (FP64 vector ALU)", "kernel_avg_us": 1e3 * t_bp,
                "algorithmic_flops_per_launch": bp_flops}
    else:
        roof = {"bound": "hbm", "achieved": bin_bytes / (t_sino * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                "kernel": "k_fbp_clear + k_fbp_bin_lds + k_fbp_mean (the binning step)", "kernel_avg_us": 1e3 * t_sino,
                "algorithmic_bytes_per_launch": bin_bytes}
    roof["frac"] = roof["achieved"] / roof["peak"]
    kname = "k_fbp_backproject_tiled" if roof["bound"] == "alu" else ["k_fbp_clear", "k_fbp_bin_lds", "k_fbp_mean"]
    traffic, source = measured_fbp_traffic(cfg.name, kname)
    roof["traffic"] = traffic
    roof["traffic_source"] = source
    # DROP from x0 = 1 and from the FBP image
    n_sweeps = 0 if args.no_drop_compare else 6
    runs = {}
    for name in (("x0_one", "x0_fbp") if n_sweeps else ()):
        xs = torch.ones(sc.grid.nvox, dtype=torch.float32, device=dev)
        api.pct_drop_iterate(plan, pr, b, xs, block=cfg.block, lam=cfg.lam, n_iter=1)      # warm-up (graph)
        if name == "x0_one":
            xs.fill_(1.0)
        else:
            api.pct_fbp(plan, pr, b, geom, x=xs, ws=ws)
        sweeps = [{"sweep": 0, "inserts": insert_errors(sc, xs)}]
        for k in range(n_sweeps):
            t = time_events(lambda: api.pct_drop_iterate(plan, pr, b, xs, block=cfg.block, lam=cfg.lam, n_iter=1))
            sweeps.append({"sweep": k + 1, "ms": t, "inserts": insert_errors(sc, xs)})
        runs[name] = sweeps
        worst = [max(abs(i["err_pct"]) for i in s["inserts"]) for s in sweeps]
        log(f"[bench] DROP from {name}: worst insert error per sweep {[round(w, 2) for w in worst]} %")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import fbp as ofbp
        log("[bench] CPU oracle FBP ...")
        t0 = time.perf_counter()
        rp, _ = ofbp.sinogram(sc.grid, sc.mlp, sc.protons, sc.b, geom.n_angles, geom.n_t, geom.t0, geom.dt)
        rx = ofbp.backproject(sc.grid, ofbp.filter_rows(rp, geom.dt), geom.n_angles, geom.t0, geom.dt)
        t_cpu = time.perf_counter() - t0
        err = float(np.abs(x.double().cpu().numpy() - rx).max() / max(1.0, np.abs(rx).max()))
        cpu = {"value": m / t_cpu, "unit": "protons/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole FBP image of the same scan (numpy FP64, one thread), {t_cpu:.1f} s",
               "max_rel_err_gpu_vs_oracle": err}
    out = {
        "metric": "protons/s into the FBP initial image (binning, ramp filter, back-projection) at 1 GPU",
        "value": m / (ms * 1e-3), "unit": "protons/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} grid, {m} protons, "
                               f"FBP with {geom.n_angles} angle bins x {geom.n_t} lateral bins of {geom.dt} mm x "
                               f"{sc.grid.nz} slices ({nb} bins), FP32 image",
                   "geom": {"n_angles": geom.n_angles, "n_t": geom.n_t, "t0": geom.t0, "dt": geom.dt}},
        "stages": stages,
        "roofline": roof,
        "cpu_baseline": cpu,
        "drop_from_x0": runs,
    }
    calibration_copy(args, dev)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="3")
    ap.add_argument("--protons", type=int, default=0, help="override the number of protons")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-order", action="store_true", help="keep the acquisition order inside blocks")
    ap.add_argument("--hull", type=float, default=0.0,
                    help="radius (mm) of a z-cylinder object hull: per-proton paths between the hull crossings")
    ap.add_argument("--cpu-blocks", type=int, default=320)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per proton in the block kernel (0: automatic)")
    ap.add_argument("--no-drop-compare", action="store_true",
                    help="--config fbp: skip the DROP sweeps from x0 = 1 and from the FBP image")
    ap.add_argument("--fused-commit", action="store_true",
                    help="FP32: the atomic schedules (commit of block t-1 inside the launch of block t)")
    ap.add_argument("--no-compensation", action="store_true",
                    help="binned schedule: round x at every commit instead of carrying its rounding error")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the block kernels one by one on the stream instead of replaying a HIP graph")
    ap.add_argument("--separate-commit", action="store_true",
                    help="FP32: the separate schedule (block kernel, then a commit kernel per block)")
    ap.add_argument("--host-sort", action="store_true",
                    help="continuous-rotation scans: take the generator's angle-bin order instead of the device sort")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU region split is "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1802_01070_amd import api, synth
    from paper_1802_01070_amd._lib import (PCT_DROP_FUSED_COMMIT, PCT_DROP_NO_COMPENSATION, PCT_DROP_NO_GRAPH,
                                           PCT_DROP_PROFILE, PCT_DROP_SEPARATE_COMMIT)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.config == "4":
        return run_precision(args)
    if args.config == "5":
        return run_gradient(args)
    if args.config == "alg1":
        return run_regions(args)
    if args.config == "bsweep":
        return run_block_sizes(args)
    if args.config == "fbp":
        return run_fbp(args)
    key = int(args.config) if args.config.isdigit() else args.config
    cfg = synth.WORKLOADS[key]
    m = args.protons or cfg.m
    # a continuous-rotation scan arrives in acquisition order and is sorted
    # into angle bins on the device (pct_sort_scan); --host-sort takes the
    # generator's sorted copy instead
    device_sort = cfg.continuous_angles and cfg.order == "angle_slab" and not args.host_sort
    log(f"[bench] generating {cfg.name}: {m} protons")
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg.with_(order="acquisition") if device_sort else cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    if args.hull > 0:
        plan.set_hull(args.hull)
    pr = api.Protons(sc.protons, dev)
    b = torch.from_numpy(sc.b).to(dev)
    vdtype = torch.float64 if cfg.value_type == "f64" else torch.float32
    x = torch.ones(sc.grid.nvox, dtype=vdtype, device=dev)
    torch.cuda.synchronize()

    sort_ms = None
    if device_sort:
        api.pct_sort_scan(plan, pr, b, cfg.n_angles, cfg.slab_mm)        # first call: allocator warm-up
        box = {}
        sort_ms = time_events(lambda: box.setdefault("s", api.pct_sort_scan(plan, pr, b, cfg.n_angles, cfg.slab_mm)))
        pr, b, _ = box["s"]
        # the CPU-baseline sample reads the records the device sorted
        sc = dataclasses.replace(sc, protons={k: pr.t[k].cpu().numpy() for k in synth.FIELDS}, b=b.cpu().numpy())
        log(f"[bench] sorted {m} acquisition-order records into {cfg.n_angles} angle bins on the device in "
            f"{sort_ms:.2f} ms")

    sum_nnz = count_nonzeros(api, plan, pr)
    order_ms = None
    if not args.no_order:
        # within-block ordering (one-time): each block's rows sorted by entry
        # slice and lateral position, so each XCD walks neighbouring paths
        box = {}
        order_ms = time_events(lambda: box.setdefault("o", api.pct_order_blocks(plan, pr, b, cfg.block)))
        pr, b = box["o"]
        log(f"[bench] ordered blocks in {order_ms:.1f} ms")
    T = (m + cfg.block - 1) // cfg.block
    sched = ((PCT_DROP_SEPARATE_COMMIT if args.separate_commit else 0) |
             (PCT_DROP_FUSED_COMMIT if args.fused_commit else 0) |
             (PCT_DROP_NO_COMPENSATION if args.no_compensation else 0) |
             (PCT_DROP_NO_GRAPH if args.no_graph else 0))
    log(f"[bench] sum of nonzeros {sum_nnz} ({sum_nnz / m:.1f} per proton), {T} blocks per sweep")

    # untimed warmup sweeps (the first run also compiles nothing: the library is prebuilt)
    for _ in range(args.warmup):
        api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, lanes=args.lanes, flags=sched)
    torch.cuda.synchronize()
    x.fill_(1.0)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # one event after every sweep as well: the median sweep is reported beside
    # the mean over the timed region
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    e0.record(stream)
    t_host = time.perf_counter()
    for k in range(args.steps):
        api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, lanes=args.lanes, flags=sched)
        marks[k].record(stream)
        log(f"[bench] step {k + 1}/{args.steps} enqueued")
    e1.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms_total = e0.elapsed_time(e1)
    step_ms = [e0.elapsed_time(marks[0])] + [marks[k - 1].elapsed_time(marks[k]) for k in range(1, args.steps)]
    # One more sweep, right after the timed region and on the same stream, with
    # a sample of the block-kernel and commit launches bracketed by HIP events
    # (recorded by the library) to time the dominant kernel itself.
    api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, lanes=args.lanes,
                         flags=PCT_DROP_PROFILE | sched)
    torch.cuda.synchronize()
    bits = api.pct_device_status(plan)
    if bits:
        log(f"[bench] WARNING device status {bits:#x}")
    ms_per_step = ms_total / args.steps
    value = m * args.steps / (ms_total / 1e3)
    (k_ms, c_ms), (k_n, c_n) = api.pct_profile_read(plan)
    k_sampled_ms = k_ms / max(k_n, 1)
    c_avg_ms = c_ms / max(c_n, 1)
    # Average launch of the block kernel over the timed region.  The sweep's
    # stream carries nothing else but one or two small kernels per sweep and,
    # on the binned and separate schedules, the per-block commit kernel, so a
    # block step of the timed region is ms_total / steps / T.  With a commit
    # kernel the step is split between the two by their event-timed sample:
    # the sampled sweep runs launch by launch (launches that record their own
    # events are not captured in a graph), and every such launch takes a few
    # microseconds longer than the same launch replayed in the graph, so each
    # sampled average gives up an equal share of the sample's excess over the
    # timed step.
    blk_ms = ms_total / args.steps / T
    if c_n and k_n:
        excess_ms = max(0.0, (k_sampled_ms + c_avg_ms - blk_ms) / 2)
        k_avg_ms = k_sampled_ms - excess_ms
        c_step_ms = c_avg_ms - excess_ms
    else:
        excess_ms = 0.0
        k_avg_ms = blk_ms
        c_step_ms = None
    bytes_per_launch = (BYTES_PER_PROTON * m + BYTES_PER_NONZERO * sum_nnz) / T
    achieved_gbs = bytes_per_launch / (k_avg_ms * 1e-3) / 1e9
    whole_gbs = (BYTES_PER_PROTON * m + BYTES_PER_NONZERO * sum_nnz) * args.steps / (ms_total * 1e-3) / 1e9
    log(f"[bench] {ms_per_step:.1f} ms/step, block kernel avg {k_avg_ms * 1e3:.2f} us over the timed region, "
        f"{k_sampled_ms * 1e3:.2f} us in {k_n} event-timed launches, "
        f"commit kernel avg {c_avg_ms * 1e3:.2f} us ({c_n} sampled); host wall {t_host:.2f} s")

    ceiling = parallel_sweep_ceiling(api, plan, pr, x)
    # which block schedule pct_drop_iterate takes (the library's rules): FP32
    # with lanes > 1 and blocks of at most 8192 protons: the binned schedule
    # (block kernel + slab commit); with --fused-commit, 64 lanes per proton
    # and blocks of at most 4096 protons the traced-ahead atomic schedule, else
    # the fused one; FP64 runs the block kernel and a separate commit
    lanes = args.lanes or (64 if max(sc.grid.nx, sc.grid.ny) >= 160 else 32 if max(sc.grid.nx, sc.grid.ny) >= 64
                           else 16)
    f32 = vdtype == torch.float32
    if f32 and lanes > 1 and cfg.block <= 8192 and not (args.separate_commit or args.fused_commit):
        kname, kdesc = "k_drop_bin", ("k_drop_bin (MLP trace + a.x + |a|^2 + rho of block t, packed D-weighted "
                                      "contributions stored into per-(slab, row) bins; the slab commit "
                                      "k_slab_commit sums them in LDS and commits the touched voxels)")
    elif f32 and lanes == 64 and cfg.block <= 4096 and not args.separate_commit:
        kname, kdesc = "k_drop_pipe", ("k_drop_pipe (trace of block t+1 into a row slot, DROP step of block t: "
                                       "a.x + |a|^2 + rho + D-weighted scatter, commit of block t-1)")
    elif f32 and not args.separate_commit:
        kname, kdesc = "k_drop_fused", ("k_drop_fused (MLP trace + a.x + |a|^2 + rho + D-weighted scatter of "
                                        "block t, commit of block t-1)")
    else:
        kname, kdesc = "k_drop_block", "k_drop_block (MLP trace + a.x + |a|^2 + rho + scatter) + k_drop_commit"
    traffic, traffic_src = (measured_traffic(cfg.name, kname) if not (args.protons or args.hull or args.separate_commit)
                            else (None, "counters taken on the default tracker-to-tracker run"))

    out = {
        "metric": "proton-iterations/sec (fused MLP+DROP) at 1 GPU",
        "value": value,
        "unit": "proton-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": float(np.median(step_ms)),
        "ms_per_step_min_max": [float(min(step_ms)), float(max(step_ms))],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if vdtype == torch.float32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} grid of 1 mm voxels, {m} protons, "
                        f"{cfg.n_angles} angles, DROP block {cfg.block}, lambda {cfg.lam}, one sweep per step "
                        f"({cfg.n_iter} sweeps = one reconstruction), MLP step 1 mm over {sc.mlp.depth:.0f} mm, "
                        f"FP64 geometry, {'FP32' if vdtype == torch.float32 else 'FP64'} RSP",
            "protons": m, "block": cfg.block, "lambda": cfg.lam, "grid": [sc.grid.nx, sc.grid.ny, sc.grid.nz],
            "nonzeros_per_proton": sum_nnz / m, "blocks_per_sweep": T,
            "order_inside_blocks": "acquisition" if order_ms is None else "entry slice, t_in (pct_order_blocks)",
            "hull_radius_mm": args.hull or None,
            "order_ms_once": order_ms,
            "angle_bins": ("device sort of the acquisition-order scan (pct_sort_scan: angle bin, 4 mm slab of "
                           "v_in, t_in)" if device_sort else "generator order"),
            "angle_sort_ms_once": sort_ms,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_source": traffic_src,
            "kernel": kdesc,
            "lanes_per_proton": args.lanes or "auto",
            "kernel_avg_us": k_avg_ms * 1e3,
            "kernel_avg_us_how": ("block step of the timed region (HIP events on the sweep's stream, graph "
                                  "replay) less the commit kernel's share; the shares are the event-timed "
                                  "sample averages less an equal part of their excess over the step"),
            "block_step_us": blk_ms * 1e3,
            "commit_kernel_avg_us": c_step_ms * 1e3 if c_step_ms is not None else None,
            "sample_excess_us_per_launch": excess_ms * 1e3,
            "kernel_avg_us_event_timed": k_sampled_ms * 1e3,
            "kernel_avg_us_event_timed_how": ("a sample of the launches timed by HIP events: recorded by the launch "
                                              "itself (hipExtLaunchKernelGGL) on the binned schedule, bracketing "
                                              "the launch on the others"),
            "kernel_launches_sampled": k_n,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "whole_step_GBps": whole_gbs,
            "whole_step_frac": whole_gbs / HBM_PEAK_GBS,
            "commit_kernel_avg_us_event_timed": c_avg_ms * 1e3 if c_n else None,
        },
        "cpu_baseline": None,
        "parallel_sweep_ceiling": ceiling,
    }
    if not args.no_cpu_baseline:
        nb = min(args.cpu_blocks, T)
        xs = torch.ones(sc.grid.nvox, dtype=vdtype, device=dev)
        api.pct_drop_iterate(plan, pr, b, xs, block=cfg.block, lam=cfg.lam, n_iter=1, block_end=nb, lanes=args.lanes,
                             flags=sched)
        torch.cuda.synchronize()
        log(f"[bench] CPU oracle baseline on {nb} blocks ...")
        cb, emax, emean = cpu_baseline(sc, cfg, xs.double().cpu().numpy(), nb, args.hull)
        out["cpu_baseline"] = cb
        out["rsp_err_vs_fp64_oracle"] = {"sample": f"first {nb} blocks of one sweep", "max": emax, "mean": emean}
    calibration_copy(args, dev)
    print(json.dumps(out), flush=True)


def calibration_copy(args, dev):
    """A plain device copy of known size, three times: the scale of the HBM
    counters (FETCH_SIZE, WRITE_SIZE) is read off it."""
    if not args.calib_copy_mib:
        return
    import torch
    nbytes = args.calib_copy_mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {args.calib_copy_mib} MiB x3 done")


if __name__ == "__main__":
    main()

"""Benchmark of the fused MLP + DROP reconstruction path on one MI355X.

Workload: the 200x200x32 (1 mm) cylinder scan with 10^7 protons over 180
projection angles, DROP block 3200, lambda 0.1, FP32 RSP volume, 12 sweeps
(one reconstruction).  One step is one DROP sweep over all 10^7 protons: for
every block, each proton's most likely path is traced, a_i.x and ||a_i||^2
computed, and the D-weighted back-projection committed.  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line:  value = proton-iterations/s, a roofline object for the
dominant kernel (the fused block kernel) and the CPU oracle baseline measured
on a bounded sample of the same scan.

    python bench.py [--gpus 1] [--steps 12] [--warmup 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def cpu_baseline(sc, cfg, x_gpu_sample, n_blocks):
    """FP64 oracle on the first n_blocks blocks of one sweep (from x0 = 1):
    throughput on the host cores and the RSP error of the GPU result on the
    same sample."""
    import oracle
    oracle.build(force=False)
    m = min(sc.m, n_blocks * cfg.block)
    sub = sc.subset(0, m)
    t0 = time.perf_counter()
    ref = oracle.drop(sc.grid, sc.mlp, sub.protons, sub.b, 1.0, block=cfg.block, lam=cfg.lam, n_iter=1)
    dt = time.perf_counter() - t0
    err = np.abs(x_gpu_sample - ref) / np.maximum(np.abs(ref), 1.0)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": m / dt, "unit": "proton-iterations/s", "cores": threads, "kind": "oracle",
        "sample": f"first {n_blocks} blocks ({m} protons) of one sweep of the same scan, FP64 C oracle, "
                  f"{dt:.1f} s",
    }, float(err.max()), float(err.mean())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="2")
    ap.add_argument("--protons", type=int, default=0, help="override the number of protons")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-blocks", type=int, default=320)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per proton in the block kernel (0: automatic)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU region split is "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1802_01070_amd import api, synth
    from paper_1802_01070_amd._lib import PCT_DROP_PROFILE

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    key = int(args.config) if args.config.isdigit() else args.config
    cfg = synth.CONFIGS[key]
    m = args.protons or cfg.m
    t0 = time.perf_counter()
    sc = synth.make_scan(cfg, m=m)
    log(f"[bench] generated {cfg.name}: {m} protons in {time.perf_counter() - t0:.1f} s")
    dev = "cuda:0"
    plan = api.Plan(sc.grid, sc.mlp, dev)
    pr = api.Protons(sc.protons, dev)
    b = torch.from_numpy(sc.b).to(dev)
    vdtype = torch.float64 if cfg.value_type == "f64" else torch.float32
    x = torch.ones(sc.grid.nvox, dtype=vdtype, device=dev)
    torch.cuda.synchronize()

    sum_nnz = count_nonzeros(api, plan, pr)
    T = (m + cfg.block - 1) // cfg.block
    log(f"[bench] sum of nonzeros {sum_nnz} ({sum_nnz / m:.1f} per proton), {T} blocks per sweep")

    # untimed warmup sweeps (the first run also compiles nothing: the library is prebuilt)
    for _ in range(args.warmup):
        api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, lanes=args.lanes)
    torch.cuda.synchronize()
    x.fill_(1.0)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t_host = time.perf_counter()
    for k in range(args.steps):
        api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, lanes=args.lanes)
        log(f"[bench] step {k + 1}/{args.steps} enqueued")
    e1.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms_total = e0.elapsed_time(e1)
    # One more sweep, right after the timed region and on the same stream, with
    # a sample of the block-kernel and commit launches bracketed by HIP events
    # (recorded by the library) to time the dominant kernel itself.
    api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=1, lanes=args.lanes,
                         flags=PCT_DROP_PROFILE)
    torch.cuda.synchronize()
    bits = api.pct_device_status(plan)
    if bits:
        log(f"[bench] WARNING device status {bits:#x}")
    ms_per_step = ms_total / args.steps
    value = m * args.steps / (ms_total / 1e3)
    (k_ms, c_ms), (k_n, c_n) = api.pct_profile_read(plan)
    k_avg_ms = k_ms / max(k_n, 1)
    c_avg_ms = c_ms / max(c_n, 1)
    bytes_per_launch = (BYTES_PER_PROTON * m + BYTES_PER_NONZERO * sum_nnz) / T
    achieved_gbs = bytes_per_launch / (k_avg_ms * 1e-3) / 1e9
    whole_gbs = (BYTES_PER_PROTON * m + BYTES_PER_NONZERO * sum_nnz) * args.steps / (ms_total * 1e-3) / 1e9
    log(f"[bench] {ms_per_step:.1f} ms/step, block kernel avg {k_avg_ms * 1e3:.2f} us ({k_n} sampled), "
        f"separate commit avg {c_avg_ms * 1e3:.2f} us ({c_n} sampled); host wall {t_host:.2f} s")

    out = {
        "metric": "proton-iterations/sec (fused MLP+DROP) at 1 GPU",
        "value": value,
        "unit": "proton-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
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
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": ("k_drop_fused (MLP trace + a.x + |a|^2 + rho + D-weighted scatter of block t, commit of "
                       "block t-1)") if c_n == 0 else "k_drop_block (MLP trace + a.x + |a|^2 + rho + scatter)",
            "lanes_per_proton": args.lanes or "auto",
            "kernel_avg_us": k_avg_ms * 1e3,
            "kernel_launches_sampled": k_n,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "whole_step_GBps": whole_gbs,
            "whole_step_frac": whole_gbs / HBM_PEAK_GBS,
            "separate_commit_avg_us": c_avg_ms * 1e3 if c_n else None,
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        nb = min(args.cpu_blocks, T)
        xs = torch.ones(sc.grid.nvox, dtype=vdtype, device=dev)
        api.pct_drop_iterate(plan, pr, b, xs, block=cfg.block, lam=cfg.lam, n_iter=1, block_end=nb, lanes=args.lanes)
        torch.cuda.synchronize()
        log(f"[bench] CPU oracle baseline on {nb} blocks ...")
        cb, emax, emean = cpu_baseline(sc, cfg, xs.double().cpu().numpy(), nb)
        out["cpu_baseline"] = cb
        out["rsp_err_vs_fp64_oracle"] = {"sample": f"first {nb} blocks of one sweep", "max": emax, "mean": emean}
    if args.calib_copy_mib:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB x3 done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Writes drop_cyl200_12sweeps.csv: the FP64 oracle's full DROP reconstruction
(Section IV-B: block-iterative DROP, 12 sweeps from x0 = 1) of a 3.2*10^6-proton
scan on the 200x200x32 cylinder geometry (the seeded generator, 180 angles,
acquisition order, block 3200 -> 1000 blocks per sweep, lambda 0.1), sampled at
8192 seeded voxels.  Calls the oracle only; the GPU test that reads the file
runs the default FP32 schedule on the same generated scan.

    python tests/golden/make_drop_cyl200_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

M = 3_200_000
N_ITER = 12
SAMPLE = 8192
SAMPLE_SEED = 77
OUT = os.path.join(HERE, "drop_cyl200_12sweeps.csv")


def sample_voxels(nvox: int) -> np.ndarray:
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(nvox, SAMPLE, replace=False))


def main():
    import oracle
    from paper_1802_01070_amd import synth
    oracle.build(force=False)
    cfg = synth.WORKLOADS[2]
    sc = synth.make_scan(cfg, m=M)
    t0 = time.perf_counter()
    x = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=cfg.block, lam=cfg.lam, n_iter=N_ITER)
    dt = time.perf_counter() - t0
    idx = sample_voxels(sc.grid.nvox)
    with open(OUT, "w") as f:
        f.write(f"# FP64 oracle DROP, {cfg.name} geometry {sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz}, m={M}, "
                f"seed {cfg.seed}, block {cfg.block}, lambda {cfg.lam}, {N_ITER} sweeps from x0 = 1, "
                f"{SAMPLE} voxels sampled with seed {SAMPLE_SEED}; oracle time {dt:.0f} s\n")
        f.write("voxel,rsp\n")
        for j in idx:
            f.write(f"{int(j)},{float(x[j])!r}\n")
    print(f"wrote {OUT} ({dt:.0f} s)")


if __name__ == "__main__":
    main()

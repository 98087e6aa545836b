"""A whole FP32 reconstruction against the FP64 oracle: 12 DROP sweeps of a
3.2*10^6-proton scan on the 200x200x32 cylinder geometry (1000 blocks of 3200
per sweep), the final RSP volume compared at the 8192 voxels of
tests/golden/drop_cyl200_12sweeps.csv (written by make_drop_cyl200_golden.py,
which calls the oracle only).  The default schedule carries the FP32
iterate's rounding error through a call, so x is rounded once per call: the
whole reconstruction in one call, and one call per sweep (12 roundings), both
stay within 1e-5 of the oracle relative to max(|x|, 0.05)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from _tol import rsp_err  # noqa: E402
from paper_1802_01070_amd import api, synth  # noqa: E402
from paper_1802_01070_amd._lib import PCT_DROP_NO_COMPENSATION  # noqa: E402

DEV = "cuda:0"
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "drop_cyl200_12sweeps.csv")
M = 3_200_000
N_ITER = 12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_full_fp32_reconstruction_matches_the_fp64_oracle():
    data = np.loadtxt(GOLDEN, delimiter=",", comments="#", skiprows=2)
    idx = data[:, 0].astype(np.int64)
    ref = data[:, 1]
    cfg = synth.WORKLOADS[2]
    say(f"full reconstruction: generating {M} protons")
    sc = synth.make_scan(cfg, m=M)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    errs = {}
    for name, calls, flags in (("one call", 1, 0), ("one call per sweep", N_ITER, 0),
                               ("no compensation, one call", 1, PCT_DROP_NO_COMPENSATION)):
        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
        for _ in range(calls):
            api.pct_drop_iterate(plan, pr, b, x, block=cfg.block, lam=cfg.lam, n_iter=N_ITER // calls, flags=flags)
        torch.cuda.synchronize()
        got = x.double().cpu().numpy()[idx]
        e = rsp_err(got, ref)
        errs[name] = e.max()
        say(f"  {name}: max rel err {e.max():.3e}, mean {e.mean():.3e}")
    assert api.pct_device_status(plan) == 0
    assert errs["one call"] <= 1e-5
    assert errs["one call per sweep"] <= 1e-5

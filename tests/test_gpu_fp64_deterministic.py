"""Deterministic FP64 DROP (PCT_DROP_DETERMINISTIC): the block sums of the
D-weighted back-projection (Section IV-B) formed as integer pairs (bits of
each contribution above 2^-28, the rest rounded at 2^-72), so repeated runs,
graph and eager launches, and a run split into block ranges are bitwise
equal, while the result stays within FP64 rounding of the FP64 oracle and of
the default FP64 schedule (double atomics)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1802_01070_amd import api, synth  # noqa: E402
from paper_1802_01070_amd._lib import (PCT_DROP_DETERMINISTIC, PCT_DROP_NO_GRAPH,  # noqa: E402
                                       PCT_DROP_CANCELLABLE)

from _tol import rsp_err  # noqa: E402

DEV = "cuda:0"
DET = PCT_DROP_DETERMINISTIC
_scans = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def scan(cfg, m):
    if (cfg, m) not in _scans:
        _scans[(cfg, m)] = synth.make_scan(synth.WORKLOADS[cfg], m=m)
    return _scans[(cfg, m)]


def drop(plan, pr, b, c, flags, x=None, **kw):
    if x is None:
        x = torch.ones(plan.nvox, dtype=torch.float64, device=DEV)
    kw.setdefault("n_iter", 2)
    api.pct_drop_iterate(plan, pr, b, x, block=c.block, lam=c.lam, flags=flags, **kw)
    torch.cuda.synchronize()
    return x


@pytest.mark.parametrize("lanes", [0, 1, 16, 64])
def test_repeated_runs_are_bitwise_equal_and_match_the_oracle(lanes):
    c = synth.WORKLOADS[1]                    # 64 x 64 x 4, FP64
    sc = scan(1, 60000)
    say(f"FP64 deterministic, lanes={lanes}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    x1 = drop(plan, pr, b, c, DET, lanes=lanes)
    x2 = drop(plan, pr, b, c, DET, lanes=lanes)
    x3 = drop(plan, pr, b, c, DET | PCT_DROP_NO_GRAPH, lanes=lanes)
    assert torch.equal(x1, x2) and torch.equal(x1, x3)
    # a sweep split into two calls applies the same block steps
    x4 = drop(plan, pr, b, c, DET, lanes=lanes, n_iter=1, block_end=7)
    x4 = drop(plan, pr, b, c, DET, x=x4, lanes=lanes, n_iter=1, block_begin=7)
    x4 = drop(plan, pr, b, c, DET, x=x4, lanes=lanes, n_iter=1)
    assert torch.equal(x1, x4)
    ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=c.block, lam=c.lam, n_iter=2)
    err = rsp_err(x1.cpu().numpy(), ref).max()
    say(f"  vs oracle {err:.3e}")
    assert err <= 1e-10
    # the default FP64 schedule (double atomics) agrees to rounding
    xa = drop(plan, pr, b, c, 0, lanes=lanes)
    assert (xa - x1).abs().max().item() <= 1e-12 * max(1.0, x1.abs().max().item())
    assert api.pct_device_status(plan) & ~0x4 == 0


def test_hull_paths_and_ragged_blocks():
    c = synth.WORKLOADS[1]
    sc = scan(1, 20000)
    plan = api.Plan(sc.grid, sc.mlp, DEV).set_hull(sc.cfg.r_hull)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    oracle.set_hull(sc.cfg.r_hull)
    try:
        for B in (37, 3200):
            x1 = torch.ones(plan.nvox, dtype=torch.float64, device=DEV)
            x2 = torch.ones(plan.nvox, dtype=torch.float64, device=DEV)
            for x in (x1, x2):
                api.pct_drop_iterate(plan, pr, b, x, block=B, lam=0.3, n_iter=2, flags=DET)
            torch.cuda.synchronize()
            assert torch.equal(x1, x2), B
            ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=B, lam=0.3, n_iter=2)
            assert rsp_err(x1.cpu().numpy(), ref).max() <= 1e-10, B
    finally:
        oracle.set_hull(None)


def test_out_of_range_contribution_is_clamped_and_flagged():
    # one ray whose rho a_ij exceeds 2^16: clamped, PCT_DEV_ACC_RANGE raised
    grid = synth.Grid(8, 8, 2)
    mlp = synth.MLPModel(u_in=-5.0, u_out=5.0)
    plan = api.Plan(grid, mlp, DEV)
    pr_np = {k: np.zeros(2, np.float32) for k in ("t_in", "v_in", "th_in", "ph_in", "t_out", "v_out", "th_out",
                                                   "ph_out", "gantry")}
    pr_np["v_in"][:] = 0.5
    pr_np["v_out"][:] = 0.5
    pr = api.Protons(pr_np, DEV)
    for bval, flagged in ((1.0, False), (3.0e6, True)):
        b = torch.full((2,), bval, dtype=torch.float32, device=DEV)
        x = torch.zeros(plan.nvox, dtype=torch.float64, device=DEV)
        # one block of both rows: each voxel's update is the mean of at most
        # two clamped contributions
        api.pct_drop_iterate(plan, pr, b, x, block=2, lam=1.0, n_iter=1, flags=DET)
        st = api.pct_device_status(plan)
        assert bool(st & 0x8) == flagged, (bval, st)
        assert torch.isfinite(x).all()
        if flagged:
            assert x.abs().max().item() == 65536.0


def test_cancel_and_resume_is_bitwise():
    c = synth.WORKLOADS[1]
    sc = scan(1, 60000)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    ref = drop(plan, pr, b, c, DET)
    api.pct_drop_cancel(plan, True)
    try:
        x = drop(plan, pr, b, c, DET | PCT_DROP_CANCELLABLE)
        assert api.pct_drop_progress(plan) == (1, True)
    finally:
        api.pct_drop_cancel(plan, False)
    x = drop(plan, pr, b, c, DET, x=x, n_iter=1, block_begin=1)
    x = drop(plan, pr, b, c, DET, x=x, n_iter=1)
    assert torch.equal(x, ref)

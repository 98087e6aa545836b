"""Cancellation of DROP between block steps (PCT_DROP_CANCELLABLE,
pct_drop_cancel, pct_drop_progress).  DROP's block step (Section IV-B) updates
x once per block, so a run stopped at a block boundary holds whole block steps
only and resumes from there: the stopped run plus its resumption must equal
the uninterrupted run, bitwise where the schedule is deterministic (the
binned FP32 schedule without compensation), else to rounding."""
import sys
import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1802_01070_amd import _lib, api, synth  # noqa: E402
from paper_1802_01070_amd._lib import (PCT_DROP_CANCELLABLE, PCT_DROP_NO_COMPENSATION,  # noqa: E402
                                       PCT_DROP_NO_GRAPH, PCT_DROP_SEPARATE_COMMIT)

DEV = "cuda:0"
CFG = synth.WORKLOADS[2]          # 200 x 200 x 32, blocks of 3200
_scans = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def scan(m):
    if m not in _scans:
        _scans[m] = synth.make_scan(CFG, m=m)
    return _scans[m]


def setup(m):
    sc = scan(m)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    return sc, plan, pr, b


def run(plan, pr, b, x0, flags, **kw):
    x = x0.clone()
    kw.setdefault("n_iter", 1)
    api.pct_drop_iterate(plan, pr, b, x, block=CFG.block, lam=CFG.lam, flags=flags, **kw)
    torch.cuda.synchronize()
    return x


def x_start(sc, dtype):
    return torch.ones(sc.grid.nvox, dtype=dtype, device=DEV)


def close(a, b, dtype, flags):
    """Bitwise for the deterministic schedules (FP32 integer block sums); FP64
    block sums are formed with FP64 atomics, whose order varies."""
    if dtype == torch.float32:
        return torch.equal(a, b)
    return float((a - b).abs().max()) <= 1e-12 * max(1.0, float(b.abs().max()))


SCHEDULES = [(torch.float32, 0), (torch.float32, PCT_DROP_NO_COMPENSATION),
             (torch.float32, PCT_DROP_SEPARATE_COMMIT), (torch.float64, 0),
             (torch.float32, PCT_DROP_NO_COMPENSATION | PCT_DROP_NO_GRAPH),
             (torch.float32, PCT_DROP_NO_COMPENSATION | _lib.PCT_DROP_PROFILE)]


@pytest.mark.parametrize("dtype,flags", SCHEDULES)
def test_request_before_the_call_applies_one_block_step(dtype, flags):
    sc, plan, pr, b = setup(48000)
    say(f"cancel before the call: dtype={dtype} flags={flags:#x}")
    x0 = x_start(sc, dtype)
    api.pct_drop_cancel(plan, True)
    try:
        x = run(plan, pr, b, x0, flags | PCT_DROP_CANCELLABLE, n_iter=2)
        done, stopped = api.pct_drop_progress(plan)
        assert (done, stopped) == (1, True)
        assert api.pct_device_status(plan) & 0x20
    finally:
        api.pct_drop_cancel(plan, False)
    ref = run(plan, pr, b, x0, flags, block_end=1)
    assert close(x, ref, dtype, flags)
    assert not torch.equal(x, x0)


@pytest.mark.parametrize("dtype,flags", SCHEDULES)
def test_without_a_request_the_call_runs_to_its_end(dtype, flags):
    sc, plan, pr, b = setup(48000)
    x0 = x_start(sc, dtype)
    nblk = (sc.m + CFG.block - 1) // CFG.block
    x = run(plan, pr, b, x0, flags | PCT_DROP_CANCELLABLE, n_iter=2)
    assert api.pct_drop_progress(plan) == (2 * nblk, False)
    assert api.pct_device_status(plan) & 0x20 == 0
    ref = run(plan, pr, b, x0, flags, n_iter=2)
    assert close(x, ref, dtype, flags)
    # a block range: steps counted over the range only
    x = run(plan, pr, b, x0, flags | PCT_DROP_CANCELLABLE, n_iter=3, block_begin=4, block_end=9)
    assert api.pct_drop_progress(plan) == (15, False)
    # no work: the progress of this (empty) call
    x = run(plan, pr, b, x0, flags | PCT_DROP_CANCELLABLE, n_iter=0)
    assert api.pct_drop_progress(plan) == (0, False)


def test_calls_without_the_flag_ignore_a_request():
    sc, plan, pr, b = setup(48000)
    x0 = x_start(sc, torch.float32)
    ref = run(plan, pr, b, x0, 0, n_iter=2)
    api.pct_drop_cancel(plan, True)
    try:
        x = run(plan, pr, b, x0, 0, n_iter=2)
    finally:
        api.pct_drop_cancel(plan, False)
    assert torch.equal(x, ref)
    # the fused atomic schedule is not used by a cancellable call: the flag
    # runs the separate schedule, bitwise the same block sums
    fused = run(plan, pr, b, x0, _lib.PCT_DROP_FUSED_COMMIT | PCT_DROP_NO_COMPENSATION, n_iter=2)
    sep = run(plan, pr, b, x0, _lib.PCT_DROP_FUSED_COMMIT | PCT_DROP_NO_COMPENSATION | PCT_DROP_CANCELLABLE, n_iter=2)
    assert torch.equal(fused, sep)


@pytest.mark.parametrize("dtype,flags", [(torch.float32, PCT_DROP_NO_COMPENSATION), (torch.float32, 0),
                                         (torch.float64, 0), (torch.float64, _lib.PCT_DROP_DETERMINISTIC)])
def test_cancel_mid_run_then_resume(dtype, flags):
    m = 10_000_000 if dtype == torch.float32 else 2_000_000
    sc, plan, pr, b = setup(m)
    nblk = (sc.m + CFG.block - 1) // CFG.block
    n_iter = 3
    x0 = x_start(sc, dtype)
    # one timed sweep: the request lands about half a sweep into the run
    t0 = time.perf_counter()
    ref1 = run(plan, pr, b, x0, flags, n_iter=1)
    sweep_s = time.perf_counter() - t0
    ref = run(plan, pr, b, ref1, flags, n_iter=n_iter - 1)
    x = x0.clone()
    api.pct_drop_iterate(plan, pr, b, x, block=CFG.block, lam=CFG.lam, n_iter=n_iter,
                         flags=flags | PCT_DROP_CANCELLABLE)
    th = threading.Thread(target=lambda: (time.sleep(0.5 * sweep_s), api.pct_drop_cancel(plan, True)))
    th.start()
    th.join()
    done, stopped = api.pct_drop_progress(plan)
    api.pct_drop_cancel(plan, False)
    say(f"  {dtype} flags={flags:#x}: sweep {sweep_s * 1e3:.0f} ms, stopped after {done} of {n_iter * nblk} steps")
    assert stopped and 0 < done < n_iter * nblk
    # resume: the rest of the interrupted sweep, then the remaining sweeps
    s, k = divmod(done, nblk)
    if k > 0:
        api.pct_drop_iterate(plan, pr, b, x, block=CFG.block, lam=CFG.lam, n_iter=1, block_begin=k, flags=flags)
        s += 1
    if n_iter - s > 0:
        api.pct_drop_iterate(plan, pr, b, x, block=CFG.block, lam=CFG.lam, n_iter=n_iter - s, flags=flags)
    torch.cuda.synchronize()
    if (dtype == torch.float32 and flags & PCT_DROP_NO_COMPENSATION) or flags & _lib.PCT_DROP_DETERMINISTIC:
        assert torch.equal(x, ref)
    elif dtype == torch.float32:
        # compensated: each call starts its compensation word at zero, so the
        # resumed run carries one more FP32 rounding of x
        d = (x.double() - ref.double()).abs().max().item()
        assert d <= 2.0 ** -22 * max(1.0, ref.abs().max().item()), d
    else:
        assert close(x, ref, dtype, flags)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_hull_paths_stop_at_a_block_boundary(dtype):
    # per-proton hull paths run their own kernel instances; the gate is the same
    sc, plan, pr, b = setup(20000)
    plan.set_hull(sc.cfg.r_hull - 8.0)
    x0 = x_start(sc, dtype)
    flags = PCT_DROP_NO_COMPENSATION if dtype == torch.float32 else _lib.PCT_DROP_DETERMINISTIC
    api.pct_drop_cancel(plan, True)
    try:
        x = run(plan, pr, b, x0, flags | PCT_DROP_CANCELLABLE, n_iter=2)
        assert api.pct_drop_progress(plan) == (1, True)
    finally:
        api.pct_drop_cancel(plan, False)
    ref = run(plan, pr, b, x0, flags, block_end=1)
    assert torch.equal(x, ref)
    # and resumed: the rest of the first sweep and one more
    x = run(plan, pr, b, x, flags, block_begin=1)
    x = run(plan, pr, b, x, flags)
    assert torch.equal(x, run(plan, pr, b, x0, flags, n_iter=2))

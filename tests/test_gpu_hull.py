"""GPU parity of the per-proton hull paths (the MLP between the points where
the tracks cross the object hull, straight tracks outside): traces bit-exact
against the oracle, operators, DROP on every block schedule, stored rows."""
import sys

import numpy as np
import pytest
import torch

import oracle
from _tol import rsp_err
from paper_1802_01070_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
HULLS = {1: 24.0, 2: 92.0}      # radii (mm): inside the tracker span of each scan


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _hull_off():
    oracle.build(force=False)
    oracle.set_hull(None)
    yield
    oracle.set_hull(None)
    torch.cuda.synchronize()


_scans = {}


def scan(cfg, m):
    if (cfg, m) not in _scans:
        _scans[(cfg, m)] = synth.make_scan(synth.WORKLOADS[cfg], m=m)
    return _scans[(cfg, m)]


def setup(cfg, m, radius):
    sc = scan(cfg, m)
    plan = api.Plan(sc.grid, sc.mlp, DEV).set_hull(radius)
    oracle.set_hull(radius)
    return sc, plan, api.Protons(sc.protons, DEV)


@pytest.mark.parametrize("cfg", [1, 2])
def test_hull_traces_bit_exact(cfg):
    sc, plan, pr = setup(cfg, 20000, HULLS[cfg])
    say(f"hull trace {sc.cfg.name} R={HULLS[cfg]}")
    cap = 1024
    vox, ch, nnz = api.pct_mlp_trace(plan, pr, 0, sc.m, max_nnz=cap)
    torch.cuda.synchronize()
    vox, ch, nnz = vox.cpu().numpy(), ch.cpu().numpy(), nnz.cpu().numpy()
    rv, rc, rn = oracle.trace(sc.grid, sc.mlp, sc.protons, cap=cap)
    assert np.array_equal(nnz, rn)
    mask = np.arange(cap)[None, :] < rn[:, None]
    assert np.array_equal(vox[mask], rv[mask])
    assert np.abs(ch - rc)[mask].max() <= 1e-9
    # the hull changes the rows: some protons miss it, all others bend inside it
    plain = api.Plan(sc.grid, sc.mlp, DEV)
    _, _, n0 = api.pct_mlp_trace(plain, pr, 0, sc.m, max_nnz=1)
    assert not np.array_equal(n0.cpu().numpy(), nnz)
    assert api.pct_device_status(plan) == 0


def test_hull_beyond_the_trackers_is_the_tracker_path():
    sc = scan(1, 5000)
    pr = api.Protons(sc.protons, DEV)
    hull = api.Plan(sc.grid, sc.mlp, DEV).set_hull(1.0e4)
    plain = api.Plan(sc.grid, sc.mlp, DEV)
    a = api.pct_mlp_trace(hull, pr, 0, sc.m, max_nnz=512)
    b = api.pct_mlp_trace(plain, pr, 0, sc.m, max_nnz=512)
    torch.cuda.synchronize()
    assert torch.equal(a[2], b[2]) and torch.equal(a[0], b[0])
    assert (a[1] - b[1]).abs().max().item() <= 1e-9        # device vs host coefficients: last bits


def test_hull_forward_backproject_match_oracle():
    sc, plan, pr = setup(2, 20000, HULLS[2])
    x = torch.from_numpy(sc.x_true()).to(DEV)
    y, n2 = api.pct_forward(plan, pr, x, with_norm=True)
    ry, rn2, _ = oracle.forward(sc.grid, sc.mlp, sc.protons, sc.x_true())
    assert np.max(np.abs(y.cpu().numpy() - ry)) <= 1e-8 * max(1.0, np.abs(ry).max())
    np.testing.assert_allclose(n2.cpu().numpy(), rn2, rtol=1e-9, atol=1e-9)
    r = np.random.default_rng(3).standard_normal(sc.m)
    g = api.pct_backproject(plan, pr, torch.from_numpy(r).to(DEV))
    rg = oracle.backproject(sc.grid, sc.mlp, sc.protons, r)
    assert np.max(np.abs(g.cpu().numpy() - rg)) <= 1e-9 * max(1.0, np.abs(rg).max())


def test_hull_drop_fp64_matches_oracle():
    c = synth.WORKLOADS[1]
    sc, plan, pr = setup(1, 20000, HULLS[1])
    b = torch.from_numpy(sc.b).to(DEV)
    ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=c.block, lam=c.lam, n_iter=2)
    for lanes in (0, 1):
        x = torch.ones(sc.grid.nvox, dtype=torch.float64, device=DEV)
        api.pct_drop_iterate(plan, pr, b, x, block=c.block, lam=c.lam, n_iter=2, lanes=lanes)
        err = np.max(rsp_err(x.cpu().numpy(), ref))
        say(f"  hull FP64 lanes={lanes}: {err:.3e}")
        assert err <= 1e-10
    assert api.pct_device_status(plan) == 0


def test_hull_drop_fp32_schedules_bitwise_and_match_oracle():
    from paper_1802_01070_amd._lib import (PCT_DROP_FUSED_COMMIT, PCT_DROP_NO_COMPENSATION,
                                           PCT_DROP_NO_TRACE_AHEAD, PCT_DROP_SEPARATE_COMMIT)
    c = synth.WORKLOADS[2]
    sc, plan, pr = setup(2, 64000, HULLS[2])
    b = torch.from_numpy(sc.b).to(DEV)
    pr, b = api.pct_order_blocks(plan, pr, b, c.block)
    order_np = {k: v.cpu().numpy() for k, v in pr.t.items()}
    out = []
    # atomic schedules and the binned one without compensation: bitwise; the
    # default (binned, compensated) within the FP32 tolerance of the oracle
    for flags in (PCT_DROP_FUSED_COMMIT, PCT_DROP_FUSED_COMMIT | PCT_DROP_NO_TRACE_AHEAD, PCT_DROP_SEPARATE_COMMIT,
                  PCT_DROP_NO_COMPENSATION, 0):
        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
        api.pct_drop_iterate(plan, pr, b, x, block=c.block, lam=c.lam, n_iter=2, flags=flags)
        out.append(x)
    torch.cuda.synchronize()
    for k in (1, 2, 3):
        assert torch.equal(out[0], out[k]), k
    ref = oracle.drop(sc.grid, sc.mlp, order_np, b.cpu().numpy(), 1.0, block=c.block, lam=c.lam, n_iter=2)
    for k in (0, 4):
        err = np.max(rsp_err(out[k].double().cpu().numpy(), ref))
        say(f"  hull FP32 200x200x32 ({k}): {err:.3e}")
        assert err <= 1e-5
    assert api.pct_device_status(plan) == 0


def test_hull_stored_rows_match_oracle():
    c = synth.WORKLOADS[4]
    sc, plan, pr = setup(2, 32000, HULLS[2])
    b = torch.from_numpy(sc.b).to(DEV)
    rows = api.Rows(plan, pr, "f16")
    off = rows.offsets.cpu().numpy()
    _, _, rn = oracle.trace(sc.grid, sc.mlp, sc.protons, cap=1)
    assert np.array_equal(np.diff(off), rn)
    x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
    api.pct_drop_iterate_rows(plan, rows, b, x, block=c.block, lam=c.lam, n_iter=2)
    ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=c.block, lam=c.lam, n_iter=2, mode="f16")
    err = np.max(rsp_err(x.double().cpu().numpy(), ref))
    say(f"  hull stored f16 rows: {err:.3e}")
    assert err <= 1e-5
    assert api.pct_device_status(plan) == 0


@pytest.mark.parametrize("radius", [None, 24.0])
def test_drop_rows_ending_on_a_grid_plane(radius):
    # at gantry 0 the tracker planes u = -30, 30 mm are the grid planes
    # x = -30, 30 of the 64-voxel grid, so every path ends on a plane; with 64
    # lanes per proton the lane whose range starts at that plane adds no piece
    # (a piece of rounding length would add a voxel to the row and to s_j)
    grid = synth.Grid(64, 64, 4)
    mlp = synth.MLPModel(u_in=-30.0, u_out=30.0)
    rng = np.random.default_rng(11)
    n = 1280
    th = rng.uniform(-0.1, 0.1, n)
    ph = rng.uniform(-0.02, 0.02, n)
    t_in = rng.uniform(-25.0, 25.0, n)
    v_in = rng.uniform(-1.5, 1.5, n)
    rays = np.stack([t_in, v_in, th, ph, t_in + 60.0 * th + rng.normal(0, 0.5, n),
                     np.clip(v_in + 60.0 * ph, -1.9, 1.9), th + rng.normal(0, 0.01, n), ph,
                     np.zeros(n)], axis=1)
    protons = synth.make_rays(grid, mlp, rays)
    b = rng.uniform(10.0, 60.0, n).astype(np.float32)
    plan = api.Plan(grid, mlp, DEV)
    if radius is not None:
        plan.set_hull(radius)
    oracle.set_hull(radius)
    pr = api.Protons(protons, DEV)
    _, _, nnz = api.pct_mlp_trace(plan, pr, 0, n, max_nnz=128)
    _, _, rn = oracle.trace(grid, mlp, protons, cap=1)
    assert rn.max() <= 128 and np.array_equal(nnz.cpu().numpy(), rn)
    ref = oracle.drop(grid, mlp, protons, b, 1.0, block=64, lam=0.5, n_iter=2)
    for lanes in (64, 1):
        x = torch.ones(grid.nvox, dtype=torch.float64, device=DEV)
        api.pct_drop_iterate(plan, pr, torch.from_numpy(b).to(DEV), x, block=64, lam=0.5, n_iter=2, lanes=lanes)
        err = np.max(rsp_err(x.cpu().numpy(), ref))
        say(f"  end-on-plane R={radius} lanes={lanes}: {err:.3e}")
        assert err <= 1e-10
    assert api.pct_device_status(plan) == 0

"""GPU parity of the multi-region reconstruction (Algorithm 1, Section III):
region selection bit-exact against the oracle's membership, slice copies, and
the region-split DROP against the region-aware oracle."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import oracle
from _tol import rsp_err
from oracle import regions as R
from paper_1802_01070_amd import _lib, api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    oracle.build(force=False)
    yield
    torch.cuda.synchronize()


@pytest.fixture(autouse=True)
def _hull_off():
    oracle.set_hull(None)
    yield
    oracle.set_hull(None)


_scans = {}


def scan(key, m=None):
    if (key, m) not in _scans:
        _scans[(key, m)] = synth.make_scan(synth.WORKLOADS[key], m=m)
    return _scans[(key, m)]


def with_edge_tracks(sc):
    """Copy of the scan's records with tracks on slice boundaries, outside
    the grid in z and non-finite, spread over the input."""
    pr = {k: v.copy() for k, v in sc.protons.items()}
    z0, pz, nz = sc.grid.origin[2], sc.grid.pitch[2], sc.grid.nz
    n = len(pr["v_in"])
    idx = np.arange(5, n, max(1, n // 200))
    vals = np.array([z0, z0 + 7 * pz, z0 + 13 * pz, z0 + nz * pz, z0 - 3.0, z0 + nz * pz + 2.0, np.nan, np.inf],
                    dtype=np.float32)
    pr["v_in"][idx] = vals[np.arange(len(idx)) % len(vals)]
    pr["v_out"][idx[::3]] = vals[(np.arange(len(idx[::3])) + 3) % len(vals)]
    return pr


@pytest.mark.parametrize("z_lo,z_hi", [(0, 12), (7, 19), (0, 19), (5, 5), (19, 19)])
def test_region_select_bit_exact(z_lo, z_hi):
    sc = scan("regions")
    pr_np = with_edge_tracks(sc)
    say(f"region select [{z_lo},{z_hi}] m={sc.m}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(pr_np, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    sub, b_sub = api.pct_region_select(plan, pr, b, z_lo, z_hi)
    idx = R.members(sc.grid, pr_np, z_lo, z_hi)
    assert sub.n == len(idx)
    for k in _lib.FIELDS:
        got = sub.t[k].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), pr_np[k][idx].view(np.uint32)), k
    assert np.array_equal(b_sub.cpu().numpy(), sc.b[idx])
    # without b
    sub2, none = api.pct_region_select(plan, pr, None, z_lo, z_hi)
    assert none is None and sub2.n == len(idx)


@pytest.mark.parametrize("key", ["regions", 2])
def test_slice_span_histogram_and_halo(key):
    sc = scan(key)
    pr_np = with_edge_tracks(sc) if key == "regions" else sc.protons
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(pr_np, DEV)
    hist = api.pct_slice_span_histogram(plan, pr).cpu().numpy()
    si = R.slice_of(sc.grid, pr_np["v_in"])
    so = R.slice_of(sc.grid, pr_np["v_out"])
    ok = (si >= 0) & (so >= 0)
    ref = np.bincount(np.abs(si - so)[ok], minlength=sc.grid.nz)
    assert np.array_equal(hist, ref)
    for target in (0.5, 0.9, 0.96, 0.99):
        assert api.overlap_halo(torch.from_numpy(hist), target) == R.halo_for(sc.grid, {k: v[ok] for k, v in
                                                                                         pr_np.items()}, target)
    say(f"  {sc.cfg.name}: halo for 96% = {api.overlap_halo(torch.from_numpy(hist), 0.96)}")


def test_region_select_capacity_and_empty_input():
    sc = scan("regions")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    idx = R.members(sc.grid, sc.protons, 3, 9)
    cap = len(idx) // 2
    bufs = {k: torch.full((cap,), -7.0, dtype=torch.float32, device=DEV) for k in _lib.FIELDS}
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    out = _lib.make_protons_buf({k: v.data_ptr() for k, v in bufs.items()}, cap)
    st = _lib.lib().pct_region_select(plan.handle, C.byref(pr.s), None, 3, 9, C.byref(out), None,
                                      C.c_void_p(cnt.data_ptr()), plan.ws_ptr, plan.ws_bytes,
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    assert int(cnt.item()) == len(idx)                      # the true count
    for k in _lib.FIELDS:
        assert np.array_equal(bufs[k].cpu().numpy(), sc.protons[k][idx[:cap]])
    empty = pr.slice(0, 0)
    sub, bs = api.pct_region_select(plan, empty, None, 0, 19)
    assert sub.n == 0


def test_region_select_full_size_counts():
    c = synth.WORKLOADS[2]
    sc = scan(2, c.m)
    say(f"region select full size m={sc.m}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    halo = R.halo_for(sc.grid, sc.protons, 0.96)
    for z_lo, z_hi, _, _ in R.layout(sc.grid.nz, 2, halo):
        sub, _ = api.pct_region_select(plan, pr, None, z_lo, z_hi)
        idx = R.members(sc.grid, sc.protons, z_lo, z_hi)
        assert sub.n == len(idx)
        rng = np.random.default_rng(z_lo)
        pick = rng.choice(len(idx), 2000, replace=False)
        for k in ("v_in", "v_out", "t_in", "gantry"):
            got = sub.t[k][torch.from_numpy(pick).to(DEV)].cpu().numpy()
            assert np.array_equal(got, sc.protons[k][idx[pick]]), k


def test_select_slices_round_trip():
    sc = scan("regions", 1000)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    plane = sc.grid.nx * sc.grid.ny
    for dtype in (torch.float32, torch.float64):
        x = torch.arange(sc.grid.nvox, dtype=dtype, device=DEV)
        xr = torch.zeros(6 * plane, dtype=dtype, device=DEV)
        api.pct_select_slices(plan, x, 0, xr, 7, 7, 6)               # slices 7..12 out
        assert torch.equal(xr, x[7 * plane:13 * plane])
        y = torch.full_like(x, -1)
        api.pct_select_slices(plan, xr, 7, y, 0, 9, 2)               # slices 9..10 back
        assert torch.equal(y[9 * plane:11 * plane], x[9 * plane:11 * plane])
        assert torch.all(y[:9 * plane] == -1) and torch.all(y[11 * plane:] == -1)


@pytest.mark.parametrize("n_reg,halo,dtype,tol,hull", [(2, 3, torch.float64, 1e-10, None),
                                                       (3, 2, torch.float64, 1e-10, None),
                                                       (2, 3, torch.float32, 1e-5, None),
                                                       (2, 3, torch.float64, 1e-10, 29.0)])
def test_region_drop_matches_region_oracle(n_reg, halo, dtype, tol, hull):
    sc = scan("regions")
    c = sc.cfg
    say(f"region DROP R={n_reg} halo={halo} {dtype} m={sc.m} hull={hull}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    if hull is not None:
        plan.set_hull(hull)                 # region plans inherit it
    oracle.set_hull(hull)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    x0 = np.random.default_rng(4).uniform(0.8, 1.2, sc.grid.nvox)
    x = torch.from_numpy(x0).to(DEV, dtype)
    x0_used = x0.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)
    # one sweep, then one more on the same per-region state
    state = api.region_drop(plan, pr, b, x, n_reg, halo, c.block, c.lam, 1)
    api.region_drop(plan, pr, b, x, n_reg, halo, c.block, c.lam, 1, regions=state)
    torch.cuda.synchronize()
    ref, info = R.region_drop(sc.grid, sc.mlp, sc.protons, sc.b, x0_used, n_reg, halo, c.block, c.lam, 2)
    assert [s["protons"].n for s in state] == [r[4] for r in info]
    err = rsp_err(x.double().cpu().numpy(), ref)
    say(f"  max err {err.max():.3e}")
    assert err.max() <= tol
    for s in state:
        assert api.pct_device_status(s["plan"]) == 0
        assert s["plan"].hull == plan.hull

"""Edge cases of the binned FP32 schedule (Section IV-B's block step with the
D-weighted back-projection summed per slab in LDS): a slab whose window does
not fit one workgroup's LDS (split into z chunks), blocks that mix both
dominant axes and every gantry angle (rows sent to the overflow accumulator),
the largest block the bins hold and the first one past it (atomic schedule),
a ragged last block, against the FP64 oracle and, without compensation,
bitwise against the separate schedule."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1802_01070_amd import api, synth  # noqa: E402
from paper_1802_01070_amd._lib import (PCT_DROP_NO_COMPENSATION, PCT_DROP_NO_GRAPH,  # noqa: E402
                                       PCT_DROP_SEPARATE_COMMIT)

from _tol import rsp_err  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def random_scan(grid, mlp, m, seed):
    """Straight-ish rays at uniform gantry angles across the grid (lateral
    position and height uniform, small track angles), with positive WEPL."""
    rng = np.random.default_rng(seed)
    half = 0.5 * max(grid.nx * grid.pitch[0], grid.ny * grid.pitch[1])
    t = rng.uniform(-half, half, m)
    v = rng.uniform(-0.45 * grid.nz * grid.pitch[2], 0.45 * grid.nz * grid.pitch[2], m)
    th = rng.normal(0.0, 0.01, m)
    ph = rng.normal(0.0, 0.01, m)
    depth = mlp.u_out - mlp.u_in
    phi = rng.uniform(0.0, 2.0 * np.pi, m)
    prot = {k: a.astype(np.float32) for k, a in dict(
        t_in=t, v_in=v, th_in=th, ph_in=ph, t_out=t + depth * th, v_out=v + depth * ph, th_out=th, ph_out=ph,
        gantry=phi).items()}
    b = rng.uniform(20.0, 120.0, m).astype(np.float32)
    return prot, b


def run(plan, pr, b, nvox, block, flags, n_iter=2):
    x = torch.ones(nvox, dtype=torch.float32, device=DEV)
    api.pct_drop_iterate(plan, pr, b, x, block=block, lam=0.1, n_iter=n_iter, flags=flags)
    torch.cuda.synchronize()
    return x


@pytest.mark.parametrize("grid,sort", [
    # x slabs of 300 x 64 cells: two z chunks per slab (54 + 10 slices)
    (synth.Grid(40, 300, 64), True),
    # every angle inside a block: rows of both dominant axes, overflow words
    (synth.Grid(96, 64, 12), False),
])
def test_binned_schedule_edges_match_oracle_and_separate(grid, sort):
    half = 0.5 * max(grid.nx, grid.ny) + 10.0
    mlp = synth.MLPModel(u_in=-half, u_out=half)
    m, block = 25_000, 3200
    prot, bb = random_scan(grid, mlp, m, seed=grid.nx)
    if sort:
        # blocks of one dominant axis, as an angle-sorted scan gives
        key = np.where(np.abs(np.cos(prot["gantry"])) >= np.abs(np.sin(prot["gantry"])), 0, 1)
        perm = np.argsort(key, kind="stable")
        prot = {k: a[perm] for k, a in prot.items()}
        bb = bb[perm]
    say(f"binned edges: grid {grid.nx}x{grid.ny}x{grid.nz}, sorted={sort}")
    plan = api.Plan(grid, mlp, DEV)
    pr = api.Protons(prot, DEV)
    b = torch.from_numpy(bb).to(DEV)
    nvox = grid.nx * grid.ny * grid.nz
    xb = run(plan, pr, b, nvox, block, 0)
    xn = run(plan, pr, b, nvox, block, PCT_DROP_NO_COMPENSATION)
    xe = run(plan, pr, b, nvox, block, PCT_DROP_NO_COMPENSATION | PCT_DROP_NO_GRAPH)
    xs = run(plan, pr, b, nvox, block, PCT_DROP_SEPARATE_COMMIT)
    assert torch.equal(xn, xs) and torch.equal(xn, xe)
    ref = oracle.drop(grid, mlp, prot, bb, 1.0, block=block, lam=0.1, n_iter=2)
    err = rsp_err(xb.double().cpu().numpy(), ref).max()
    say(f"  compensated binned vs oracle {err:.3e}")
    assert err <= 1e-5
    assert not torch.equal(xb, torch.ones_like(xb))
    assert api.pct_device_status(plan) & ~0x4 == 0


def test_largest_binned_block_and_the_first_past_it():
    grid = synth.Grid(64, 64, 8)
    mlp = synth.MLPModel(u_in=-45.0, u_out=45.0)
    m = 8192 + 8193 + 517                          # ragged last block for both block sizes
    prot, bb = random_scan(grid, mlp, m, seed=5)
    plan = api.Plan(grid, mlp, DEV, n_hint=8193)
    pr = api.Protons(prot, DEV)
    b = torch.from_numpy(bb).to(DEV)
    nvox = grid.nx * grid.ny * grid.nz
    for block in (8192, 8193):
        say(f"  block {block}")
        xn = run(plan, pr, b, nvox, block, PCT_DROP_NO_COMPENSATION)
        xs = run(plan, pr, b, nvox, block, PCT_DROP_SEPARATE_COMMIT)
        assert torch.equal(xn, xs), block
        xb = run(plan, pr, b, nvox, block, 0)
        ref = oracle.drop(grid, mlp, prot, bb, 1.0, block=block, lam=0.1, n_iter=2)
        assert rsp_err(xb.double().cpu().numpy(), ref).max() <= 1e-5, block
    assert api.pct_device_status(plan) & ~0x4 == 0

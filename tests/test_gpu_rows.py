"""GPU parity of the stored-row form of the precision path: the CSR rows the
library traces once (offsets, voxel lists with first-visit bits, rounded
chords, ||a_i||^2) against the oracle's emission lists, and DROP sweeps over
the stored rows against the oracle's DROP with the same chord rounding."""
import sys

import numpy as np
import pytest
import torch

import oracle
from _tol import rsp_err
from paper_1802_01070_amd import api, synth

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


_scans = {}


def scan(cfg, m):
    if (cfg, m) not in _scans:
        _scans[(cfg, m)] = synth.make_scan(synth.WORKLOADS[cfg], m=m)
    return _scans[(cfg, m)]


def stored_values(rows):
    c = rows.chord[:rows.nnz]
    if rows.chord_name == "f32":
        return c.double().cpu().numpy()
    if rows.chord_name == "f16":
        return c.view(torch.float16).double().cpu().numpy()
    return c.view(torch.bfloat16).double().cpu().numpy()


@pytest.mark.parametrize("chord", ["f32", "f16", "bf16"])
def test_rows_match_oracle_emission_lists(chord):
    sc = scan(1, 4000)
    say(f"rows {chord} 64x64x4 m={sc.m}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    rows = api.Rows(plan, pr, chord)
    torch.cuda.synchronize()
    assert api.pct_device_status(plan) == 0
    rv, rc, rn = oracle.trace(sc.grid, sc.mlp, sc.protons, cap=1024)
    off = rows.offsets.cpu().numpy()
    assert off[0] == 0 and np.array_equal(np.diff(off), rn)
    vox = rows.vox[:rows.nnz].cpu().numpy()
    got_c = stored_values(rows)
    n2_ref = oracle.forward(sc.grid, sc.mlp, sc.protons, None, mode=chord)[1]
    n2 = rows.n2.cpu().numpy()
    rnd = np.vectorize(lambda v: oracle.round_chord(v, chord))
    flips = 0
    for i in range(sc.m):
        seg = slice(off[i], off[i + 1])
        j = vox[seg] & 0x7FFFFFFF
        assert np.array_equal(j, rv[i, :rn[i]]), i
        # bit 31 marks the first piece of every distinct voxel of the row
        seen = set()
        first = np.array([not (v in seen or seen.add(v)) for v in j.tolist()])
        assert np.array_equal(vox[seg] < 0, first), i
        ref_c = rnd(rc[i, :rn[i]]) if rn[i] else np.zeros(0)
        # chords agree to 1e-9 mm before rounding; a value that close to a
        # rounding boundary may land one unit apart
        d = got_c[seg] != ref_c
        flips += int(d.sum())
        if d.any():
            ulp = np.abs(ref_c[d]) * (2.0 ** -10 if chord == "f16" else 2.0 ** -7 if chord == "bf16" else 2.0 ** -23)
            assert np.all(np.abs(got_c[seg][d] - ref_c[d]) <= ulp * 1.01), i
    assert flips <= max(2, rows.nnz // 100000)
    np.testing.assert_allclose(n2, n2_ref, rtol=1e-4 if flips else 1e-12, atol=0)


@pytest.mark.parametrize("chord,lanes", [("f16", 0), ("bf16", 32), ("f32", 16)])
def test_drop_over_stored_rows_matches_oracle(chord, lanes):
    c = synth.WORKLOADS[4]
    sc = scan(4, 32000)
    say(f"stored-row DROP {chord} lanes={lanes} m={sc.m}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    rows = api.Rows(plan, pr, chord)
    x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
    api.pct_drop_iterate_rows(plan, rows, b, x, block=c.block, lam=c.lam, n_iter=2, lanes=lanes)
    # the recomputing path with the same rounding
    xr = torch.ones_like(x)
    api.pct_drop_iterate(plan, pr, b, xr, block=c.block, lam=c.lam, n_iter=2, chord=chord)
    torch.cuda.synchronize()
    ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=c.block, lam=c.lam, n_iter=2, mode=chord)
    got = x.double().cpu().numpy()
    err = np.max(rsp_err(got, ref))
    say(f"  vs oracle {err:.3e}; vs recomputed rows {(x - xr).abs().max().item():.3e}")
    assert err <= 1e-5
    assert (x - xr).abs().max().item() <= 1e-5
    assert api.pct_device_status(plan) == 0


def test_stored_rows_ragged_blocks_resume_and_empty():
    sc = scan(1, 10000)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    rows = api.Rows(plan, pr, "f32")
    for B in (37, 3200):
        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
        api.pct_drop_iterate_rows(plan, rows, b, x, block=B, lam=0.3, n_iter=2)
        ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, 1.0, block=B, lam=0.3, n_iter=2, mode="f32")
        err = np.max(rsp_err(x.double().cpu().numpy(), ref))
        assert err <= 1e-5, (B, err)
    # resume and bitwise reproducibility (integer block accumulator)
    x1 = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
    api.pct_drop_iterate_rows(plan, rows, b, x1, block=3200, lam=0.1, n_iter=1)
    x2 = torch.ones_like(x1)
    api.pct_drop_iterate_rows(plan, rows, b, x2, block=3200, lam=0.1, n_iter=1, block_end=2)
    api.pct_drop_iterate_rows(plan, rows, b, x2, block=3200, lam=0.1, n_iter=1, block_begin=2)
    assert torch.equal(x1, x2)
    x3 = torch.ones_like(x1)
    api.pct_drop_iterate_rows(plan, rows, b, x3, block=3200, lam=0.1, n_iter=0)
    api.pct_drop_iterate_rows(plan, rows, b, x3, block=3200, lam=0.1, n_iter=1, block_begin=2, block_end=2)
    assert torch.all(x3 == 1.0)
    empty = api.Rows(plan, pr.slice(0, 0), "f16")
    assert empty.nnz == 0
    assert api.pct_device_status(plan) == 0


def test_stored_rows_full_size_sampled_blocks():
    # 2*10^7 protons on the 200x200x32 grid with FP16 chords (the precision
    # workload at its full size); sampled blocks checked one by one against
    # the oracle started from the GPU's own iterate
    c = synth.WORKLOADS[4]
    sc = scan(4, c.m)
    say(f"stored rows full size m={sc.m}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    rows = api.Rows(plan, pr, "f16")
    say(f"  {rows.nnz} pieces ({rows.nnz / sc.m:.1f} per row), {rows.nbytes / 2**30:.1f} GiB")
    x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
    T = (sc.m + c.block - 1) // c.block
    done = 0
    for t in (0, 1, 2500, T - 1):
        if t > done:
            api.pct_drop_iterate_rows(plan, rows, b, x, block=c.block, lam=c.lam, n_iter=1, block_begin=done,
                                      block_end=t)
        x_before = x.double().cpu().numpy()
        api.pct_drop_iterate_rows(plan, rows, b, x, block=c.block, lam=c.lam, n_iter=1, block_begin=t,
                                  block_end=t + 1)
        sub = sc.subset(t * c.block, min(sc.m, (t + 1) * c.block))
        ref = oracle.drop(sc.grid, sc.mlp, sub.protons, sub.b, x_before, block=c.block, lam=c.lam, n_iter=1,
                          mode="f16")
        err = np.max(rsp_err(x.double().cpu().numpy(), ref))
        say(f"  block {t}: max err {err:.3e}")
        assert err <= 1e-5
        done = t + 1
    assert api.pct_device_status(plan) == 0

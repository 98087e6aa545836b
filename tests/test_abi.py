"""C-ABI contract tests that need no GPU: the library loads, exports every
function include/pct.h declares, validates arguments on the host before any
HIP call, and its host-side MLP table (Gauss-Legendre + Kalman-gain form)
agrees with the oracle's (closed-form integrals + information form)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1802_01070_amd import _lib, synth
from paper_1802_01070_amd.synth import Grid, MLPModel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "pct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pct_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def plan_for(grid, mlp):
    h = C.c_void_p()
    st = _lib.lib().pct_plan_create(C.byref(_lib.make_grid(grid)), C.byref(_lib.make_mlp(mlp)), C.byref(h))
    return st, h


def table_of(h):
    k = C.c_int32()
    assert _lib.lib().pct_plan_segments(h, C.byref(k)) == 0
    tab = np.zeros((k.value + 1) * 4)
    assert _lib.lib().pct_plan_table(h, tab.ctypes.data_as(C.POINTER(C.c_double)), tab.size) == 0
    return tab.reshape(-1, 4)


@pytest.mark.parametrize("cfg", [1, 2, 3, "tiny"])
def test_library_table_matches_oracle(cfg):
    c = synth.WORKLOADS[cfg]
    st, h = plan_for(c.grid, c.mlp)
    assert st == 0
    got = table_of(h)
    ref = oracle.mlp_table(c.mlp)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got[:, 0], ref[:, 0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(got[:, 2], ref[:, 2], rtol=0, atol=1e-13)
    np.testing.assert_allclose(got[:, 1], ref[:, 1], rtol=0, atol=1e-11)
    np.testing.assert_allclose(got[:, 3], ref[:, 3], rtol=0, atol=1e-11)
    _lib.lib().pct_plan_destroy(h)


def test_library_table_odd_step_and_no_log_term():
    for mlp in (MLPModel(u_in=-30, u_out=29.3, step=0.7), MLPModel(u_in=-100, u_out=100, log_term=0)):
        st, h = plan_for(Grid(8, 8, 2), mlp)
        assert st == 0
        np.testing.assert_allclose(table_of(h), oracle.mlp_table(mlp), rtol=0, atol=1e-11)
        _lib.lib().pct_plan_destroy(h)


@pytest.mark.parametrize("bad", [
    dict(grid=Grid(0, 8, 2)),
    dict(grid=Grid(8, 8, 2, pitch=(1.0, -1.0, 1.0))),
    dict(grid=Grid(8, 8, 2, pitch=(1.0, float("nan"), 1.0))),
    dict(grid=Grid(2048, 2048, 1024)),
    dict(mlp=MLPModel(u_in=5, u_out=5)),
    dict(mlp=MLPModel(u_in=-5, u_out=5, step=0.0)),
    dict(mlp=MLPModel(u_in=-5, u_out=5, E0=-1.0)),
    dict(mlp=MLPModel(u_in=-5, u_out=5, X0=0.0)),
    dict(mlp=MLPModel(u_in=-5, u_out=5, log_term=2)),
    dict(mlp=MLPModel(u_in=-1e9, u_out=1e9, step=1.0)),
    dict(mlp=MLPModel(u_in=-5, u_out=5, poly=(-1.0, 0, 0, 0, 0, 0))),  # negative scattering power
])
def test_plan_create_rejects(bad):
    grid = bad.get("grid", Grid(8, 8, 2))
    mlp = bad.get("mlp", MLPModel(u_in=-5, u_out=5))
    st, h = plan_for(grid, mlp)
    assert st == -1
    assert h.value is None


def test_plan_create_null_args():
    L = _lib.lib()
    g = _lib.make_grid(Grid(8, 8, 2))
    assert L.pct_plan_create(None, None, None) == -1
    assert L.pct_plan_create(C.byref(g), None, C.byref(C.c_void_p())) == -1


@pytest.fixture
def plan():
    st, h = plan_for(Grid(8, 8, 2), MLPModel(u_in=-5, u_out=5))
    assert st == 0
    yield h
    _lib.lib().pct_plan_destroy(h)


def fake_protons(n):
    # non-null dummies: validation never dereferences them
    return _lib.make_protons({k: 0x1000 + 64 * i for i, k in enumerate(_lib.FIELDS)}, n)


FAKE_WS = C.c_void_p(0x7F0000000000)  # 256-aligned, never uploaded


def ws_size(h, dtype=0):
    b = C.c_size_t()
    assert _lib.lib().pct_workspace_size(h, 100, dtype, C.byref(b)) == 0
    return b.value


def test_workspace_size_rules(plan):
    L = _lib.lib()
    b = C.c_size_t()
    assert L.pct_workspace_size(plan, -1, 0, C.byref(b)) == -1
    assert L.pct_workspace_size(plan, 10, 7, C.byref(b)) == -1
    assert ws_size(plan, 0) == ws_size(plan, 1)
    assert ws_size(plan) >= 128 * 8 + 128 * 4 * 2


def test_compute_calls_validate_before_device(plan):
    L = _lib.lib()
    p = fake_protons(100)
    nb = ws_size(plan)
    stream = None
    # workspace missing / too small / misaligned / not uploaded
    assert L.pct_forward(plan, C.byref(p), C.c_void_p(0x2000), 0, C.c_void_p(0x3000), None, None, nb, stream) == -2
    assert L.pct_forward(plan, C.byref(p), C.c_void_p(0x2000), 0, C.c_void_p(0x3000), None, FAKE_WS, 16, stream) == -2
    assert L.pct_forward(plan, C.byref(p), C.c_void_p(0x2000), 0, C.c_void_p(0x3000), None,
                         C.c_void_p(0x7F0000000010), nb, stream) == -2
    assert L.pct_forward(plan, C.byref(p), C.c_void_p(0x2000), 0, C.c_void_p(0x3000), None, FAKE_WS, nb, stream) == -2
    # bad dtype, null x, negative n
    assert L.pct_forward(plan, C.byref(p), C.c_void_p(0x2000), 5, C.c_void_p(0x3000), None, FAKE_WS, nb, stream) == -1
    assert L.pct_forward(plan, C.byref(p), None, 0, C.c_void_p(0x3000), None, FAKE_WS, nb, stream) == -1
    neg = fake_protons(-1)
    assert L.pct_backproject(plan, C.byref(neg), C.c_void_p(1), 0, C.c_void_p(1), FAKE_WS, nb, stream) == -1
    nullp = _lib.make_protons({k: 0 for k in _lib.FIELDS}, 10)
    assert L.pct_backproject(plan, C.byref(nullp), C.c_void_p(1), 0, C.c_void_p(1), FAKE_WS, nb, stream) == -1
    # trace ranges
    tr = L.pct_mlp_trace
    v = C.c_void_p(0x4000)
    assert tr(plan, C.byref(p), 90, 20, 64, v, v, v, FAKE_WS, nb, stream) == -1     # past the end
    assert tr(plan, C.byref(p), -1, 5, 64, v, v, v, FAKE_WS, nb, stream) == -1
    assert tr(plan, C.byref(p), 0, 5, 0, v, v, v, FAKE_WS, nb, stream) == -1        # max_nnz
    assert tr(plan, C.byref(p), 0, 5, 64, None, v, v, FAKE_WS, nb, stream) == -1
    assert tr(plan, C.byref(p), 0, 5, 64, v, v, v, FAKE_WS, nb, stream) == -2       # not uploaded


@pytest.mark.parametrize("field,value", [("block", 0), ("lambda_", 0.0), ("lambda_", float("inf")), ("n_iter", -1),
                                         ("dtype", 3), ("chord", 9), ("flags", 0x200), ("block_begin", -1),
                                         ("block_end", 2), ("block_begin", 3), ("lanes", 2), ("lanes", 128), ("block", 1 << 19),
                                         ("reserved", 1)])
def test_drop_options_validated(plan, field, value):
    L = _lib.lib()
    p = fake_protons(100)
    o = _lib.make_opts(64, 0.1, 1, 0)     # T = 2 blocks
    setattr(o, field, value)
    if field == "block_begin" and value == 3:
        o.block_end = 1
    if field == "block_end":
        o.block_end = 3
    st = L.pct_drop_iterate(plan, C.byref(p), C.c_void_p(0x5000), C.c_void_p(0x6000), C.byref(o), FAKE_WS,
                            ws_size(plan), None)
    assert st == -1, (field, value, st)


def test_drop_valid_options_reach_workspace_check(plan):
    L = _lib.lib()
    p = fake_protons(100)
    for flags in (0, _lib.PCT_DROP_CANCELLABLE, _lib.PCT_DROP_CANCELLABLE | _lib.PCT_DROP_NO_COMPENSATION,
                  _lib.PCT_DROP_DETERMINISTIC):
        for dtype in (0, 1):
            o = _lib.make_opts(64, 0.1, 1, dtype, flags=flags)
            st = L.pct_drop_iterate(plan, C.byref(p), C.c_void_p(0x5000), C.c_void_p(0x6000), C.byref(o), FAKE_WS,
                                    ws_size(plan), None)
            assert st == -2, (flags, dtype)


def test_deterministic_fp64_limits_the_block(plan):
    # the integer block sums hold blocks below 2^19 rows (FP64 otherwise allows 2^31)
    L = _lib.lib()
    p = fake_protons(1 << 20)
    for flags, want in ((0, -2), (_lib.PCT_DROP_DETERMINISTIC, -1)):
        o = _lib.make_opts(1 << 19, 0.1, 1, 1, flags=flags)
        st = L.pct_drop_iterate(plan, C.byref(p), C.c_void_p(0x5000), C.c_void_p(0x6000), C.byref(o), FAKE_WS,
                                ws_size(plan), None)
        assert st == want, flags


def test_drop_cancel_and_progress_validation(plan):
    L = _lib.lib()
    nb = ws_size(plan)
    done = C.c_int64(-5)
    assert L.pct_drop_cancel(None, FAKE_WS, nb, 1) == -1
    assert L.pct_drop_cancel(plan, None, nb, 1) == -1
    assert L.pct_drop_cancel(plan, FAKE_WS, nb, 1) == -2        # not uploaded: nothing written
    assert L.pct_drop_cancel(plan, FAKE_WS, 16, 0) == -2        # too small
    assert L.pct_drop_progress(None, FAKE_WS, nb, C.byref(done), None) == -1
    assert L.pct_drop_progress(plan, None, nb, C.byref(done), None) == -1
    assert L.pct_drop_progress(plan, FAKE_WS, nb, None, None) == -1
    assert L.pct_drop_progress(plan, FAKE_WS, nb, C.byref(done), None) == -2
    assert done.value == -5
    assert L.pct_status_string(-8) == b"stopped on a cancel request"


def test_tv_validation(plan):
    L = _lib.lib()
    nb = ws_size(plan)
    assert L.pct_tv(plan, None, 0, 1e-3, C.c_void_p(8), None, FAKE_WS, nb, None) == -1
    assert L.pct_tv(plan, C.c_void_p(8), 0, 0.0, C.c_void_p(8), None, FAKE_WS, nb, None) == -1
    assert L.pct_tv(plan, C.c_void_p(8), 3, 1e-3, C.c_void_p(8), None, FAKE_WS, nb, None) == -1
    assert L.pct_tv(plan, C.c_void_p(8), 0, 1e-3, C.c_void_p(8), None, FAKE_WS, nb, None) == -2
    # the variant without a workspace validates the same arguments (no launch here)
    assert L.pct_tv_static(None, C.c_void_p(8), 0, 1e-3, C.c_void_p(8), None, None) == -1
    assert L.pct_tv_static(plan, None, 0, 1e-3, C.c_void_p(8), None, None) == -1
    assert L.pct_tv_static(plan, C.c_void_p(8), 0, 0.0, C.c_void_p(8), None, None) == -1
    assert L.pct_tv_static(plan, C.c_void_p(8), 3, 1e-3, C.c_void_p(8), None, None) == -1
    assert L.pct_tv_static(plan, C.c_void_p(8), 0, 1e-3, None, None, None) == -1


def test_region_layout_matches_the_papers_example():
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "alg1_two_regions_20_slices.json")))
    from paper_1802_01070_amd import api
    lay = api.pct_region_layout(g["nz"], g["n_regions"], g["overlap"] // 2)
    assert [[a, b] for a, b, _, _ in lay] == g["regions"]
    assert [[c, d] for _, _, c, d in lay] == g["owned"]
    from oracle import regions
    for args in ((20, 2, 3), (32, 4, 2), (7, 7, 0), (33, 5, 40), (64, 3, 9)):
        assert api.pct_region_layout(*args) == regions.layout(*args)
    L = _lib.lib()
    a = (C.c_int32 * 4)()
    for bad in ((0, 1, 0), (5, 0, 0), (5, 6, 0), (5, 2, -1)):
        assert L.pct_region_layout(*bad, a, a, a, a) == -1
    assert L.pct_region_layout(5, 1, 0, None, a, a, a) == -1


def test_plan_region_and_region_calls_validate(plan):
    L = _lib.lib()
    h = C.c_void_p()
    assert L.pct_plan_region(plan, -1, 1, C.byref(h)) == -1
    assert L.pct_plan_region(plan, 1, 0, C.byref(h)) == -1
    assert L.pct_plan_region(plan, 0, 2, C.byref(h)) == -1          # the fixture grid has nz = 2
    assert L.pct_plan_region(plan, 1, 1, C.byref(h)) == 0
    np.testing.assert_array_equal(table_of(h), table_of(plan))     # same MLP model
    L.pct_plan_destroy(h)
    p = fake_protons(100)
    nb = ws_size(plan)
    buf = _lib.make_protons_buf({k: 0x9000 + 64 * i for i, k in enumerate(_lib.FIELDS)}, 100)
    cnt = C.c_void_p(0xA000)
    sel = L.pct_region_select
    assert sel(plan, C.byref(p), None, 1, 0, C.byref(buf), None, cnt, FAKE_WS, nb, None) == -1
    assert sel(plan, C.byref(p), None, 0, 2, C.byref(buf), None, cnt, FAKE_WS, nb, None) == -1
    assert sel(plan, C.byref(p), None, 0, 1, C.byref(buf), None, None, FAKE_WS, nb, None) == -1
    assert sel(plan, C.byref(p), C.c_void_p(0xB000), 0, 1, C.byref(buf), None, cnt, FAKE_WS, nb, None) == -1
    assert sel(plan, C.byref(p), None, 0, 1, C.byref(buf), None, cnt, FAKE_WS, nb, None) == -2   # not uploaded
    ss = L.pct_select_slices
    v = C.c_void_p(0xC000)
    assert ss(plan, v, 0, v, 0, 0, 3, 0, None) == -1                 # past nz
    assert ss(plan, v, 1, v, 0, 0, 1, 0, None) == -1                 # src starts after z_first
    assert ss(plan, v, 0, v, 0, 0, 1, 4, None) == -1                 # dtype
    assert ss(plan, None, 0, v, 0, 0, 1, 0, None) == -1
    assert ss(plan, v, 0, v, 0, 1, 0, 0, None) == 0                  # nothing to copy


def test_stored_row_calls_validate(plan):
    L = _lib.lib()
    p = fake_protons(100)
    nb = ws_size(plan)
    v = C.c_void_p(0xD000)
    assert L.pct_rows_count(plan, C.byref(p), None, FAKE_WS, nb, None) == -1
    assert L.pct_rows_count(plan, C.byref(p), v, FAKE_WS, nb, None) == -2            # not uploaded
    assert L.pct_rows_build(plan, C.byref(p), 0, v, v, v, v, FAKE_WS, nb, None) == -1  # FP64 chords are not stored
    assert L.pct_rows_build(plan, C.byref(p), 2, None, v, v, v, FAKE_WS, nb, None) == -1
    assert L.pct_rows_build(plan, C.byref(p), 2, v, v, v, v, FAKE_WS, nb, None) == -2
    rows = _lib.pct_rows(0xE000, 0xE100, 0xE200, 0xE300, 100, 2, 0)
    ok = _lib.make_opts(64, 0.1, 1, 0, chord="f16")
    run = L.pct_drop_iterate_rows
    assert run(plan, C.byref(rows), v, v, C.byref(ok), FAKE_WS, nb, None) == -2       # valid up to the workspace
    for field, value in (("chord", 1), ("lanes", 8), ("block", 0), ("reserved", 1), ("flags", 0x20),
                         ("block_end", 3)):
        o = _lib.make_opts(64, 0.1, 1, 0, chord="f16")
        setattr(o, field, value)
        assert run(plan, C.byref(rows), v, v, C.byref(o), FAKE_WS, nb, None) == -1, field
    for field, value in (("dtype", 1), ("flags", 0x8), ("flags", _lib.PCT_DROP_CANCELLABLE)):
        o = _lib.make_opts(64, 0.1, 1, 0, chord="f16")
        setattr(o, field, value)
        assert run(plan, C.byref(rows), v, v, C.byref(o), FAKE_WS, nb, None) == -7, field
    bad = _lib.pct_rows(0xE000, 0xE100, 0xE200, 0xE300, 100, 0, 0)                    # FP64 stored chords
    assert run(plan, C.byref(bad), v, v, C.byref(ok), FAKE_WS, nb, None) == -1
    bad = _lib.pct_rows(0xE000, 0, 0xE200, 0xE300, 100, 2, 0)
    assert run(plan, C.byref(bad), v, v, C.byref(ok), FAKE_WS, nb, None) == -1
    assert run(plan, C.byref(rows), None, v, C.byref(ok), FAKE_WS, nb, None) == -1


def test_order_blocks_validates(plan):
    L = _lib.lib()
    p = fake_protons(100)
    buf = _lib.make_protons_buf({k: 0x9000 + 64 * i for i, k in enumerate(_lib.FIELDS)}, 100)
    small = _lib.make_protons_buf({k: 0x9000 + 64 * i for i, k in enumerate(_lib.FIELDS)}, 99)
    v = C.c_void_p(0xA000)
    assert L.pct_order_blocks(plan, C.byref(p), None, 0, C.byref(buf), None, None) == -1
    assert L.pct_order_blocks(plan, C.byref(p), None, 8193, C.byref(buf), None, None) == -1
    assert L.pct_order_blocks(plan, C.byref(p), None, 64, C.byref(small), None, None) == -1
    assert L.pct_order_blocks(plan, C.byref(p), v, 64, C.byref(buf), None, None) == -1     # b without b_out
    assert L.pct_order_blocks(plan, C.byref(p), None, 64, None, None, None) == -1


def test_header_compiles_as_c():
    import subprocess
    r = subprocess.run(["gcc", "-fsyntax-only", "-std=c11", "-Wall", "-Werror", "-x", "c",
                        os.path.join(ROOT, "include", "pct.h")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_status_strings():
    for st in range(-7, 1):
        s = _lib.status_string(st)
        assert s and s != "unknown status"
    assert _lib.status_string(-99) == "unknown status"


def test_library_has_no_oracle_dependency():
    # the product library must not link, load or name the oracle
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"orc_" not in data and b"liborc" not in data


def test_fbp_calls_validate(plan):
    # plan: 8 x 8 x 2 grid.  Every call below fails validation on the host, so
    # nothing is launched.
    L = _lib.lib()
    G = _lib.pct_fbp_geom
    good = G(12, 16, -8.0, 1.0)
    nb = 2 * 12 * 16
    sz = C.c_size_t()
    assert L.pct_fbp_workspace_size(plan, C.byref(good), C.byref(sz)) == 0
    align = lambda v: (v + 255) // 256 * 256
    assert sz.value == align(8 * nb) + align(4 * nb) + 2 * align(8 * nb)
    for bad in (G(0, 16, -8.0, 1.0), G(4097, 16, -8.0, 1.0), G(12, 0, -8.0, 1.0), G(12, 4097, -8.0, 1.0),
                G(12, 16, float("nan"), 1.0), G(12, 16, -8.0, 0.0), G(12, 16, -8.0, -1.0),
                G(12, 16, -8.0, float("inf"))):
        assert L.pct_fbp_workspace_size(plan, C.byref(bad), C.byref(sz)) == -1
        assert L.pct_fbp_filter(plan, C.byref(bad), C.c_void_p(0x10000), C.c_void_p(0x20000), None) == -1
    assert L.pct_fbp_workspace_size(plan, None, C.byref(sz)) == -1
    assert L.pct_fbp_workspace_size(plan, C.byref(good), None) == -1
    p = fake_protons(100)
    b = C.c_void_p(0x8000)
    x = C.c_void_p(0x40000000)
    ws = C.c_void_p(0x7F0000000000)
    wsb = align(8 * nb) + align(4 * nb) + 2 * align(8 * nb)
    # workspace missing, too small, misaligned
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), b, x, 0, None, wsb, None) == -2
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), b, x, 0, ws, wsb - 1, None) == -2
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), b, x, 0, C.c_void_p(0x7F0000000010), wsb, None) == -2
    # x inside the workspace, bad dtype, missing b or x
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), b, C.c_void_p(0x7F0000000100), 0, ws, wsb, None) == -1
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), b, x, 7, ws, wsb, None) == -1
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), None, x, 0, ws, wsb, None) == -1
    assert L.pct_fbp(plan, C.byref(good), C.byref(p), b, None, 0, ws, wsb, None) == -1
    # sinogram: output overlapping the sums, workspace without its sum and count parts
    assert L.pct_fbp_sinogram(plan, C.byref(good), C.byref(p), b, ws, None, ws, wsb, None) == -1
    assert L.pct_fbp_sinogram(plan, C.byref(good), C.byref(p), b, x, None, ws, align(8 * nb), None) == -2
    assert L.pct_fbp_sinogram(plan, C.byref(good), C.byref(p), b, None, None, ws, wsb, None) == -1
    # filter in place, back-projection onto its own input
    assert L.pct_fbp_filter(plan, C.byref(good), x, C.c_void_p(0x40000000 + 8), None) == -1
    assert L.pct_fbp_backproject(plan, C.byref(good), x, C.c_void_p(0x40000000 + 64), 0, None) == -1
    assert L.pct_fbp_backproject(plan, C.byref(good), x, C.c_void_p(0x50000000), 2, None) == -1
    # too many bins for a 32-bit bin index
    big = G(4096, 4096, -8.0, 1.0)
    st, h = plan_for(Grid(8, 8, 200), MLPModel(u_in=-5, u_out=5))
    assert st == 0
    assert L.pct_fbp_workspace_size(h, C.byref(big), C.byref(sz)) == -1
    L.pct_plan_destroy(h)


def test_sort_scan_validates(plan):
    # plan: 8 x 8 x 2 grid of 1 mm voxels.  Every call below fails validation
    # on the host, so nothing is launched.
    L = _lib.lib()
    O = _lib.pct_sort_opts
    sz = C.c_size_t()
    align = lambda v: (v + 255) // 256 * 256
    assert L.pct_sort_scan_workspace_size(100, C.byref(sz)) == 0
    full = 2 * align(800) + 2 * align(400) + align(4 * 256) + align(4) + align(4000)
    assert sz.value == full
    assert L.pct_sort_scan_workspace_size(0, C.byref(sz)) == 0 and sz.value == 0
    assert L.pct_sort_scan_workspace_size(-1, C.byref(sz)) == -1
    assert L.pct_sort_scan_workspace_size(1 << 31, C.byref(sz)) == -1
    assert L.pct_sort_scan_workspace_size(100, None) == -1
    p = fake_protons(100)
    buf = _lib.make_protons_buf({k: 0x9000 + 64 * i for i, k in enumerate(_lib.FIELDS)}, 100)
    small = _lib.make_protons_buf({k: 0x9000 + 64 * i for i, k in enumerate(_lib.FIELDS)}, 99)
    ws = C.c_void_p(0x7F0000000000)
    wsb = full
    good = O(90, 0, 0.5)
    for bad in (O(0, 0, 0.5), O(4097, 0, 0.5), O(90, 1, 0.5), O(90, 0, 0.0), O(90, 0, -1.0), O(90, 0, float("nan")),
                O(90, 0, float("inf")), O(90, 0, 2.0 / 4097)):
        assert L.pct_sort_scan(plan, C.byref(p), None, C.byref(bad), C.byref(buf), None, None, ws, wsb, None) == -1
    assert L.pct_sort_scan(plan, C.byref(p), None, None, C.byref(buf), None, None, ws, wsb, None) == -1
    assert L.pct_sort_scan(None, C.byref(p), None, C.byref(good), C.byref(buf), None, None, ws, wsb, None) == -1
    assert L.pct_sort_scan(plan, C.byref(p), None, C.byref(good), None, None, None, ws, wsb, None) == -1
    assert L.pct_sort_scan(plan, C.byref(p), None, C.byref(good), C.byref(small), None, None, ws, wsb, None) == -1
    assert L.pct_sort_scan(plan, C.byref(p), C.c_void_p(0xA000), C.byref(good), C.byref(buf), None, None, ws, wsb,
                           None) == -1                                                         # b without b_out
    # workspace missing, too small, misaligned
    assert L.pct_sort_scan(plan, C.byref(p), None, C.byref(good), C.byref(buf), None, None, None, wsb, None) == -2
    assert L.pct_sort_scan(plan, C.byref(p), None, C.byref(good), C.byref(buf), None, None, ws, wsb - 1, None) == -2
    assert L.pct_sort_scan(plan, C.byref(p), None, C.byref(good), C.byref(buf), None, None,
                           C.c_void_p(0x7F0000000010), wsb, None) == -2
    # too many records
    big = fake_protons(1 << 31)
    assert L.pct_sort_scan(plan, C.byref(big), None, C.byref(good), C.byref(buf), None, None, ws, wsb, None) == -1

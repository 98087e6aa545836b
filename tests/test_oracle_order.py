"""Pins of the angle-bin ordering oracle (continuous-rotation scans, Section
IV-A): a hand-worked example, the special case that reduces to a stable
argsort, the order of the input generator's sorted scans, and the sortedness
and stability invariants on inputs full of ties."""
import numpy as np
import pytest

from oracle import order as O
from paper_1802_01070_amd import synth


def records(rows):
    """rows of (gantry, v_in, t_in); the other fields carry the row number so
    that a permutation of them is visible."""
    arr = np.asarray(rows, dtype=np.float64)
    n = len(arr)
    pos = np.arange(n, dtype=np.float64)
    pr = {k: pos.astype(np.float32) for k in synth.FIELDS}
    pr["gantry"] = arr[:, 0].astype(np.float32)
    pr["v_in"] = arr[:, 1].astype(np.float32)
    pr["t_in"] = arr[:, 2].astype(np.float32)
    return pr


def test_hand_worked_example():
    # 4 x 4 x 4 grid, 4 mm slices: z in [-8, 8), slabs of 4 mm -> 4 slabs;
    # 4 angle bins of pi/2 centred on 0, pi/2, pi, 3 pi/2
    grid = synth.Grid(4, 4, 4, pitch=(1.0, 1.0, 4.0))
    rows = [
        (3.0, -7.0, 1.0),            # 0: 3.0 / (pi/2) = 1.91 -> bin 2; slab 0
        (0.1, 5.0, 0.0),             # 1: bin 0; slab 3
        (6.2, -3.9, -2.0),           # 2: 3.95 + 1/2 -> 4, wraps to bin 0; slab 1
        (-1.0, 100.0, 0.5),          # 3: -0.64 + 1/2 -> -1, wraps to bin 3; above the grid: slab 3
        (0.7, -3.9, -2.0),           # 4: 0.45 + 1/2 -> bin 0; slab 1; ties with 2 and stays after it
        (0.9, -100.0, 3.0),          # 5: 0.57 + 1/2 -> bin 1; below the grid: slab 0
        (np.nan, 0.0, 0.0),          # 6: not finite: last
        (0.1, 5.0, -0.0),            # 7: same key as 1 (-0 = +0): after 1
        (1.0, 0.0, -5.0),            # 8: bin 1; v on the slab edge 0 -> slab 2
        (0.2, np.inf, 0.0),          # 9: not finite: last, after 6
        (0.2, -3.9, -3.0),           # 10: bin 0, slab 1, before 2 and 4
        (1e30, -7.0, 7.0),           # 11: a huge multiple of 4 bins -> bin 0; slab 0
        (-0.0, -8.0, 2.0),           # 12: bin 0; the grid's lower edge -> slab 0
        (np.pi / 4, 3.999, 1.0),     # 13: FP32 pi/4 is above pi/4: bin 1; slab 2
    ]
    pr = records(rows)
    a, s, t, bad = O.keys(grid, pr, 4, 4.0)
    assert a.tolist() == [2, 0, 0, 3, 0, 1, 4, 0, 1, 4, 0, 0, 0, 1]
    assert s.tolist() == [0, 3, 1, 3, 1, 0, 0, 3, 2, 0, 1, 0, 0, 2]
    assert O.n_slabs(grid, 4.0) == 4
    perm = O.order(grid, pr, 4, 4.0)
    assert perm.tolist() == [12, 11, 10, 2, 4, 1, 7, 5, 8, 13, 0, 3, 6, 9]
    out, _, _ = O.sort_scan(grid, pr, None, 4, 4.0)
    assert out["th_out"].tolist() == [float(i) for i in perm]


def test_one_bin_one_slab_is_a_stable_argsort():
    rng = np.random.default_rng(3)
    grid = synth.Grid(8, 8, 8)
    n = 5000
    t = rng.integers(-40, 40, n).astype(np.float32) * 0.5      # many ties
    t[::7] = -0.0
    rows = np.stack([rng.uniform(-0.1, 0.1, n), rng.uniform(-4, 4, n), t], axis=1)
    pr = records(rows)
    perm = O.order(grid, pr, 16, 1000.0)                           # one slab covers the grid
    assert np.array_equal(perm, np.argsort(t.astype(np.float64) + 0.0, kind="stable"))
    assert perm.tolist() == sorted(range(n), key=lambda i: float(t[i]) + 0.0)   # Python's sort is stable


@pytest.mark.parametrize("key", [3])
def test_reproduces_the_generators_sorted_scan(key):
    # fixed-angle scans from the generator are sorted by angle, 4 mm slab of
    # v_in and t_in; sorting a shuffled copy gives the same record sequence
    cfg = synth.WORKLOADS[key]
    assert cfg.order == "angle_slab" and not cfg.continuous_angles
    sc = synth.make_scan(cfg, m=20000, with_b=False)
    perm = np.random.default_rng(5).permutation(sc.m)
    shuffled = {k: v[perm] for k, v in sc.protons.items()}
    out, _, _ = O.sort_scan(sc.grid, shuffled, None, cfg.n_angles, cfg.slab_mm)
    for k in synth.FIELDS:
        assert np.array_equal(out[k], sc.protons[k]), k


def test_sorted_and_stable_with_ties_and_edge_records():
    rng = np.random.default_rng(11)
    grid = synth.Grid(10, 10, 20, pitch=(1.0, 1.0, 1.5))
    n = 20000
    phi = rng.integers(-3, 40, n) * (2 * np.pi / 36) + rng.choice([0.0, 0.04, -0.04], n)
    v = rng.integers(-20, 20, n) * 1.0
    t = rng.integers(-5, 5, n) * 1.0
    phi[::101] = np.nan
    v[3::211] = -np.inf
    t[5::307] = np.inf
    pr = records(np.stack([phi, v, t], axis=1))
    n_ang, slab = 36, 2.5
    perm = O.order(grid, pr, n_ang, slab)
    assert np.array_equal(np.sort(perm), np.arange(n))
    # keys written out with Python's math module, record by record
    import math
    ns = math.ceil(20 * 1.5 / slab)

    def key(i):
        f = [float(pr["gantry"][i]), float(pr["v_in"][i]), float(pr["t_in"][i])]
        if not all(math.isfinite(x) for x in f):
            return (n_ang, 0, 0.0)
        a = int(math.floor(f[0] / (2 * math.pi / n_ang) + 0.5)) % n_ang
        s = min(max(int(math.floor((f[1] + 15.0) / slab)), 0), ns - 1)
        return (a, s, f[2] + 0.0)

    ks = [key(int(i)) for i in perm]
    for j in range(1, n):
        assert ks[j - 1] < ks[j] or (ks[j - 1] == ks[j] and perm[j - 1] < perm[j]), j


@pytest.mark.parametrize("mistake", ["no_wrap", "truncate", "no_half", "no_clamp", "bins_by_degrees"])
def test_hand_example_catches_planted_mistakes(mistake, monkeypatch):
    # each plausible slip in the angle or slab formula, planted in the oracle
    # (through the numpy functions it calls, restored after the test),
    # changes the hand-worked bins or order
    grid = synth.Grid(4, 4, 4, pitch=(1.0, 1.0, 4.0))
    rows = [(3.0, -7.0, 1.0), (0.1, 5.0, 0.0), (6.2, -3.9, -2.0), (-1.0, 100.0, 0.5), (0.7, -3.9, -2.0),
            (0.9, -100.0, 3.0), (np.nan, 0.0, 0.0), (0.1, 5.0, -0.0), (1.0, 0.0, -5.0), (0.2, np.inf, 0.0),
            (0.2, -3.9, -3.0), (1e30, -7.0, 7.0), (-0.0, -8.0, 2.0), (np.pi / 4, 3.999, 1.0)]
    pr = records(rows)
    expected = ([2, 0, 0, 3, 0, 1, 4, 0, 1, 4, 0, 0, 0, 1], [0, 3, 1, 3, 1, 0, 0, 3, 2, 0, 1, 0, 0, 2],
                [12, 11, 10, 2, 4, 1, 7, 5, 8, 13, 0, 3, 6, 9])
    real_floor = np.floor
    if mistake == "no_wrap":                      # angle bin not taken modulo the turn
        monkeypatch.setattr(O.np, "mod", lambda a, n: a)
    elif mistake == "truncate":                   # rounding toward zero instead of down
        monkeypatch.setattr(O.np, "floor", np.trunc)
    elif mistake == "no_half":                    # bins with edges, not centres, at multiples of dphi
        calls = {"k": 0}

        def floor_without_half(x):
            calls["k"] += 1
            return real_floor(x - 0.5) if calls["k"] == 1 else real_floor(x)
        monkeypatch.setattr(O.np, "floor", floor_without_half)
    elif mistake == "no_clamp":                   # heights outside the grid not clamped to its slabs
        monkeypatch.setattr(O.np, "clip", lambda a, lo, hi: a)
    elif mistake == "bins_by_degrees":            # angles taken as degrees
        monkeypatch.setattr(O.np, "pi", 180.0)
    with np.errstate(all="ignore"):
        a, s_, _, _ = O.keys(grid, pr, 4, 4.0)
        got = (a.tolist(), s_.tolist(), O.order(grid, pr, 4, 4.0).tolist())
    assert got != expected

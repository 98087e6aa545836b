"""GPU parity of the FBP initial iterate (Section I) against the FP64 oracle:
bin counts bit-exact, bin means, the ramp filter and the back-projection to
FP64 rounding, the whole chain at full size on sampled voxels, edge cases, and
DROP started from the FBP image."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import fbp as ofbp
from paper_1802_01070_amd import api, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_scans = {}


def scan(cfg, m=None):
    if (cfg, m) not in _scans:
        _scans[(cfg, m)] = synth.make_scan(synth.WORKLOADS[cfg], m=m)
    return _scans[(cfg, m)]


def geom_of(sc, n_ang):
    return api.FbpGeom.for_grid(sc.grid, n_ang)


def image_tol(geo, ref):
    """Bound on |x - x_oracle| for an image made from the library's own
    sinogram: each b is summed in 2^-24 mm fixed point (error <= 2^-25 mm, so
    a bin mean is off by at most that), the ramp filter's gain is
    dt sum_m |h(m)| = 1 / (2 dt) and the back-projection's pi; plus FP64
    rounding."""
    return np.pi / (2.0 * geo.dt) * 2.0 ** -25 + 1e-11 * max(1.0, np.abs(ref).max())


# (cfg, protons, angle bins, shuffled): angle-sorted scans take the LDS-privatised
# binning where one angle's bins fit in LDS (the 256 x 256 x 64 grid's do not);
# a shuffled scan sends almost every proton to the global bins
@pytest.mark.parametrize("cfg,m,n_ang,shuffle", [(1, 200000, 90, False), (2, 2000000, 180, False),
                                                 ("cont", 1000000, 180, False), (1, 50000, 7, False),
                                                 (3, 1000000, 360, False), (2, 1000000, 180, True)])
def test_sinogram_matches_oracle(cfg, m, n_ang, shuffle):
    sc = scan(cfg, m)
    g = geom_of(sc, n_ang)
    say(f"fbp sinogram {sc.cfg.name} m={sc.m} geom={g} shuffled={shuffle}")
    prot, bb = sc.protons, sc.b
    if shuffle:
        perm = np.random.default_rng(4).permutation(sc.m)
        prot, bb = {k: v[perm] for k, v in prot.items()}, bb[perm]
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(prot, DEV)
    proj, cnt = api.pct_fbp_sinogram(plan, pr, torch.from_numpy(bb).to(DEV), g)
    rp, rc = ofbp.sinogram(sc.grid, sc.mlp, prot, bb, g.n_angles, g.n_t, g.t0, g.dt)
    assert np.array_equal(cnt.cpu().numpy(), rc)
    assert int(rc.sum()) > 0.9 * sc.m
    # 2^-24 mm fixed point of each b against the FP64 sum
    err = np.abs(proj.cpu().numpy() - rp)
    assert err.max() <= 1e-7 + 1e-12 * np.abs(rp).max()


def test_filter_and_backprojection_match_oracle():
    sc = scan(2, 1000000)
    g = geom_of(sc, 180)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    rp, _ = ofbp.sinogram(sc.grid, sc.mlp, sc.protons, sc.b, g.n_angles, g.n_t, g.t0, g.dt)
    rq = ofbp.filter_rows(rp, g.dt)
    q = api.pct_fbp_filter(plan, torch.from_numpy(rp).to(DEV), g)
    scale = np.abs(rq).max()
    assert np.abs(q.cpu().numpy() - rq).max() <= 1e-12 * scale
    # back-projection of the oracle's filtered rows, FP64 and FP32 images
    x64 = api.pct_fbp_backproject(plan, torch.from_numpy(rq).to(DEV), g, dtype=torch.float64).cpu().numpy()
    x32 = api.pct_fbp_backproject(plan, torch.from_numpy(rq).to(DEV), g, dtype=torch.float32).cpu().numpy()
    rng = np.random.default_rng(1)
    vox = np.unique(np.concatenate([rng.integers(0, sc.grid.nvox, 20000), np.arange(sc.grid.nx * sc.grid.ny)]))
    rx = ofbp.backproject(sc.grid, rq, g.n_angles, g.t0, g.dt, voxels=vox)
    s = max(1.0, np.abs(rx).max())
    assert np.abs(x64[vox] - rx).max() <= 1e-11 * s
    assert np.abs(x32[vox] - rx).max() <= 1e-6 * s


def test_full_size_fbp_on_sampled_voxels():
    sc = scan(2)                                   # 10^7 protons, 200 x 200 x 32
    g = geom_of(sc, 180)
    say(f"fbp full size m={sc.m}")
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    x = api.pct_fbp(plan, pr, torch.from_numpy(sc.b).to(DEV), g, dtype=torch.float32).cpu().numpy()
    rp, _ = ofbp.sinogram(sc.grid, sc.mlp, sc.protons, sc.b, g.n_angles, g.n_t, g.t0, g.dt)
    rq = ofbp.filter_rows(rp, g.dt)
    rng = np.random.default_rng(2)
    vox = rng.integers(0, sc.grid.nvox, 30000)
    rx = ofbp.backproject(sc.grid, rq, g.n_angles, g.t0, g.dt, voxels=vox)
    assert np.abs(x[vox] - rx).max() <= 1e-6 * max(1.0, np.abs(rx).max())
    # the image is an RSP map: water-like inside the phantom
    xt = sc.x_true()
    inside = xt[vox] > 0.5
    assert abs(np.median(x[vox][inside] / xt[vox][inside]) - 1.0) < 0.1


def test_edge_cases():
    sc = scan(1, 20000)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    # no protons: an all-zero image
    g = geom_of(sc, 90)
    empty = api.Protons({k: v[:0] for k, v in sc.protons.items()}, DEV)
    x = api.pct_fbp(plan, empty, b[:0], g, dtype=torch.float64)
    assert not x.any().item()
    # bins that see no proton (lateral range off to the side): zero image
    off = api.FbpGeom(90, 16, 500.0, 1.0)
    pr = api.Protons(sc.protons, DEV)
    x = api.pct_fbp(plan, pr, b, off, dtype=torch.float64)
    assert not x.any().item()
    # one angle bin, one lateral bin; non-finite records and b dropped as in the oracle
    prot = {k: v.copy() for k, v in sc.protons.items()}
    bb = sc.b.copy()
    prot["t_in"][::97] = np.nan
    prot["gantry"][5::89] = np.inf
    bb[7::83] = np.nan
    bb[9::101] = 3.0e6                  # beyond 2^20 mm: not a WEPL
    pr = api.Protons(prot, DEV)
    for geo in (api.FbpGeom(1, 1, -40.0, 80.0), api.FbpGeom(3, 5, -30.0, 7.0), geom_of(sc, 90)):
        p, c = api.pct_fbp_sinogram(plan, pr, torch.from_numpy(bb).to(DEV), geo)
        rp, rc = ofbp.sinogram(sc.grid, sc.mlp, prot, bb, geo.n_angles, geo.n_t, geo.t0, geo.dt)
        assert np.array_equal(c.cpu().numpy(), rc), geo
        assert np.abs(p.cpu().numpy() - rp).max() <= 1e-7 + 1e-12 * np.abs(rp).max()
        x = api.pct_fbp(plan, pr, torch.from_numpy(bb).to(DEV), geo, dtype=torch.float64).cpu().numpy()
        rx = ofbp.backproject(sc.grid, ofbp.filter_rows(rp, geo.dt), geo.n_angles, geo.t0, geo.dt)
        assert np.abs(x - rx).max() <= image_tol(geo, rx), geo


def test_ragged_grid():
    # nx * ny not a multiple of the workgroup, nz not a multiple of the 8 XCDs
    grid = synth.Grid(37, 23, 11, pitch=(1.5, 2.0, 1.0))
    mlp = synth.MLPModel(u_in=-40.0, u_out=40.0)
    rng = np.random.default_rng(9)
    n = 300000
    t = rng.uniform(-40, 40, n)
    v = rng.uniform(-6, 6, n)
    th = rng.normal(0, 0.01, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    prot = {k: a.astype(np.float32) for k, a in dict(t_in=t, v_in=v, th_in=th, ph_in=th, t_out=t + 80 * th,
                                                      v_out=v + 80 * th, th_out=th, ph_out=th, gantry=phi).items()}
    b = rng.uniform(0, 60, n).astype(np.float32)
    g = api.FbpGeom.for_grid(grid, 64, dt=0.75)
    plan = api.Plan(grid, mlp, DEV)
    x = api.pct_fbp(plan, api.Protons(prot, DEV), torch.from_numpy(b).to(DEV), g, dtype=torch.float64)
    rx = ofbp.fbp(grid, mlp, prot, b, g.n_angles, g.n_t, g.t0, g.dt)
    assert np.abs(x.cpu().numpy() - rx).max() <= image_tol(g, rx)


def test_drop_from_the_fbp_image_matches_oracle():
    oracle.build(force=False)
    c = synth.WORKLOADS[1]
    sc = scan(1, 40000)
    g = geom_of(sc, 90)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    x = api.pct_fbp(plan, pr, b, g, dtype=torch.float64)
    x0 = ofbp.fbp(sc.grid, sc.mlp, sc.protons, sc.b, g.n_angles, g.n_t, g.t0, g.dt)
    assert np.abs(x.cpu().numpy() - x0).max() <= image_tol(g, x0)
    ref = oracle.drop(sc.grid, sc.mlp, sc.protons, sc.b, x0, block=c.block, lam=c.lam, n_iter=2)
    # DROP from the oracle's FBP image: the solver alone
    xo = torch.from_numpy(x0).to(DEV)
    api.pct_drop_iterate(plan, pr, b, xo, block=c.block, lam=c.lam, n_iter=2)
    err = np.max(np.abs(xo.cpu().numpy() - ref) / np.maximum(np.abs(ref), 1.0))
    say(f"  DROP from the oracle's FBP image: {err:.3e}")
    assert err <= 1e-10
    # the chain: the image's fixed-point bound carries through the sweeps
    api.pct_drop_iterate(plan, pr, b, x, block=c.block, lam=c.lam, n_iter=2)
    err = np.abs(x.cpu().numpy() - ref).max()
    say(f"  FBP then DROP: {err:.3e}")
    assert err <= 2.0 * image_tol(g, ref) + 1e-10 * max(1.0, np.abs(ref).max())


def test_fbp_ignores_the_hull_and_follows_region_grids():
    # straight chords: a hull setting does not change the image; a region plan
    # bins v by its own slices (z origin moved up by z_lo slices)
    sc = scan(2, 400000)
    g = geom_of(sc, 180)
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    plain = api.Plan(sc.grid, sc.mlp, DEV)
    hull = api.Plan(sc.grid, sc.mlp, DEV).set_hull(92.0)
    x0 = api.pct_fbp(plain, pr, b, g, dtype=torch.float64)
    x1 = api.pct_fbp(hull, pr, b, g, dtype=torch.float64)
    assert torch.equal(x0, x1)
    reg = plain.region(10, 21)
    xr = api.pct_fbp(reg, pr, b, g, dtype=torch.float64).cpu().numpy()
    rx = ofbp.fbp(reg.grid, sc.mlp, sc.protons, sc.b, g.n_angles, g.n_t, g.t0, g.dt)
    assert np.abs(xr - rx).max() <= image_tol(g, rx)


# (grid, geometry): the tiled kernel with partial tiles, angles in several
# chunks, windows that run past either end of the rows, coarse bins, an
# off-centre grid, and angle sets whose sines, cosines and window starts take
# more than 8 KB of LDS; the untiled kernel for lateral bins much finer than
# the voxels, for a far-off t0 and for 4096 angles
_RAGGED = synth.Grid(37, 23, 11, pitch=(1.5, 2.0, 1.0))
_OFFSET = synth.Grid(40, 40, 3, origin=(30.0, -70.0, -1.5))


@pytest.mark.parametrize("grid,geo", [
    (_RAGGED, api.FbpGeom.for_grid(_RAGGED, 64, dt=0.75)),
    (_RAGGED, api.FbpGeom(64, 40, -10.0, 0.75)),
    (_RAGGED, api.FbpGeom(7, 5, -30.0, 7.0)),
    (_OFFSET, api.FbpGeom(32, 300, -150.0, 1.0)),
    (_RAGGED, api.FbpGeom.for_grid(_RAGGED, 400, dt=0.75)),
    (_RAGGED, api.FbpGeom.for_grid(_RAGGED, 600, dt=0.75)),
    (_RAGGED, api.FbpGeom.for_grid(_RAGGED, 4096, dt=0.75)),
    (_RAGGED, api.FbpGeom.for_grid(_RAGGED, 24, dt=0.05)),
    (_RAGGED, api.FbpGeom(16, 8, 1.0e12, 1.0)),
])
def test_backprojection_of_random_rows(grid, geo):
    rng = np.random.default_rng(geo.n_t)
    rq = rng.standard_normal((grid.nz, geo.n_angles, geo.n_t))
    say(f"back-projection: grid {grid.nx}x{grid.ny}x{grid.nz}, {geo}")
    plan = api.Plan(grid, synth.MLPModel(u_in=-60.0, u_out=60.0), DEV)
    q = torch.from_numpy(rq).to(DEV)
    x64 = api.pct_fbp_backproject(plan, q, geo, dtype=torch.float64).cpu().numpy()
    x32 = api.pct_fbp_backproject(plan, q, geo, dtype=torch.float32).cpu().numpy()
    rx = ofbp.backproject(grid, rq, geo.n_angles, geo.t0, geo.dt)
    s = max(1.0, np.abs(rx).max())
    assert np.abs(x64 - rx).max() <= 1e-12 * s
    assert np.abs(x32 - rx).max() <= 1e-6 * s
    if geo.t0 > 1e9:
        assert not rx.any() and not x64.any()
    else:
        assert np.count_nonzero(rx) > grid.nvox // 4


@pytest.mark.parametrize("n_t", [1, 2, 17, 37, 284, 4096])
def test_filter_of_random_rows(n_t):
    # rows shorter than one output group, ragged groups of both parities, and
    # rows long enough that one row fills a workgroup
    grid = synth.Grid(8, 8, 3)
    plan = api.Plan(grid, synth.MLPModel(u_in=-20.0, u_out=20.0), DEV)
    geo = api.FbpGeom(5, n_t, -0.5 * n_t * 0.7, 0.7)
    rp = np.random.default_rng(n_t).standard_normal((grid.nz, geo.n_angles, n_t))
    q = api.pct_fbp_filter(plan, torch.from_numpy(rp).to(DEV), geo).cpu().numpy()
    rq = ofbp.filter_rows(rp, geo.dt)
    assert np.abs(q - rq).max() <= 1e-12 * max(1.0, np.abs(rq).max())

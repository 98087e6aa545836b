"""Seeded synthetic proton-CT scans: phantoms, proton records and WEPL data.

This module is the single input generator that both the HIP path and the
CPU oracle consume.  It holds none of the reconstruction method's arithmetic:
no most-likely-path coefficients, no voxel walk, no DROP update.  It produces

* the voxel grid and the MLP model parameters (plain numbers that both sides
  take as inputs);
* an analytic phantom (cylinders / ellipsoid / spheres of constant relative
  stopping power) and its 4x4x4-supersampled voxelisation;
* per-proton tracker data (entry/exit lateral positions and slopes in the
  beam frame, gantry angle) and the WEPL vector ``b``.

The paper's CTP404 datasets (Geant4-simulated and scanner data, Section IV-A)
are not available; these scans stand in for them.  Their shape follows the
paper's acquisition (discrete projection angles over a full rotation, Section
IV-A) and the configurations listed in ``WORKLOADS``.

Physics stand-ins (not the reconstruction model):
* exit deflections use the Fermi-Eyges covariance of a constant scattering
  power ``T`` (rad^2/mm): cov(t, theta) = T [[D^3/3, D^2/2], [D^2/2, D]];
* WEPL is the exact line integral of the analytic phantom along a smooth
  stand-in for the proton's true path -- the cubic Hermite curve through the
  entry and exit positions with the entry and exit slopes, taken as
  ``WEPL_PIECES`` straight pieces -- clipped to the grid box, plus Gaussian
  noise (sigma = 1 mm).  (A straight entry-to-exit chord leaves the grid's z
  range at other depths than any curved path and makes the data markedly
  inconsistent near the top and bottom slices.)

Random draws: numpy ``Generator(PCG64)``, one ``SeedSequence(seed).spawn``
child per chunk of 10^6 protons, fixed draw order (t, v, theta, phi, two
normals for the t-plane, two for the v-plane, noise).
"""
from __future__ import annotations

import dataclasses
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

CHUNK = 1_000_000

# Polynomial fit of 1/(beta^2 p^2) [MeV^-2 cm^-k] versus water depth [cm] for
# 200 MeV protons, the Highland-type constant E0 [MeV] and the radiation
# length of water X0 [cm], as published with the most-likely-path formalism
# (Schulte et al., Med. Phys. 35:4849, 2008), which the paper cites for the
# per-proton path (Section I).  These are inputs of both implementations.
MLP_WATER_200MEV = dict(
    poly=(7.457e-6, 4.548e-7, -5.777e-8, 1.301e-8, -9.228e-10, 2.687e-11),
    E0=13.6,
    X0=36.08,
    log_term=1,
)

# Constant scattering power of the exit-deflection stand-in [rad^2/mm]:
# sigma_theta = sqrt(T*D) gives 38 mrad after 200 mm of water.
SCATTER_POWER = 7.2e-6


# --------------------------------------------------------------------------
# geometry and model parameters
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    pitch: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    origin: Optional[Tuple[float, float, float]] = None  # None -> centred

    def __post_init__(self):
        if self.origin is None:
            o = tuple(-0.5 * n * p for n, p in zip((self.nx, self.ny, self.nz), self.pitch))
            object.__setattr__(self, "origin", o)

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape_zyx(self):
        return (self.nz, self.ny, self.nx)

    @property
    def lo(self):
        return np.array(self.origin, dtype=np.float64)

    @property
    def hi(self):
        return np.array([o + n * p for o, n, p in zip(self.origin, (self.nx, self.ny, self.nz), self.pitch)])


@dataclass(frozen=True)
class MLPModel:
    u_in: float
    u_out: float
    step: float = 1.0
    poly: Tuple[float, ...] = MLP_WATER_200MEV["poly"]
    E0: float = MLP_WATER_200MEV["E0"]
    X0: float = MLP_WATER_200MEV["X0"]
    log_term: int = MLP_WATER_200MEV["log_term"]

    @property
    def depth(self) -> float:
        return self.u_out - self.u_in


# --------------------------------------------------------------------------
# analytic phantom
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Shape:
    kind: str          # "zcyl" (infinite along z), "ellipsoid", "sphere"
    centre: Tuple[float, float, float]
    axes: Tuple[float, float, float]  # zcyl: (r, r, inf); sphere: (r, r, r)
    rsp: float

    def inside(self, p: np.ndarray) -> np.ndarray:
        c = np.asarray(self.centre)
        q = (p - c)
        if self.kind == "zcyl":
            return q[..., 0] ** 2 + q[..., 1] ** 2 < self.axes[0] ** 2
        a = np.asarray(self.axes)
        return np.sum((q / a) ** 2, axis=-1) < 1.0

    def chord_interval(self, A: np.ndarray, d: np.ndarray):
        """Parameter interval [s0, s1] of the line A + s d inside the shape
        (empty intervals come back with s1 <= s0)."""
        c = np.asarray(self.centre)
        q = A - c
        if self.kind == "zcyl":
            qa, da = q[:, :2], d[:, :2]
            inv = np.full(2, 1.0 / self.axes[0])
        else:
            qa, da = q, d
            inv = 1.0 / np.asarray(self.axes)
        qa = qa * inv
        da = da * inv
        a = np.sum(da * da, axis=1)
        bq = np.sum(qa * da, axis=1)
        cq = np.sum(qa * qa, axis=1) - 1.0
        disc = bq * bq - a * cq
        ok = (disc > 0) & (a > 0)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        asafe = np.where(a > 0, a, 1.0)
        s0 = np.where(ok, (-bq - sq) / asafe, 1.0)
        s1 = np.where(ok, (-bq + sq) / asafe, 0.0)
        return s0, s1


@dataclass
class Phantom:
    background: Shape
    inserts: List[Shape] = field(default_factory=list)

    def rsp_at(self, p: np.ndarray) -> np.ndarray:
        out = np.where(self.background.inside(p), self.background.rsp, 0.0)
        for s in self.inserts:
            out = np.where(s.inside(p), s.rsp, out)
        return out

    def voxelize(self, grid: Grid, sub: int = 4) -> np.ndarray:
        """Mean RSP over sub^3 points per voxel, flat index ix + nx*(iy + ny*iz)."""
        out = np.empty(grid.nvox, dtype=np.float64)
        offs = (np.arange(sub) + 0.5) / sub
        ox, oy, oz = grid.origin
        px, py, pz = grid.pitch
        xs = ox + (np.arange(grid.nx)[:, None] + offs[None, :]).ravel() * px
        ys = oy + (np.arange(grid.ny)[:, None] + offs[None, :]).ravel() * py
        plane = grid.nx * grid.ny
        for iz in range(grid.nz):
            acc = np.zeros((grid.ny, grid.nx))
            for fz in offs:
                z = oz + (iz + fz) * pz
                X, Y = np.meshgrid(xs, ys)
                P = np.stack([X, Y, np.full_like(X, z)], axis=-1)
                r = self.rsp_at(P).reshape(grid.ny, sub, grid.nx, sub)
                acc += r.sum(axis=(1, 3))
            out[iz * plane:(iz + 1) * plane] = (acc / sub ** 3).ravel()
        return out

    def line_integral(self, A: np.ndarray, B: np.ndarray, grid: Grid) -> np.ndarray:
        """Exact integral of RSP along the straight segments A->B (mm), with
        the phantom clipped to the grid box.  Inserts must not overlap each
        other; they may overlap the background partially."""
        d = B - A
        L = np.linalg.norm(d, axis=1)
        # box interval (slab method)
        s_lo = np.zeros(len(A))
        s_hi = np.ones(len(A))
        lo, hi = grid.lo, grid.hi
        for ax in range(3):
            da = d[:, ax]
            nz = da != 0
            t0 = np.where(nz, (lo[ax] - A[:, ax]) / np.where(nz, da, 1.0), -np.inf)
            t1 = np.where(nz, (hi[ax] - A[:, ax]) / np.where(nz, da, 1.0), np.inf)
            inside_flat = (A[:, ax] >= lo[ax]) & (A[:, ax] < hi[ax])
            t0 = np.where(nz, t0, np.where(inside_flat, -np.inf, np.inf))
            t1 = np.where(nz, t1, np.where(inside_flat, np.inf, -np.inf))
            s_lo = np.maximum(s_lo, np.minimum(t0, t1))
            s_hi = np.minimum(s_hi, np.maximum(t0, t1))

        def clip(s0, s1):
            return np.maximum(s0, s_lo), np.minimum(s1, s_hi)

        def length(s0, s1):
            return np.maximum(s1 - s0, 0.0) * L

        bg = self.background
        b0, b1 = clip(*bg.chord_interval(A, d))
        total = bg.rsp * length(b0, b1)
        for s in self.inserts:
            i0, i1 = clip(*s.chord_interval(A, d))
            total += s.rsp * length(i0, i1) - bg.rsp * length(np.maximum(i0, b0), np.minimum(i1, b1))
        return total


# --------------------------------------------------------------------------
# scan configurations
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class ScanConfig:
    name: str
    grid: Grid
    m: int
    n_angles: int
    r_hull: float
    block: int
    lam: float
    n_iter: int
    phantom: str
    order: str = "acquisition"  # or "angle_slab"
    value_type: str = "f32"     # value type of x on the GPU
    seed: int = 0
    slab_mm: float = 4.0
    sigma_dir: float = 0.010   # entry slope sigma [rad]
    noise_mm: float = 1.0
    continuous_angles: bool = False  # gantry angle per proton ~ U[0, 2pi) (drawn last)

    def with_(self, **kw) -> "ScanConfig":
        return dataclasses.replace(self, **kw)

    @property
    def mlp(self) -> MLPModel:
        return MLPModel(u_in=-self.r_hull, u_out=self.r_hull, step=1.0)


def _phantom(name: str, grid: Grid, seed: int) -> Phantom:
    if name == "cyl64":
        bg = Shape("zcyl", (0, 0, 0), (28.0, 28.0, math.inf), 1.0)
        ins = [Shape("zcyl", (15 * math.cos(a), 15 * math.sin(a), 0), (5.0, 5.0, math.inf), r)
               for a, r in zip((0.0, 2 * math.pi / 3, 4 * math.pi / 3), (0.2, 1.1, 1.7))]
        return Phantom(bg, ins)
    if name == "cyl200":
        # insert RSPs: the true values of the CTP404 inserts (Table VIII)
        rsps = (0.883, 0.980, 1.024, 1.160, 1.359, 1.790)
        bg = Shape("zcyl", (0, 0, 0), (90.0, 90.0, math.inf), 1.0)
        ins = [Shape("zcyl", (48 * math.cos(k * math.pi / 3), 48 * math.sin(k * math.pi / 3), 0),
                     (16.0, 16.0, math.inf), r) for k, r in enumerate(rsps)]
        return Phantom(bg, ins)
    if name == "head256":
        axes = (100.0, 80.0, 30.0)
        bg = Shape("ellipsoid", (0, 0, 0), axes, 1.04)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
        spheres: List[Shape] = []
        tries = 0
        while len(spheres) < 10 and tries < 100000:
            tries += 1
            r = rng.uniform(3.0, 12.0)
            sh = np.array(axes) - r
            c = rng.uniform(-sh, sh)
            if np.sum((c / sh) ** 2) >= 1.0:
                continue
            if any(np.linalg.norm(c - np.array(s.centre)) < r + s.axes[0] for s in spheres):
                continue
            spheres.append(Shape("sphere", tuple(float(v) for v in c), (r, r, r), float(rng.uniform(0.25, 1.7))))
        return Phantom(bg, spheres)
    if name == "tiny":
        bg = Shape("zcyl", (0, 0, 0), (3.5, 3.5, math.inf), 1.0)
        ins = [Shape("zcyl", (1.5, 0.5, 0), (1.2, 1.2, math.inf), 1.6)]
        return Phantom(bg, ins)
    raise KeyError(name)


WORKLOADS = {
    1: ScanConfig("cyl64_fp64", Grid(64, 64, 4), m=200_000, n_angles=90, r_hull=30.0, block=3200,
                  lam=0.1, n_iter=6, phantom="cyl64", value_type="f64", seed=1001),
    2: ScanConfig("cyl200_fp32", Grid(200, 200, 32), m=10_000_000, n_angles=180, r_hull=100.0,
                  block=3200, lam=0.1, n_iter=12, phantom="cyl200", seed=1002),
    3: ScanConfig("head256_sorted", Grid(256, 256, 64), m=50_000_000, n_angles=360, r_hull=110.0,
                  block=6400, lam=0.1, n_iter=8, phantom="head256", order="angle_slab", seed=1003),
    4: ScanConfig("cyl200_lowprec", Grid(200, 200, 32), m=20_000_000, n_angles=180, r_hull=100.0,
                  block=3200, lam=0.1, n_iter=8, phantom="cyl200", seed=1004),
    5: ScanConfig("head256_tvgd", Grid(256, 256, 64), m=20_000_000, n_angles=360, r_hull=110.0,
                  block=6400, lam=0.1, n_iter=20, phantom="head256", order="angle_slab", seed=1005),
    # continuous gantry rotation (as in the paper's scanner data, Section IV-A)
    # on the 200x200x32 geometry, protons sorted into 180 angle bins, then by
    # slab and t_in
    "cont": ScanConfig("cont_cyl200_anglebins", Grid(200, 200, 32), m=10_000_000, n_angles=180, r_hull=100.0,
                       block=3200, lam=0.1, n_iter=12, phantom="cyl200", order="angle_slab", seed=1007,
                       continuous_angles=True),
    # multi-region case: 20 slices like the reconstructions of the paper's
    # Section III example (two regions, slices 0-12 and 7-19)
    "regions": ScanConfig("regions_cyl64x20", Grid(64, 64, 20), m=60_000, n_angles=90, r_hull=30.0, block=3200,
                          lam=0.1, n_iter=3, phantom="cyl64", value_type="f64", seed=1006),
    "tiny": ScanConfig("tiny_8x8x2", Grid(8, 8, 2), m=20_000, n_angles=90, r_hull=4.0, block=200,
                       lam=0.1, n_iter=4, phantom="tiny", value_type="f64", seed=1000),
}


# --------------------------------------------------------------------------
# scans
# --------------------------------------------------------------------------
FIELDS = ("t_in", "v_in", "th_in", "ph_in", "t_out", "v_out", "th_out", "ph_out", "gantry")


@dataclass
class Scan:
    cfg: ScanConfig
    grid: Grid
    mlp: MLPModel
    protons: dict          # FIELDS -> float32 arrays [m]
    b: np.ndarray          # float32 [m]
    phantom: Phantom

    @property
    def m(self) -> int:
        return len(self.b)

    def subset(self, lo: int, hi: int) -> "Scan":
        return Scan(self.cfg.with_(m=hi - lo), self.grid, self.mlp,
                    {k: v[lo:hi] for k, v in self.protons.items()}, self.b[lo:hi], self.phantom)

    def x_true(self) -> np.ndarray:
        return self.phantom.voxelize(self.grid)


def lab_point(u, t, v, phi):
    """Beam-frame (u, t, v) at gantry angle phi -> lab (x, y, z), float64."""
    c, s = np.cos(phi), np.sin(phi)
    return np.stack([u * c - t * s, u * s + t * c, v], axis=1)


WEPL_PIECES = 4


def wepl_along_hermite(phantom: "Phantom", grid: Grid, mlp: MLPModel, f: dict) -> np.ndarray:
    """Phantom integral along the cubic Hermite curve of every record (float64
    fields), in WEPL_PIECES straight pieces, clipped to the grid box."""
    D = mlp.depth
    n = len(f["t_in"])
    pts = []
    for s in np.linspace(0.0, 1.0, WEPL_PIECES + 1):
        h00, h10, h01, h11 = 2 * s**3 - 3 * s**2 + 1, s**3 - 2 * s**2 + s, -2 * s**3 + 3 * s**2, s**3 - s**2
        t = h00 * f["t_in"] + h10 * D * f["th_in"] + h01 * f["t_out"] + h11 * D * f["th_out"]
        v = h00 * f["v_in"] + h10 * D * f["ph_in"] + h01 * f["v_out"] + h11 * D * f["ph_out"]
        pts.append(lab_point(np.full(n, mlp.u_in + s * D), t, v, f["gantry"]))
    return sum(phantom.line_integral(pts[k], pts[k + 1], grid) for k in range(WEPL_PIECES))


def make_scan(cfg: ScanConfig, m: Optional[int] = None, seed: Optional[int] = None,
              with_b: bool = True) -> Scan:
    m = cfg.m if m is None else int(m)
    seed = cfg.seed if seed is None else seed
    grid = cfg.grid
    mlp = cfg.mlp
    phantom = _phantom(cfg.phantom, grid, seed)
    D = mlp.depth
    T = SCATTER_POWER
    cov = T * np.array([[D ** 3 / 3, D ** 2 / 2], [D ** 2 / 2, D]])
    chol = np.linalg.cholesky(cov)
    zlo, zhi = grid.lo[2], grid.hi[2]

    out = {k: np.empty(m, np.float32) for k in FIELDS}
    b = np.empty(m, np.float32)
    n_chunks = max(1, (m + CHUNK - 1) // CHUNK)
    children = np.random.SeedSequence(seed).spawn(n_chunks)

    def chunk(c):
        lo, hi = c * CHUNK, min(m, (c + 1) * CHUNK)
        n = hi - lo
        if n <= 0:
            return
        rng = np.random.Generator(np.random.PCG64(children[c]))
        t_in = rng.uniform(-cfg.r_hull, cfg.r_hull, n)
        v_in = rng.uniform(zlo, zhi, n)
        th_in = rng.normal(0.0, cfg.sigma_dir, n)
        ph_in = rng.normal(0.0, cfg.sigma_dir, n)
        zt = rng.standard_normal((n, 2))
        zv = rng.standard_normal((n, 2))
        noise = rng.standard_normal(n) * cfg.noise_mm
        # correlated deflections chol @ z, written out (no BLAS call: results
        # must not depend on how a library splits work across threads)
        t_out = t_in + th_in * D + (chol[0, 0] * zt[:, 0] + chol[0, 1] * zt[:, 1])
        th_out = th_in + (chol[1, 0] * zt[:, 0] + chol[1, 1] * zt[:, 1])
        v_out = v_in + ph_in * D + (chol[0, 0] * zv[:, 0] + chol[0, 1] * zv[:, 1])
        ph_out = ph_in + (chol[1, 0] * zv[:, 0] + chol[1, 1] * zv[:, 1])
        if cfg.continuous_angles:
            phi = rng.uniform(0.0, 2.0 * np.pi, n).astype(np.float32)
        else:
            idx = np.arange(lo, hi, dtype=np.int64)
            ang = (idx * cfg.n_angles) // m
            phi = (2.0 * np.pi * ang / cfg.n_angles).astype(np.float32)
        rec = dict(t_in=t_in, v_in=v_in, th_in=th_in, ph_in=ph_in, t_out=t_out, v_out=v_out,
                   th_out=th_out, ph_out=ph_out)
        for k, v in rec.items():
            out[k][lo:hi] = v.astype(np.float32)
        out["gantry"][lo:hi] = phi
        if with_b:
            f = {k: out[k][lo:hi].astype(np.float64) for k in FIELDS}
            b[lo:hi] = (wepl_along_hermite(phantom, grid, mlp, f) + noise).astype(np.float32)
        else:
            b[lo:hi] = 0.0

    # chunks are independent (own seed, disjoint output ranges); numpy
    # releases the GIL inside its array operations, so threads overlap them
    if n_chunks > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(8, n_chunks, os.cpu_count() or 1)) as ex:
            list(ex.map(chunk, range(n_chunks)))
    else:
        chunk(0)
    if cfg.order == "angle_slab":
        ang = np.floor(out["gantry"].astype(np.float64) * cfg.n_angles / (2 * np.pi) + 0.5).astype(np.int64)
        slab = np.floor((out["v_in"].astype(np.float64) - zlo) / cfg.slab_mm).astype(np.int64)
        order = np.lexsort((out["t_in"], slab, ang))
        out = {k: np.ascontiguousarray(v[order]) for k, v in out.items()}
        b = np.ascontiguousarray(b[order])
    return Scan(cfg.with_(m=m, seed=seed), grid, mlp, out, b, phantom)


def power_start(nvox: int, seed: int = 0) -> np.ndarray:
    """Seeded positive start vector for power iteration (uniform in [0.5, 1.5))."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    return rng.random(nvox) + 0.5


def make_rays(grid: Grid, mlp: MLPModel, rays: Sequence[Sequence[float]]) -> dict:
    """Hand-placed protons: each ray is (t_in, v_in, th_in, ph_in, t_out, v_out,
    th_out, ph_out, gantry)."""
    arr = np.asarray(rays, dtype=np.float64).reshape(-1, 9)
    return {k: arr[:, i].astype(np.float32) for i, k in enumerate(FIELDS)}


def straight_rays(mlp: MLPModel, n: int, rng: np.random.Generator, t_range: float, v_range: Tuple[float, float],
                  slope: float = 0.05, angles: Optional[np.ndarray] = None) -> dict:
    """Protons whose exit data is exactly collinear with the entry data
    (t_out = t_in + theta*D, theta_out = theta_in): zero-deflection data."""
    D = mlp.depth
    t_in = rng.uniform(-t_range, t_range, n)
    v_in = rng.uniform(v_range[0], v_range[1], n)
    th = rng.uniform(-slope, slope, n)
    ph = rng.uniform(-slope, slope, n)
    phi = angles if angles is not None else rng.uniform(0, 2 * np.pi, n)
    rec = dict(t_in=t_in, v_in=v_in, th_in=th, ph_in=ph, t_out=t_in + th * D, v_out=v_in + ph * D,
               th_out=th, ph_out=ph, gantry=phi)
    return {k: np.asarray(v, dtype=np.float32) for k, v in rec.items()}

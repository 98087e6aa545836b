"""FP64 oracle of the filtered back-projection (FBP) initial iterate.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the package; it shares no code
with the HIP library.

Section I of the paper starts the iterative solve from an FBP image but does
not print the FBP it uses.  The reading implemented here is textbook
parallel-beam FBP (Kak & Slaney, Principles of Computerized Tomographic
Imaging, ch. 3), slice by slice, along the straight entry-to-exit chord of
every proton:

binning
    proton i goes to angle bin a = floor(phi / dphi + 1/2) mod n_angles
    (dphi = 2 pi / n_angles), lateral bin k = floor((t_c - t0) / dt) and the
    slice iz of the grid holding v_c, where (t_c, v_c) is the chord at depth
    u = 0: w = -u_in / (u_out - u_in), t_c = t_in + w (t_out - t_in), same for
    v.  Protons outside the bins, with a non-finite field or b, or with
    |b| >= 2^20 mm (not a WEPL), are dropped.  The projection of a bin is the
    mean b of its protons (0 when it is empty).
filter
    ramp (Ram-Lak) filter along t, as a plain convolution over the row with
    zeros beyond it: q_k = dt sum_n p_n h(k - n), h(0) = 1/(4 dt^2),
    h(m) = -1/(pi^2 m^2 dt^2) for odd m, 0 for even m != 0.
back-projection
    x at a voxel centre (x, y) of slice iz = (pi / n_angles) sum_a q_a(t),
    t = -x sin(phi_a) + y cos(phi_a), phi_a = a dphi; q_a(t) interpolates
    linearly between the lateral bin centres t0 + (k + 1/2) dt, with q = 0
    beyond the first and last bins.  (pi / n_angles = dphi / 2: angles cover
    the full turn, every line is seen twice.)

Sinograms are arrays of shape (nz, n_angles, n_t).
"""
from __future__ import annotations

import numpy as np


def chord_centre(mlp, protons: dict):
    """(t_c, v_c): the straight entry-to-exit chord at depth u = 0 (FP64)."""
    w = -float(mlp.u_in) / (float(mlp.u_out) - float(mlp.u_in))
    f = {k: np.asarray(protons[k], dtype=np.float64) for k in ("t_in", "t_out", "v_in", "v_out")}
    return f["t_in"] + w * (f["t_out"] - f["t_in"]), f["v_in"] + w * (f["v_out"] - f["v_in"])


def bins(grid, mlp, protons: dict, b, n_angles: int, n_t: int, t0: float, dt: float):
    """Bin indices (iz, a, k) of every proton and the mask of kept protons."""
    tc, vc = chord_centre(mlp, protons)
    phi = np.asarray(protons["gantry"], dtype=np.float64)
    bb = np.asarray(b, dtype=np.float64)
    dphi = 2.0 * np.pi / n_angles
    ok = np.isfinite(tc) & np.isfinite(vc) & np.isfinite(phi) & np.isfinite(bb) & (np.abs(bb) < 2.0 ** 20)
    with np.errstate(invalid="ignore"):
        fa = np.floor(phi / dphi + 0.5)
        fk = np.floor((tc - float(t0)) / float(dt))
        fz = np.floor((vc - float(grid.origin[2])) / float(grid.pitch[2]))
    ok &= (fk >= 0) & (fk < n_t) & (fz >= 0) & (fz < grid.nz)
    a = np.where(ok, np.mod(np.where(ok, fa, 0), n_angles), 0).astype(np.int64)
    k = np.where(ok, fk, 0).astype(np.int64)
    iz = np.where(ok, fz, 0).astype(np.int64)
    return iz, a, k, ok


def sinogram(grid, mlp, protons: dict, b, n_angles: int, n_t: int, t0: float, dt: float):
    """Mean b per (slice, angle, lateral) bin and the bin counts."""
    iz, a, k, ok = bins(grid, mlp, protons, b, n_angles, n_t, t0, dt)
    flat = ((iz * n_angles + a) * n_t + k)[ok]
    nb = grid.nz * n_angles * n_t
    s = np.zeros(nb)
    np.add.at(s, flat, np.asarray(b, dtype=np.float64)[ok])          # in proton order
    c = np.bincount(flat, minlength=nb).astype(np.int64)
    p = np.divide(s, c, out=np.zeros(nb), where=c > 0)
    return p.reshape(grid.nz, n_angles, n_t), c.reshape(grid.nz, n_angles, n_t)


def ramlak(n_t: int, dt: float) -> np.ndarray:
    """h(m) for m = -(n_t - 1) .. n_t - 1."""
    m = np.arange(-(n_t - 1), n_t)
    h = np.zeros(m.size)
    h[m == 0] = 1.0 / (4.0 * dt * dt)
    odd = (m % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * m[odd].astype(np.float64) ** 2 * dt * dt)
    return h


def filter_rows(proj: np.ndarray, dt: float) -> np.ndarray:
    """q_k = dt sum_n p_n h(k - n) along the last axis."""
    n_t = proj.shape[-1]
    h = ramlak(n_t, dt)
    rows = proj.reshape(-1, n_t)
    q = np.empty_like(rows)
    for r in range(rows.shape[0]):
        # full convolution, then the n_t outputs aligned with the row
        q[r] = dt * np.convolve(rows[r], h)[n_t - 1:2 * n_t - 1]
    return q.reshape(proj.shape)


def interp(q: np.ndarray, iz: np.ndarray, a: int, t: np.ndarray, t0: float, dt: float) -> np.ndarray:
    """q[iz, a](t): linear interpolation between the lateral bin centres
    t0 + (k + 1/2) dt, zero beyond the first and last bins."""
    n_t = q.shape[-1]
    s = (t - t0) / dt - 0.5
    k = np.floor(s)
    w = s - k
    k = k.astype(np.int64)

    def at(kk):
        inside = (kk >= 0) & (kk < n_t)
        return np.where(inside, q[iz, a, np.clip(kk, 0, n_t - 1)], 0.0)

    return (1.0 - w) * at(k) + w * at(k + 1)


def backproject(grid, q: np.ndarray, n_angles: int, t0: float, dt: float, voxels=None) -> np.ndarray:
    """FBP image (FP64, flat voxel order) from filtered sinograms q; with
    `voxels` (flat indices) only those voxels are returned."""
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    if voxels is None:
        voxels = np.arange(nx * ny * nz)
    voxels = np.asarray(voxels, dtype=np.int64)
    ix, iy, iz = voxels % nx, (voxels // nx) % ny, voxels // (nx * ny)
    xc = float(grid.origin[0]) + (ix + 0.5) * float(grid.pitch[0])
    yc = float(grid.origin[1]) + (iy + 0.5) * float(grid.pitch[1])
    dphi = 2.0 * np.pi / n_angles
    acc = np.zeros(voxels.size)
    for a in range(n_angles):
        phi = a * dphi
        t = -xc * np.sin(phi) + yc * np.cos(phi)
        acc += interp(q, iz, a, t, t0, dt)
    return (np.pi / n_angles) * acc


def fbp(grid, mlp, protons: dict, b, n_angles: int, n_t: int, t0: float, dt: float) -> np.ndarray:
    """The whole FBP image: sinogram, ramp filter, back-projection."""
    p, _ = sinogram(grid, mlp, protons, b, n_angles, n_t, t0, dt)
    return backproject(grid, filter_rows(p, dt), n_angles, t0, dt)

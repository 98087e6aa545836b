"""FP64 oracle of the multi-region reconstruction (test infrastructure only).

Algorithm 1 of the paper (Section III): the volume is cut along z into
overlapping slab regions, each proton is given to every region that holds
both the slice it enters the volume in and the slice it leaves it in, an
independent iterative solve runs per region, and every overlapped slice is
finally taken from the region whose own, non-overlapped slices are nearest
(the selectSlice step).  Section III's example: 20 slices, two regions with
slices 0-12 and 7-19, overlap 7-12, final image = slices 0-9 of the first
region and 10-19 of the second.

Readings (where the paper is silent):
* region cores split the nz slices evenly (core r = [floor(r nz/R),
  floor((r+1) nz/R) - 1]) and each region extends `halo` slices past every
  interior core boundary, so the overlap of two neighbours is 2*halo slices
  ("twice the slices" of the coverage count); selectSlice keeps each region's
  core;
* the entry and exit slices come from v_in and v_out (the lab z of the track
  at the entry and exit planes): floor((v - z0) / pitch_z) in FP64, clamped to
  [0, nz-1];
* inside a region the protons keep their input order; its grid is the
  parent grid restricted to the region's slices (same x-y extent, origin
  moved up by z_lo slices); paths are clipped to that box;
* the initial iterate of a region is the parent's initial iterate on the
  region's slices.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import drop


def layout(nz: int, n_regions: int, halo: int) -> List[Tuple[int, int, int, int]]:
    """Per region (z_lo, z_hi, core_lo, core_hi), inclusive slice indices."""
    if n_regions < 1 or n_regions > nz or halo < 0:
        raise ValueError("need 1 <= n_regions <= nz and halo >= 0")
    out = []
    for r in range(n_regions):
        c0 = (r * nz) // n_regions
        c1 = ((r + 1) * nz) // n_regions - 1
        z0 = max(0, c0 - halo) if r > 0 else 0
        z1 = min(nz - 1, c1 + halo) if r < n_regions - 1 else nz - 1
        out.append((z0, z1, c0, c1))
    return out


def slice_of(grid, v: np.ndarray) -> np.ndarray:
    """Slice index of lab z = v (float32 promoted exactly), clamped."""
    v = np.asarray(v, dtype=np.float64)
    finite = np.isfinite(v)
    s = np.floor((np.where(finite, v, 0.0) - float(grid.origin[2])) / float(grid.pitch[2]))
    s = np.clip(s, 0, grid.nz - 1).astype(np.int64)
    return np.where(finite, s, -1)     # a non-finite track belongs to no region


def members(grid, protons: dict, z_lo: int, z_hi: int) -> np.ndarray:
    """Input-order indices of the protons whose entry and exit slices both lie
    in [z_lo, z_hi]."""
    si = slice_of(grid, protons["v_in"])
    so = slice_of(grid, protons["v_out"])
    ok = (si >= z_lo) & (si <= z_hi) & (so >= z_lo) & (so <= z_hi)
    return np.nonzero(ok)[0]


def sub_grid(grid, z_lo: int, z_hi: int):
    """The parent grid restricted to slices z_lo..z_hi."""
    import dataclasses
    o = grid.origin
    return dataclasses.replace(grid, nz=z_hi - z_lo + 1,
                               origin=(o[0], o[1], o[2] + z_lo * grid.pitch[2]))


def slices(x: np.ndarray, grid, z_lo: int, z_hi: int) -> np.ndarray:
    """Voxels of slices z_lo..z_hi of a flat volume (z is the slowest axis)."""
    plane = grid.nx * grid.ny
    return x[z_lo * plane:(z_hi + 1) * plane]


def region_drop(grid, mlp, protons: dict, b: np.ndarray, x0, n_regions: int, halo: int, block: int, lam: float,
                n_iter: int, mode: str = "none"):
    """Algorithm 1 with DROP as the per-region solver: returns the stitched
    volume and, per region, (z_lo, z_hi, core_lo, core_hi, member count)."""
    x0 = np.broadcast_to(np.asarray(x0, dtype=np.float64), (grid.nvox,)).copy()
    out = x0.copy()
    info = []
    plane = grid.nx * grid.ny
    for z_lo, z_hi, c_lo, c_hi in layout(grid.nz, n_regions, halo):
        idx = members(grid, protons, z_lo, z_hi)
        g = sub_grid(grid, z_lo, z_hi)
        sub = {k: np.ascontiguousarray(v[idx]) for k, v in protons.items()}
        xr = slices(x0, grid, z_lo, z_hi).copy()
        if len(idx):
            xr = drop(g, mlp, sub, np.ascontiguousarray(b[idx]), xr, block=block, lam=lam, n_iter=n_iter, mode=mode)
        # selectSlice: the region's own core slices
        out[c_lo * plane:(c_hi + 1) * plane] = xr[(c_lo - z_lo) * plane:(c_hi - z_lo + 1) * plane]
        info.append((z_lo, z_hi, c_lo, c_hi, len(idx)))
    return out, info


def coverage(grid, protons: dict, k: int) -> float:
    """Fraction of protons whose entry and exit slices differ by at most k
    (the quantity of the paper's Table I)."""
    d = np.abs(slice_of(grid, protons["v_out"]) - slice_of(grid, protons["v_in"]))
    return float(np.mean(d <= k))


def halo_for(grid, protons: dict, target: float = 0.96) -> int:
    """Smallest slice difference k covering at least `target` of the protons."""
    for k in range(grid.nz):
        if coverage(grid, protons, k) >= target:
            return k
    return grid.nz - 1

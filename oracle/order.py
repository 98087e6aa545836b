"""FP64 oracle of the angle-bin ordering of an acquisition-order scan.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the package; it
shares no code with the HIP library.

Section IV-A of the paper reconstructs a simulated scan taken at fixed
projection angles and an experimental scan taken with continuous gantry
rotation.  Records of a continuous scan arrive in acquisition order; before
the block-iterative solve they are grouped into angle bins and, inside a bin,
by a slab of the entry height and the lateral entry position, so that a block
of consecutive records covers neighbouring paths.  The paper does not print
the grouping; the reading implemented here is a stable sort by the key
(a, s, t_in):

    a = floor(phi / dphi + 1/2) mod n_angles, dphi = 2 pi / n_angles
        (the same angle bin as the FBP binning), in FP64 from the FP32 gantry
        angle phi;
    s = floor((v_in - z0) / slab_mm) in FP64, clamped to [0, n_slabs - 1],
        with z0 the grid's lower z edge and n_slabs = ceil(nz pz / slab_mm);
    t_in compared as a number (-0 and +0 are equal);
    equal keys keep their input order; a record whose gantry angle, v_in or
    t_in is not finite goes after all others, in input order.
"""
from __future__ import annotations

import math

import numpy as np


def n_slabs(grid, slab_mm: float) -> int:
    """Number of slabs of slab_mm along the grid's z extent."""
    return int(math.ceil(float(grid.nz) * float(grid.pitch[2]) / float(slab_mm)))


def keys(grid, protons: dict, n_angles: int, slab_mm: float):
    """(a, s, t, bad): angle bin, slab, lateral entry and the non-finite mask."""
    phi = np.asarray(protons["gantry"], dtype=np.float64)
    v = np.asarray(protons["v_in"], dtype=np.float64)
    t = np.asarray(protons["t_in"], dtype=np.float64)
    bad = ~(np.isfinite(phi) & np.isfinite(v) & np.isfinite(t))
    dphi = 2.0 * np.pi / n_angles
    with np.errstate(invalid="ignore", over="ignore"):
        fa = np.floor(np.where(bad, 0.0, phi) / dphi + 0.5)
        a = np.mod(fa, float(n_angles)).astype(np.int64)
        fs = np.floor((np.where(bad, 0.0, v) - float(grid.origin[2])) / float(slab_mm))
    s = np.clip(fs, 0, n_slabs(grid, slab_mm) - 1).astype(np.int64)
    a = np.where(bad, n_angles, a)
    s = np.where(bad, 0, s)
    t = np.where(bad, 0.0, t) + 0.0          # -0 becomes +0
    return a, s, t, bad


def order(grid, protons: dict, n_angles: int, slab_mm: float) -> np.ndarray:
    """Input position of every output record (a permutation of 0..n-1)."""
    a, s, t, _ = keys(grid, protons, n_angles, slab_mm)
    # lexsort is stable and sorts by its last key first
    return np.lexsort((t, s, a)).astype(np.int64)


def sort_scan(grid, protons: dict, b, n_angles: int, slab_mm: float):
    """The records (and b, if given) in the angle-bin order, and the order."""
    perm = order(grid, protons, n_angles, slab_mm)
    out = {k: np.asarray(v)[perm] for k, v in protons.items()}
    return out, (None if b is None else np.asarray(b)[perm]), perm

"""Tolerance of RSP comparisons against the oracle: relative error with a small
floor, so that voxels whose RSP is below 1 (inserts of RSP 0.2, air) are held
to a relative bound too; the floor only keeps voxels near zero (air) from
dividing by nothing."""
import numpy as np

RSP_FLOOR = 0.05


def rsp_err(got, ref):
    """Elementwise |got - ref| / max(|ref|, RSP_FLOOR)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), RSP_FLOOR)

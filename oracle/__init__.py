"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is a plain, slow, deterministic
FP64 implementation of the reconstruction path (see ``orc.c`` for the
readings of the paper it implements) and shares no code with the HIP library.

Functions take the objects produced by ``paper_1802_01070_amd.synth`` (a
``Grid``, an ``MLPModel`` and a dict of float32 proton arrays); nothing of the
method's arithmetic lives in that generator.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

FIELDS = ("t_in", "v_in", "th_in", "ph_in", "t_out", "v_out", "th_out", "ph_out", "gantry")
CHORD_MODES = {"none": 0, "f32": 1, "f16": 2, "bf16": 3}


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so (gcc, FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("pitch", C.c_double * 3), ("origin", C.c_double * 3)]


class _MLP(C.Structure):
    _fields_ = [("u_in", C.c_double), ("u_out", C.c_double), ("step", C.c_double),
                ("poly", C.c_double * 6), ("E0", C.c_double), ("X0", C.c_double), ("log_term", C.c_int32)]


class _Protons(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_float)) for k in FIELDS] + [("n", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, i64, i32 = C.c_double, C.c_int64, C.c_int32
        L.orc_num_segments.argtypes = [P(_MLP)]
        L.orc_num_segments.restype = C.c_int
        L.orc_depth.argtypes = [P(_MLP), C.c_int]
        L.orc_depth.restype = d
        L.orc_moment.argtypes = [P(_MLP), C.c_int, d, d]
        L.orc_moment.restype = d
        L.orc_sigma.argtypes = [P(_MLP), d, d, P(d)]
        L.orc_mlp_table.argtypes = [P(_MLP), P(d)]
        L.orc_vertices.argtypes = [P(_MLP), P(d), P(_Protons), i64, P(d)]
        L.orc_trace.argtypes = [P(_Grid), P(_MLP), P(d), P(_Protons), i64, i64, P(i32), P(d)]
        L.orc_trace.restype = i64
        L.orc_trace_batch.argtypes = [P(_Grid), P(_MLP), P(_Protons), i64, i64, i64, P(i32), P(d), P(i64)]
        L.orc_set_hull.argtypes = [C.c_int, d, d, d]
        L.orc_set_hull.restype = None
        L.orc_path.argtypes = [P(_MLP), P(d), P(_Protons), i64, P(d), C.c_int]
        L.orc_path.restype = C.c_int
        L.orc_round_chord.argtypes = [d, C.c_int]
        L.orc_round_chord.restype = d
        L.orc_row.argtypes = [P(_Grid), P(_MLP), P(_Protons), i64, C.c_int, i64, P(i32), P(d), P(i64)]
        L.orc_row.restype = i64
        L.orc_forward.argtypes = [P(_Grid), P(_MLP), P(_Protons), C.c_int, P(d), P(d), P(d), P(i64)]
        L.orc_backproject.argtypes = [P(_Grid), P(_MLP), P(_Protons), C.c_int, P(d), P(d)]
        L.orc_drop.argtypes = [P(_Grid), P(_MLP), P(_Protons), P(C.c_float), P(d), i64, d, C.c_int, i64, i64,
                               C.c_int]
        L.orc_drop.restype = i64
        L.orc_tv.argtypes = [P(_Grid), P(d), d, P(d)]
        L.orc_tv.restype = d
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# marshalling
# ---------------------------------------------------------------------------
def _ptr(a: Optional[np.ndarray], ct):
    if a is None:
        return C.POINTER(ct)()
    return a.ctypes.data_as(C.POINTER(ct))


def _grid(g) -> _Grid:
    return _Grid(g.nx, g.ny, g.nz, (C.c_double * 3)(*g.pitch), (C.c_double * 3)(*g.origin))


def _mlp(m) -> _MLP:
    return _MLP(m.u_in, m.u_out, m.step, (C.c_double * 6)(*m.poly), m.E0, m.X0, int(m.log_term))


class _ProtonView:
    """Keeps the float32 arrays alive while C sees them."""

    def __init__(self, protons: dict):
        self.arrs = {k: np.ascontiguousarray(protons[k], dtype=np.float32) for k in FIELDS}
        n = len(self.arrs["t_in"])
        self.s = _Protons(*[_ptr(self.arrs[k], C.c_float) for k in FIELDS], n)
        self.n = n


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# public oracle functions
# ---------------------------------------------------------------------------
def num_segments(mlp) -> int:
    return lib().orc_num_segments(C.byref(_mlp(mlp)))


def depth(mlp, k: int) -> float:
    return lib().orc_depth(C.byref(_mlp(mlp)), k)


def moment(mlp, mexp: int, lo_cm: float, end_cm: float) -> float:
    return lib().orc_moment(C.byref(_mlp(mlp)), mexp, lo_cm, end_cm)


def sigma(mlp, lo_cm: float, end_cm: float) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_sigma(C.byref(_mlp(mlp)), lo_cm, end_cm, _ptr(out, C.c_double))
    return out


def mlp_table(mlp) -> np.ndarray:
    K = num_segments(mlp)
    tab = np.zeros((K + 1, 4))
    lib().orc_mlp_table(C.byref(_mlp(mlp)), _ptr(tab, C.c_double))
    return tab


def vertices(mlp, protons: dict, i: int) -> np.ndarray:
    K = num_segments(mlp)
    tab = mlp_table(mlp)
    pv = _ProtonView(protons)
    out = np.zeros((K + 1, 3))
    lib().orc_vertices(C.byref(_mlp(mlp)), _ptr(tab, C.c_double), C.byref(pv.s), i, _ptr(out, C.c_double))
    return out


def set_hull(radius: Optional[float], cx: float = 0.0, cy: float = 0.0):
    """Per-proton paths through the z-cylinder hull of the given radius
    (None: tracker-to-tracker paths).  Process-wide setting of the oracle."""
    if radius is None:
        lib().orc_set_hull(0, 0.0, 0.0, 0.0)
    else:
        lib().orc_set_hull(1, float(cx), float(cy), float(radius))


def path(mlp, protons: dict, i: int) -> np.ndarray:
    """Vertices (n, 3) of proton i's polyline (hull setting applies)."""
    pv = _ProtonView(protons)
    K = num_segments(mlp)
    tab = mlp_table(mlp).ravel().copy()
    P = np.zeros((K + 3) * 3)
    n = lib().orc_path(C.byref(_mlp(mlp)), _ptr(tab, C.c_double), C.byref(pv.s), int(i), _ptr(P, C.c_double), K + 3)
    return P[:3 * n].reshape(n, 3)


def trace(grid, mlp, protons: dict, first: int = 0, count: Optional[int] = None, cap: int = 1024):
    """Ordered emission lists.  Returns (vox[count, cap] int32, chord[count, cap]
    float64, nnz[count] int64); rows longer than cap are truncated (nnz keeps
    the full length)."""
    pv = _ProtonView(protons)
    count = pv.n - first if count is None else count
    vox = np.full((count, cap), -1, np.int32)
    ch = np.zeros((count, cap))
    nnz = np.zeros(count, np.int64)
    lib().orc_trace_batch(C.byref(_grid(grid)), C.byref(_mlp(mlp)), C.byref(pv.s), first, count, cap,
                          _ptr(vox, C.c_int32), _ptr(ch, C.c_double), _ptr(nnz, C.c_int64))
    return vox, ch, nnz


def round_chord(c: float, mode: str) -> float:
    return lib().orc_round_chord(float(c), CHORD_MODES[mode])


def row(grid, mlp, protons: dict, i: int, mode: str = "none"):
    """Distinct-voxel row of proton i: (vox ascending, a_ij, re-entry count)."""
    pv = _ProtonView(protons)
    cap = 4096
    vox = np.zeros(cap, np.int32)
    a = np.zeros(cap)
    rep = np.zeros(1, np.int64)
    n = lib().orc_row(C.byref(_grid(grid)), C.byref(_mlp(mlp)), C.byref(pv.s), i, CHORD_MODES[mode], cap,
                      _ptr(vox, C.c_int32), _ptr(a, C.c_double), _ptr(rep, C.c_int64))
    return vox[:n].copy(), a[:n].copy(), int(rep[0])


def forward(grid, mlp, protons: dict, x: Optional[np.ndarray], mode: str = "none"):
    """(A x, ||a_i||^2, distinct nonzeros per row)."""
    pv = _ProtonView(protons)
    y = np.zeros(pv.n)
    n2 = np.zeros(pv.n)
    nd = np.zeros(pv.n, np.int64)
    xx = None if x is None else _f64(x)
    lib().orc_forward(C.byref(_grid(grid)), C.byref(_mlp(mlp)), C.byref(pv.s), CHORD_MODES[mode],
                      _ptr(xx, C.c_double), _ptr(y, C.c_double), _ptr(n2, C.c_double), _ptr(nd, C.c_int64))
    return y, n2, nd


def backproject(grid, mlp, protons: dict, r: np.ndarray, g0: Optional[np.ndarray] = None, mode: str = "none"):
    """g0 + A^T r."""
    pv = _ProtonView(protons)
    g = np.zeros(grid.nvox) if g0 is None else _f64(g0).copy()
    rr = _f64(r)
    lib().orc_backproject(C.byref(_grid(grid)), C.byref(_mlp(mlp)), C.byref(pv.s), CHORD_MODES[mode],
                          _ptr(rr, C.c_double), _ptr(g, C.c_double))
    return g


def drop(grid, mlp, protons: dict, b: np.ndarray, x0, block: int, lam: float, n_iter: int,
         blk_begin: int = 0, blk_end: int = -1, mode: str = "none") -> np.ndarray:
    """Block-iterative DROP from x0; returns the new iterate (float64)."""
    pv = _ProtonView(protons)
    x = _f64(np.broadcast_to(x0, (grid.nvox,))).copy()
    bb = np.ascontiguousarray(b, dtype=np.float32)
    lib().orc_drop(C.byref(_grid(grid)), C.byref(_mlp(mlp)), C.byref(pv.s), _ptr(bb, C.c_float),
                   _ptr(x, C.c_double), int(block), float(lam), int(n_iter), int(blk_begin), int(blk_end),
                   CHORD_MODES[mode])
    return x


def tv(grid, x: np.ndarray, eps: float, with_grad: bool = True):
    xx = _f64(x)
    g = np.zeros(grid.nvox) if with_grad else None
    val = lib().orc_tv(C.byref(_grid(grid)), _ptr(xx, C.c_double), float(eps), _ptr(g, C.c_double))
    return val, g


# ---------------------------------------------------------------------------
# differentiation form: L(x) = 1/2 ||A x - b||^2 + beta TV_eps(x)
# ---------------------------------------------------------------------------
def tv_loss(grid, mlp, protons: dict, b: np.ndarray, x: np.ndarray, beta: float, eps: float):
    """(loss, gradient) of the TV-regularised least-squares objective."""
    y, _, _ = forward(grid, mlp, protons, x)
    r = y - np.asarray(b, dtype=np.float64)
    tval, tgrad = tv(grid, x, eps)
    g = backproject(grid, mlp, protons, r) + beta * tgrad
    return 0.5 * float(r @ r) + beta * tval, g


def power_iteration(grid, mlp, protons: dict, v0: np.ndarray, n_steps: int = 20) -> float:
    """Estimate of the largest eigenvalue of A^T A by n_steps power steps from
    the start vector v0 (an input: random draws are not the oracle's)."""
    v = _f64(v0).copy()
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(n_steps):
        y, _, _ = forward(grid, mlp, protons, v)
        w = backproject(grid, mlp, protons, y)
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def gradient_descent(grid, mlp, protons: dict, b: np.ndarray, x0: np.ndarray, beta: float, eps: float,
                     eta: float, n_steps: int):
    """Plain fixed-step gradient descent; returns (x, losses)."""
    x = _f64(x0).copy()
    losses = []
    for _ in range(n_steps):
        loss, g = tv_loss(grid, mlp, protons, b, x, beta, eps)
        losses.append(loss)
        x = x - eta * g
    return x, losses

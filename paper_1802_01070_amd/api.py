"""PyTorch-facing binding of the C ABI, one function per entry point.

Tensors supply device memory; the current torch stream is the stream every
call is enqueued on.  Nothing here computes: each function checks tensor
shapes/dtypes/devices, marshals pointers and calls libpct.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import FIELDS, PCT_F32, PCT_F64, check, lib


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return PCT_F32
    if t.dtype == torch.float64:
        return PCT_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t: torch.Tensor, what: str, dtype=None, numel: Optional[int] = None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{what} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Plan:
    """A pct_plan plus its device workspace (uploaded once).  n_hint: the
    largest DROP block that runs with the traced-ahead schedule."""

    def __init__(self, grid, mlp, device="cuda:0", n_hint: int = 8192, _handle: Optional[C.c_void_p] = None):
        self.grid = grid
        self.mlp = mlp
        self.device = torch.device(device)
        self.nvox = int(grid.nx) * int(grid.ny) * int(grid.nz)
        self.hull = None
        h = _handle
        if h is None:
            h = C.c_void_p()
            check(lib().pct_plan_create(C.byref(_lib.make_grid(grid)), C.byref(_lib.make_mlp(mlp)), C.byref(h)),
                  "pct_plan_create")
        self.handle = h
        k = C.c_int32()
        check(lib().pct_plan_segments(h, C.byref(k)), "pct_plan_segments")
        self.K = k.value
        nbytes = C.c_size_t()
        check(lib().pct_workspace_size(h, int(n_hint), PCT_F64, C.byref(nbytes)), "pct_workspace_size")
        self.ws_bytes = nbytes.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = C.c_void_p(self.ws.data_ptr() + off)
        check(lib().pct_plan_upload(h, self.ws_ptr, self.ws_bytes, _stream(self.device)), "pct_plan_upload")

    def set_hull(self, radius: Optional[float], cx: float = 0.0, cy: float = 0.0):
        """Per-proton paths through the z-cylinder hull (pct_plan_set_hull);
        radius None: tracker-to-tracker paths."""
        h = None if radius is None else C.byref(_lib.pct_hull(float(cx), float(cy), float(radius)))
        check(lib().pct_plan_set_hull(self.handle, h), "pct_plan_set_hull")
        self.hull = None if radius is None else (float(cx), float(cy), float(radius))
        return self

    def region(self, z_lo: int, z_hi: int) -> "Plan":
        """Plan of slices z_lo..z_hi of this grid (pct_plan_region)."""
        import dataclasses
        h = C.c_void_p()
        check(lib().pct_plan_region(self.handle, int(z_lo), int(z_hi), C.byref(h)), "pct_plan_region")
        o = self.grid.origin
        g = dataclasses.replace(self.grid, nz=int(z_hi) - int(z_lo) + 1,
                                origin=(o[0], o[1], o[2] + int(z_lo) * self.grid.pitch[2]))
        sub = Plan(g, self.mlp, self.device, _handle=h)
        sub.hull = getattr(self, "hull", None)        # the library copies the parent's hull setting
        return sub

    def table(self):
        import numpy as np
        tab = np.zeros((self.K + 1) * 4)
        check(lib().pct_plan_table(self.handle, tab.ctypes.data_as(C.POINTER(C.c_double)), tab.size),
              "pct_plan_table")
        return tab.reshape(self.K + 1, 4)

    def close(self):
        if getattr(self, "handle", None):
            lib().pct_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Protons:
    """Device-resident SoA proton records (float32)."""

    def __init__(self, arrays: dict, device="cuda:0"):
        self.t = {}
        n = None
        for k in FIELDS:
            a = arrays[k]
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(a)
            t = t.to(device=device, dtype=torch.float32).contiguous()
            if n is None:
                n = t.numel()
            elif t.numel() != n:
                raise ValueError("proton arrays differ in length")
            self.t[k] = t
        self.n = int(n)
        self.s = _lib.make_protons({k: self.t[k].data_ptr() for k in FIELDS}, self.n)

    def slice(self, lo: int, hi: int) -> "Protons":
        return Protons({k: v[lo:hi] for k, v in self.t.items()}, device=self.t["t_in"].device)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def pct_mlp_trace(plan: Plan, p: Protons, first: int = 0, count: Optional[int] = None, max_nnz: int = 512):
    count = p.n - first if count is None else int(count)
    dev = plan.device
    vox = torch.full((count, max_nnz), -1, dtype=torch.int32, device=dev)
    chord = torch.zeros((count, max_nnz), dtype=torch.float64, device=dev)
    nnz = torch.zeros(count, dtype=torch.int32, device=dev)
    st = lib().pct_mlp_trace(plan.handle, C.byref(p.s), int(first), count, int(max_nnz), C.c_void_p(vox.data_ptr()),
                             C.c_void_p(chord.data_ptr()), C.c_void_p(nnz.data_ptr()), plan.ws_ptr, plan.ws_bytes,
                             _stream(dev))
    check(st, "pct_mlp_trace")
    return vox, chord, nnz


def pct_forward(plan: Plan, p: Protons, x: torch.Tensor, with_norm: bool = False, y=None, nrm2=None):
    code = _dtype_code(x)
    xp = _dev(x, "x", numel=plan.nvox)
    y = torch.empty(p.n, dtype=x.dtype, device=x.device) if y is None else y
    yp = _dev(y, "y", dtype=x.dtype, numel=p.n)
    n2p = None
    if with_norm:
        nrm2 = torch.empty(p.n, dtype=x.dtype, device=x.device) if nrm2 is None else nrm2
        n2p = _dev(nrm2, "nrm2", dtype=x.dtype, numel=p.n)
    st = lib().pct_forward(plan.handle, C.byref(p.s), xp, code, yp, n2p, plan.ws_ptr, plan.ws_bytes,
                           _stream(x.device))
    check(st, "pct_forward")
    return (y, nrm2) if with_norm else y


def pct_backproject(plan: Plan, p: Protons, r: torch.Tensor, g: Optional[torch.Tensor] = None):
    code = _dtype_code(r)
    rp = _dev(r, "r", numel=p.n)
    g = torch.zeros(plan.nvox, dtype=r.dtype, device=r.device) if g is None else g
    gp = _dev(g, "g", dtype=r.dtype, numel=plan.nvox)
    st = lib().pct_backproject(plan.handle, C.byref(p.s), rp, code, gp, plan.ws_ptr, plan.ws_bytes,
                               _stream(r.device))
    check(st, "pct_backproject")
    return g


def pct_drop_iterate(plan: Plan, p: Protons, b: torch.Tensor, x: torch.Tensor, block: int, lam: float,
                     n_iter: int, chord: str = "f64", flags: int = 0, block_begin: int = 0, block_end: int = -1,
                     lanes: int = 0):
    code = _dtype_code(x)
    bp = _dev(b, "b", dtype=torch.float32, numel=p.n)
    xp = _dev(x, "x", numel=plan.nvox)
    o = _lib.make_opts(block, lam, n_iter, code, chord, flags, block_begin, block_end, lanes)
    st = lib().pct_drop_iterate(plan.handle, C.byref(p.s), bp, xp, C.byref(o), plan.ws_ptr, plan.ws_bytes,
                                _stream(x.device))
    check(st, "pct_drop_iterate")
    return x


def pct_drop_cancel(plan: Plan, request: bool = True) -> None:
    """Ask the cancellable DROP calls on the plan's workspace to stop at the
    next block boundary (request False clears the request)."""
    check(lib().pct_drop_cancel(plan.handle, plan.ws_ptr, plan.ws_bytes, int(bool(request))), "pct_drop_cancel")


def pct_drop_progress(plan: Plan):
    """(block steps applied, stopped on request) of the last cancellable DROP
    call on the plan's workspace; synchronises the device's current stream."""
    done = C.c_int64()
    st = lib().pct_drop_progress(plan.handle, plan.ws_ptr, plan.ws_bytes, C.byref(done), _stream(plan.device))
    if st not in (_lib.PCT_OK, _lib.PCT_ERR_CANCELLED):
        check(st, "pct_drop_progress")
    return done.value, st == _lib.PCT_ERR_CANCELLED


class Rows:
    """Stored CSR rows of a proton set (pct_rows_count + pct_rows_build):
    chord lengths in FP32, FP16 or BF16, traced once on the GPU."""

    _CHORD_DTYPE = {"f32": torch.float32, "f16": torch.int16, "bf16": torch.int16}

    def __init__(self, plan: Plan, p: Protons, chord: str = "f16"):
        if chord not in self._CHORD_DTYPE:
            raise ValueError("stored chords are f32, f16 or bf16")
        dev = plan.device
        self.n = p.n
        self.chord_name = chord
        self.offsets = torch.empty(p.n + 1, dtype=torch.int64, device=dev)
        st = lib().pct_rows_count(plan.handle, C.byref(p.s), C.c_void_p(self.offsets.data_ptr()), plan.ws_ptr,
                                  plan.ws_bytes, _stream(dev))
        check(st, "pct_rows_count")
        self.nnz = int(self.offsets[-1].item())
        self.vox = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        self.chord = torch.empty(max(self.nnz, 1), dtype=self._CHORD_DTYPE[chord], device=dev)
        self.n2 = torch.empty(max(p.n, 1), dtype=torch.float64, device=dev)
        st = lib().pct_rows_build(plan.handle, C.byref(p.s), _lib.CHORDS[chord], C.c_void_p(self.offsets.data_ptr()),
                                  C.c_void_p(self.vox.data_ptr()), C.c_void_p(self.chord.data_ptr()),
                                  C.c_void_p(self.n2.data_ptr()), plan.ws_ptr, plan.ws_bytes, _stream(dev))
        check(st, "pct_rows_build")
        self.s = _lib.pct_rows(self.offsets.data_ptr(), self.vox.data_ptr(), self.chord.data_ptr(),
                               self.n2.data_ptr(), self.n, _lib.CHORDS[chord], 0)

    @property
    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.offsets, self.vox, self.chord, self.n2))


def pct_drop_iterate_rows(plan: Plan, rows: Rows, b: torch.Tensor, x: torch.Tensor, block: int, lam: float,
                          n_iter: int, flags: int = 0, block_begin: int = 0, block_end: int = -1, lanes: int = 0):
    code = _dtype_code(x)
    bp = _dev(b, "b", dtype=torch.float32, numel=rows.n)
    xp = _dev(x, "x", numel=plan.nvox)
    o = _lib.make_opts(block, lam, n_iter, code, rows.chord_name, flags, block_begin, block_end, lanes)
    st = lib().pct_drop_iterate_rows(plan.handle, C.byref(rows.s), bp, xp, C.byref(o), plan.ws_ptr, plan.ws_bytes,
                                     _stream(x.device))
    check(st, "pct_drop_iterate_rows")
    return x


def pct_tv(plan: Plan, x: torch.Tensor, eps: float, with_grad: bool = True):
    code = _dtype_code(x)
    xp = _dev(x, "x", numel=plan.nvox)
    val = torch.zeros(1, dtype=torch.float64, device=x.device)
    grad = torch.empty_like(x) if with_grad else None
    st = lib().pct_tv(plan.handle, xp, code, float(eps), C.c_void_p(val.data_ptr()),
                      C.c_void_p(grad.data_ptr()) if with_grad else None, plan.ws_ptr, plan.ws_bytes,
                      _stream(x.device))
    check(st, "pct_tv")
    return val, grad


def pct_tv_static(plan: Plan, x: torch.Tensor, eps: float, with_grad: bool = True):
    """pct_tv without a workspace (for callers that cannot allocate: the
    library's own per-GPU scratch array holds the partial sums)."""
    code = _dtype_code(x)
    xp = _dev(x, "x", numel=plan.nvox)
    val = torch.zeros(1, dtype=torch.float64, device=x.device)
    grad = torch.empty_like(x) if with_grad else None
    st = lib().pct_tv_static(plan.handle, xp, code, float(eps), C.c_void_p(val.data_ptr()),
                             C.c_void_p(grad.data_ptr()) if with_grad else None, _stream(x.device))
    check(st, "pct_tv_static")
    return val, grad


def pct_profile_read(plan: Plan):
    """(ms, launches) per kernel kind [fused block kernel, commit] of the last
    profiled pct_drop_iterate call."""
    ms = (C.c_double * 2)()
    n = (C.c_int64 * 2)()
    check(lib().pct_profile_read(plan.handle, ms, n), "pct_profile_read")
    return [ms[0], ms[1]], [n[0], n[1]]


def pct_device_status(plan: Plan, reset: bool = True) -> int:
    bits = C.c_uint32()
    st = lib().pct_device_status(plan.handle, plan.ws_ptr, plan.ws_bytes, int(reset), C.byref(bits),
                                 _stream(plan.device))
    check(st, "pct_device_status")
    return bits.value


# ---------------------------------------------------------------------------
# differentiation form
# ---------------------------------------------------------------------------
class ProjectFn(torch.autograd.Function):
    """y = A x with the hand-written adjoint: backward is A^T grad_y, the MLP
    rows being recomputed by the back-projection kernel (nothing is saved but
    the plan and the proton records)."""

    @staticmethod
    def forward(ctx, x, plan, protons):
        ctx.plan = plan
        ctx.protons = protons
        return pct_forward(plan, protons, x.contiguous())

    @staticmethod
    def backward(ctx, grad_y):
        g = pct_backproject(ctx.plan, ctx.protons, grad_y.contiguous())
        return g, None, None


class TVFn(torch.autograd.Function):
    """Smoothed total variation with its gradient from the same kernel."""

    @staticmethod
    def forward(ctx, x, plan, eps):
        val, grad = pct_tv(plan, x.contiguous(), eps, with_grad=True)
        ctx.save_for_backward(grad)
        return val[0].to(x.dtype)

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return gout * grad, None, None


def pct_region_layout(nz: int, n_regions: int, halo: int):
    """[(z_lo, z_hi, core_lo, core_hi)] per region (host call)."""
    arrs = [(C.c_int32 * n_regions)() for _ in range(4)] if n_regions > 0 else [None] * 4
    check(lib().pct_region_layout(int(nz), int(n_regions), int(halo), *arrs), "pct_region_layout")
    return [tuple(int(a[r]) for a in arrs) for r in range(n_regions)]


def pct_region_select(plan: Plan, p: Protons, b: Optional[torch.Tensor], z_lo: int, z_hi: int):
    """Records (and b) of the protons whose entry and exit slices lie in
    [z_lo, z_hi], in input order: (Protons, b or None)."""
    dev = plan.device
    bufs = {k: torch.empty(p.n, dtype=torch.float32, device=dev) for k in FIELDS}
    b_out = torch.empty(p.n, dtype=torch.float32, device=dev) if b is not None else None
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    out = _lib.make_protons_buf({k: v.data_ptr() for k, v in bufs.items()}, p.n)
    bp = _dev(b, "b", dtype=torch.float32, numel=p.n) if b is not None else None
    st = lib().pct_region_select(plan.handle, C.byref(p.s), bp, int(z_lo), int(z_hi), C.byref(out),
                                 C.c_void_p(b_out.data_ptr()) if b_out is not None else None,
                                 C.c_void_p(count.data_ptr()), plan.ws_ptr, plan.ws_bytes, _stream(dev))
    check(st, "pct_region_select")
    n = int(count.item())
    sub = Protons({k: v[:n] for k, v in bufs.items()}, device=dev)
    return sub, (b_out[:n] if b_out is not None else None)


def pct_order_blocks(plan: Plan, p: Protons, b: Optional[torch.Tensor], block: int):
    """Copy of the records (and b) with every block of `block` consecutive
    records ordered by (entry slice, t_in, input position): (Protons, b)."""
    dev = plan.device
    bufs = {k: torch.empty(p.n, dtype=torch.float32, device=dev) for k in FIELDS}
    b_out = torch.empty(p.n, dtype=torch.float32, device=dev) if b is not None else None
    out = _lib.make_protons_buf({k: v.data_ptr() for k, v in bufs.items()}, p.n)
    bp = _dev(b, "b", dtype=torch.float32, numel=p.n) if b is not None else None
    st = lib().pct_order_blocks(plan.handle, C.byref(p.s), bp, int(block), C.byref(out),
                                C.c_void_p(b_out.data_ptr()) if b_out is not None else None, _stream(dev))
    check(st, "pct_order_blocks")
    return Protons(bufs, device=dev), b_out


def pct_sort_scan(plan: Plan, p: Protons, b: Optional[torch.Tensor], n_angles: int, slab_mm: float,
                  with_perm: bool = False):
    """Copy of an acquisition-order scan sorted into angle bins: stable by
    (angle bin, slab of v_in, t_in), non-finite records last.  Returns
    (Protons, b or None, perm or None) with perm[j] the input position of
    output record j."""
    dev = plan.device
    nbytes = C.c_size_t()
    check(lib().pct_sort_scan_workspace_size(int(p.n), C.byref(nbytes)), "pct_sort_scan_workspace_size")
    ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    ws_ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    bufs = {k: torch.empty(p.n, dtype=torch.float32, device=dev) for k in FIELDS}
    b_out = torch.empty(p.n, dtype=torch.float32, device=dev) if b is not None else None
    perm = torch.empty(p.n, dtype=torch.int64, device=dev) if with_perm else None
    out = _lib.make_protons_buf({k: v.data_ptr() for k, v in bufs.items()}, p.n)
    bp = _dev(b, "b", dtype=torch.float32, numel=p.n) if b is not None else None
    opts = _lib.pct_sort_opts(int(n_angles), 0, float(slab_mm))
    st = lib().pct_sort_scan(plan.handle, C.byref(p.s), bp, C.byref(opts), C.byref(out),
                             C.c_void_p(b_out.data_ptr()) if b_out is not None else None,
                             C.c_void_p(perm.data_ptr()) if perm is not None else None, C.c_void_p(ws_ptr),
                             int(nbytes.value), _stream(dev))
    check(st, "pct_sort_scan")
    return Protons(bufs, device=dev), b_out, perm


def pct_select_slices(plan: Plan, src: torch.Tensor, src_z0: int, dst: torch.Tensor, dst_z0: int, z_first: int,
                      z_count: int):
    code = _dtype_code(src)
    if dst.dtype != src.dtype:
        raise TypeError("src and dst differ in dtype")
    plane = int(plan.grid.nx) * int(plan.grid.ny)
    sp = _dev(src, "src")
    dp = _dev(dst, "dst")
    if src.numel() < (z_first - src_z0 + z_count) * plane or dst.numel() < (z_first - dst_z0 + z_count) * plane:
        raise ValueError("volume too small for the requested slices")
    st = lib().pct_select_slices(plan.handle, sp, int(src_z0), dp, int(dst_z0), int(z_first), int(z_count), code,
                                 _stream(src.device))
    check(st, "pct_select_slices")
    return dst


def pct_slice_span_histogram(plan: Plan, p: Protons) -> torch.Tensor:
    """int64[nz]: protons per |exit slice - entry slice|."""
    hist = torch.zeros(plan.grid.nz, dtype=torch.int64, device=plan.device)
    st = lib().pct_slice_span_histogram(plan.handle, C.byref(p.s), C.c_void_p(hist.data_ptr()), plan.ws_ptr,
                                        plan.ws_bytes, _stream(plan.device))
    check(st, "pct_slice_span_histogram")
    return hist


def overlap_halo(hist: torch.Tensor, target: float = 0.96) -> int:
    """Smallest k with at least `target` of the counted protons spanning <= k
    slices (each region then reaches k slices past its core)."""
    c = torch.cumsum(hist.double().cpu(), 0)
    tot = float(c[-1])
    if tot <= 0:
        return 0
    return int(torch.nonzero(c >= target * tot)[0, 0])


def region_drop(plan: Plan, p: Protons, b: torch.Tensor, x: torch.Tensor, n_regions: int, halo: int, block: int,
                lam: float, n_iter: int, chord: str = "f64", lanes: int = 0, regions=None):
    """Algorithm 1 with DROP as the per-region solver, the regions run one
    after the other on this GPU.  x (the full volume) holds the initial iterate
    and receives the stitched result.  `regions` may carry the per-region
    state of an earlier call (plans and selected protons) to continue the
    iterations; returns it."""
    lay = pct_region_layout(plan.grid.nz, n_regions, halo)
    if regions is None:
        regions = []
        for z_lo, z_hi, c_lo, c_hi in lay:
            rp = plan.region(z_lo, z_hi)
            sub, b_sub = pct_region_select(plan, p, b, z_lo, z_hi)
            xr = torch.empty(rp.nvox, dtype=x.dtype, device=x.device)
            pct_select_slices(plan, x, 0, xr, z_lo, z_lo, z_hi - z_lo + 1)     # region's initial iterate
            regions.append({"layout": (z_lo, z_hi, c_lo, c_hi), "plan": rp, "protons": sub, "b": b_sub, "x": xr})
    for reg in regions:
        if reg["protons"].n:
            pct_drop_iterate(reg["plan"], reg["protons"], reg["b"], reg["x"], block, lam, n_iter, chord=chord,
                             lanes=lanes)
    for reg in regions:                                                      # selectSlice
        z_lo, _, c_lo, c_hi = reg["layout"]
        pct_select_slices(plan, reg["x"], z_lo, x, 0, c_lo, c_hi - c_lo + 1)
    return regions


@dataclass(frozen=True)
class FbpGeom:
    """Bins of the FBP initial iterate: n_angles angle bins over the full turn
    and n_t lateral bins [t0 + k dt, t0 + (k+1) dt) (mm); the slices of the
    plan's grid are the third axis."""
    n_angles: int
    n_t: int
    t0: float
    dt: float

    @staticmethod
    def for_grid(grid, n_angles: int, dt: Optional[float] = None) -> "FbpGeom":
        """Lateral bins of the voxel pitch covering the grid's diagonal,
        centred on the rotation axis."""
        dt = float(dt if dt is not None else min(grid.pitch[0], grid.pitch[1]))
        half = 0.5 * float(np.hypot(grid.nx * grid.pitch[0], grid.ny * grid.pitch[1]))
        n_t = 2 * int(np.ceil(half / dt))
        return FbpGeom(int(n_angles), n_t, -0.5 * n_t * dt, dt)

    def struct(self):
        return _lib.pct_fbp_geom(int(self.n_angles), int(self.n_t), float(self.t0), float(self.dt))


class FbpWorkspace:
    """Device scratch of the FBP entry points (256-byte aligned)."""

    def __init__(self, plan: Plan, geom: FbpGeom, device=None):
        nbytes = C.c_size_t()
        check(lib().pct_fbp_workspace_size(plan.handle, C.byref(geom.struct()), C.byref(nbytes)),
              "pct_fbp_workspace_size")
        self.nbytes = int(nbytes.value)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device or plan.device)
        self.ptr = C.c_void_p(self.buf.data_ptr() + (-self.buf.data_ptr()) % 256)


def pct_fbp_sinogram(plan: Plan, p: Protons, b: torch.Tensor, geom: FbpGeom, ws: Optional[FbpWorkspace] = None):
    """Mean WEPL and proton count per (slice, angle, lateral) bin."""
    dev = b.device
    bp = _dev(b, "b", dtype=torch.float32, numel=p.n)
    shape = (plan.grid.nz, geom.n_angles, geom.n_t)
    proj = torch.empty(shape, dtype=torch.float64, device=dev)
    count = torch.empty(shape, dtype=torch.int32, device=dev)
    ws = FbpWorkspace(plan, geom, dev) if ws is None else ws
    st = lib().pct_fbp_sinogram(plan.handle, C.byref(geom.struct()), C.byref(p.s), bp, proj.data_ptr(),
                                count.data_ptr(), ws.ptr, ws.nbytes, _stream(dev))
    check(st, "pct_fbp_sinogram")
    return proj, count


def pct_fbp_filter(plan: Plan, proj: torch.Tensor, geom: FbpGeom):
    """Ram-Lak filtered rows of a sinogram."""
    pp = _dev(proj, "proj", dtype=torch.float64, numel=plan.grid.nz * geom.n_angles * geom.n_t)
    q = torch.empty_like(proj)
    check(lib().pct_fbp_filter(plan.handle, C.byref(geom.struct()), pp, q.data_ptr(), _stream(proj.device)),
          "pct_fbp_filter")
    return q


def pct_fbp_backproject(plan: Plan, q: torch.Tensor, geom: FbpGeom, dtype=torch.float32):
    """FBP image (flat voxel order) from filtered rows."""
    qp = _dev(q, "q", dtype=torch.float64, numel=plan.grid.nz * geom.n_angles * geom.n_t)
    x = torch.empty(plan.nvox, dtype=dtype, device=q.device)
    check(lib().pct_fbp_backproject(plan.handle, C.byref(geom.struct()), qp, x.data_ptr(), _dtype_code(x),
                                    _stream(q.device)), "pct_fbp_backproject")
    return x


def pct_fbp(plan: Plan, p: Protons, b: torch.Tensor, geom: FbpGeom, dtype=torch.float32,
            x: Optional[torch.Tensor] = None, ws: Optional[FbpWorkspace] = None):
    """FBP image of the protons: the initial iterate of the DROP solve."""
    dev = b.device
    bp = _dev(b, "b", dtype=torch.float32, numel=p.n)
    x = torch.empty(plan.nvox, dtype=dtype, device=dev) if x is None else x
    xp = _dev(x, "x", numel=plan.nvox)
    ws = FbpWorkspace(plan, geom, dev) if ws is None else ws
    st = lib().pct_fbp(plan.handle, C.byref(geom.struct()), C.byref(p.s), bp, xp, _dtype_code(x), ws.ptr,
                       ws.nbytes, _stream(dev))
    check(st, "pct_fbp")
    return x


class DropSolver:
    """Block-iterative DROP over device-resident protons and WEPL data."""

    def __init__(self, plan: Plan, protons: Protons, b: torch.Tensor):
        self.plan, self.p, self.b = plan, protons, b

    def run(self, x: torch.Tensor, block: int, lam: float, n_iter: int, chord: str = "f64", **kw):
        return pct_drop_iterate(self.plan, self.p, self.b, x, block, lam, n_iter, chord=chord, **kw)


def tv_objective(plan: Plan, protons: Protons, b: torch.Tensor, x: torch.Tensor, beta: float, eps: float):
    """L(x) = 1/2 ||A x - b||^2 + beta TV_eps(x) as a torch graph over ProjectFn
    and TVFn (the residual norm is reduced in FP64)."""
    y = ProjectFn.apply(x, plan, protons)
    r = y.double() - b.double()
    return 0.5 * (r * r).sum() + beta * TVFn.apply(x, plan, eps).double()


def power_iteration(plan: Plan, protons: Protons, v0: torch.Tensor, n_steps: int = 20) -> float:
    """Largest eigenvalue of A^T A by n_steps power steps from the start vector
    v0 (forward and back projection kernels, in v0's dtype)."""
    dtype = v0.dtype
    v = v0.detach().clone()
    v /= torch.linalg.vector_norm(v)
    lam = 0.0
    for _ in range(n_steps):
        y = pct_forward(plan, protons, v)
        w = pct_backproject(plan, protons, y)
        lam = float(torch.linalg.vector_norm(w.double()))
        v = (w / lam).to(dtype)
    return lam


def tv_gradient_descent(plan: Plan, protons: Protons, b: torch.Tensor, x0: torch.Tensor, beta: float,
                        eps: float, n_steps: int, eta: Optional[float] = None, v0: Optional[torch.Tensor] = None,
                        power_steps: int = 20):
    """Fixed-step gradient descent on the TV-regularised least-squares
    objective; eta defaults to 1 / (lambda_max(A^T A) + 12 beta / eps) with the
    eigenvalue from power iteration started at v0.  Returns (x, losses, eta)."""
    if eta is None:
        if v0 is None:
            raise ValueError("eta or a power-iteration start vector v0 is required")
        eta = 1.0 / (power_iteration(plan, protons, v0, power_steps) + 12.0 * beta / eps)
    x = x0.detach().clone()
    losses = []
    for _ in range(n_steps):
        x.requires_grad_(True)
        loss = tv_objective(plan, protons, b, x, beta, eps)
        (g,) = torch.autograd.grad(loss, x)
        losses.append(float(loss))
        x = (x.detach() - eta * g).detach()
    return x, losses, eta

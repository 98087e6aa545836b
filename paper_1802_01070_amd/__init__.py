"""MI355X (gfx950) HIP implementation of the proton-CT reconstruction hot
path of arXiv:1802.01070: per-proton most-likely-path rows fused into the
block-iterative DROP update, behind the C ABI of include/pct.h.

Submodules:
  synth  -- seeded synthetic scans (the input generator; no method arithmetic)
  _lib   -- ctypes declarations of libpct.so
  api    -- PyTorch binding: pct_mlp_trace, pct_forward, pct_backproject,
            pct_drop_iterate, pct_tv, ProjectFn, TVFn, DropSolver
  build  -- hipcc build of libpct.so
"""

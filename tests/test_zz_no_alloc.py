"""pct_tv_static (no workspace: its partial sums live in the library's own
per-GPU array) against pct_tv (partial sums in the caller's workspace), through
the C ABI: bitwise the same value and gradient, on two calls in a row with
the second on a smaller grid, in FP64 and FP32, with and without the
gradient."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1802_01070_amd import api  # noqa: E402
from paper_1802_01070_amd.synth import Grid, MLPModel  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_tv_without_workspace_is_bitwise_the_workspace_variant(dtype):
    mlp = MLPModel(u_in=-40.0, u_out=40.0, step=1.0)
    # the first grid needs more partial sums (workgroups) than the second
    for k, grid in enumerate((Grid(96, 80, 40), Grid(30, 20, 6))):
        plan = api.Plan(grid, mlp, DEV)
        x = torch.from_numpy(np.random.default_rng(40 + k).uniform(0.2, 1.8, grid.nvox)).to(dtype).to(DEV)
        for with_grad in (True, False):
            v_ws, g_ws = api.pct_tv(plan, x, 1e-3, with_grad=with_grad)
            v_st, g_st = api.pct_tv_static(plan, x, 1e-3, with_grad=with_grad)
            torch.cuda.synchronize()
            assert torch.equal(v_ws, v_st), (k, with_grad, float(v_ws), float(v_st))
            assert float(v_st) > 0.0
            if with_grad:
                assert torch.equal(g_ws, g_st), k
        plan.close()

"""One plan shared by two host threads, each with its own workspace, stream and
iterate: the DROP calls race on the plan's cached sweep graph unless the
library serialises them; every result must equal the same call run alone."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1802_01070_amd import api, synth  # noqa: E402
from paper_1802_01070_amd._lib import PCT_DROP_FUSED_COMMIT  # noqa: E402

DEV = "cuda:0"


def test_two_streams_share_one_plan():
    c = synth.WORKLOADS[2]
    sc = synth.make_scan(c, m=48000)
    plan = api.Plan(sc.grid, sc.mlp, DEV)
    other = api.Plan(sc.grid, sc.mlp, DEV, _handle=plan.handle)     # same plan, second workspace
    pr = api.Protons(sc.protons, DEV)
    b = torch.from_numpy(sc.b).to(DEV)
    b2 = (b * 0.97).contiguous()
    jobs = [(plan, b, 0), (other, b2, 0), (plan, b, PCT_DROP_FUSED_COMMIT), (other, b2, PCT_DROP_FUSED_COMMIT)]
    # alone, one after the other
    ref = []
    for ws_plan, bb, flags in jobs:
        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
        for _ in range(2):
            api.pct_drop_iterate(ws_plan, pr, bb, x, block=c.block, lam=c.lam, n_iter=1, flags=flags)
        torch.cuda.synchronize()
        ref.append(x)
    # pairs of jobs on two threads, each on its own stream, repeatedly
    for rep in range(3):
        for pair in ((0, 1), (2, 3), (0, 3), (1, 2)):
            out = {}
            errors = []

            def run(k):
                try:
                    ws_plan, bb, flags = jobs[k]
                    st = torch.cuda.Stream()
                    with torch.cuda.stream(st):
                        x = torch.ones(sc.grid.nvox, dtype=torch.float32, device=DEV)
                        for _ in range(2):
                            api.pct_drop_iterate(ws_plan, pr, bb, x, block=c.block, lam=c.lam, n_iter=1, flags=flags)
                    st.synchronize()
                    out[k] = x
                except Exception as e:   # reported below
                    errors.append(e)

            th = [threading.Thread(target=run, args=(k,)) for k in pair]
            for t in th:
                t.start()
            for t in th:
                t.join()
            assert not errors, errors
            for k in pair:
                assert torch.equal(out[k], ref[k]), (rep, pair, k, (out[k] - ref[k]).abs().max().item())
    assert api.pct_device_status(plan) == 0 and api.pct_device_status(other) == 0
    other.handle = None          # the handle belongs to `plan`

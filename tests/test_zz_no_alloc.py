"""The allocation-free fraction to the boundary (mds_ftb_noalloc) against the
handle-based mds_ftb, through the C-ABI, on two calls in a row (the second
with a smaller input, so the partial records of the first are still in the
shared device array), then on an empty input."""
import numpy as np
import pytest

import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def _case(rng, n):
    v = 10.0 ** rng.uniform(-6, 1, n)
    dv = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)
    return v, dv


def test_ftb_noalloc_matches_handle_entry_point():
    import torch
    prob = synth.make_problem(8, 60, 10, 3, cfg=950)
    S = mds.solver_for(prob, nb=8)
    rng = np.random.default_rng(7)
    alpha = torch.full((1,), -7.0, dtype=torch.float64, device="cuda:0")
    for n, tau in ((1_000_003, 0.99), (777, 0.995)):
        v, dv = _case(rng, n)
        vt = torch.from_numpy(v).to("cuda:0")
        dvt = torch.from_numpy(dv).to("cuda:0")
        print(f"[gpu-case] ftb_noalloc n={n} tau={tau}", flush=True)
        mds.ftb_noalloc(vt, dvt, tau, alpha)
        torch.cuda.synchronize()
        a_noalloc = float(alpha.item())
        a_handle = S.ftb(vt, dvt, tau)
        assert a_noalloc == a_handle, (n, a_noalloc, a_handle)
        # the step of its definition, min(1, min over dv < 0 of -tau v / dv)
        neg = dv < 0
        ref = min(1.0, float(np.min(-tau * v[neg] / dv[neg]))) if neg.any() else 1.0
        assert a_noalloc == ref
    # no entry: alpha = 1
    empty = torch.empty(0, dtype=torch.float64, device="cuda:0")
    mds.ftb_noalloc(empty, empty, 0.99, alpha)
    torch.cuda.synchronize()
    assert float(alpha.item()) == 1.0
    # every step positive: alpha = 1
    v = torch.ones(5000, dtype=torch.float64, device="cuda:0")
    mds.ftb_noalloc(v, v, 0.99, alpha)
    torch.cuda.synchronize()
    assert float(alpha.item()) == 1.0

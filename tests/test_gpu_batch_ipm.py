"""Batched whole IPMs (mds_batch_ipm: every problem of the scenario batch an
IPM of Sec. 2.1 run by one workgroup of a persistent kernel) against the
oracle's IPM of each problem, through the C-ABI.

Per problem: the same status and number of iterations, the same barrier
parameter, inertia, correction trials and backtracks in every iteration,
and the final x and y within 1e-8 of the oracle's; the final point passes
the optimality test recomputed in numpy.  Shapes: the scenario recipe
(n_d = N/4, m = 3N/4, n_s = 50 N, 4 nonzeros per row of J_s) at small N, a
nonconvex member whose correction loop fires, and sizes spanning the
register rows of the batch kernel's panel (N up to 1100)."""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth
from helpers import dense_js

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _scenario(N, p, s_scale=1.0, ns_per=50):
    return synth.make_problem(N // 4, ns_per * N, 3 * N // 4, 4, cfg=3, p=p, s_scale=s_scale)


def _compare(probs, sols, res):
    for p, q in enumerate(probs):
        r_o = oracle.ipm(oracle.Problem(q))
        r_g = res[p]
        assert r_g["status"] == r_o["status"] == "converged", (p, r_g["status"], r_o["status"])
        assert r_g["iters"] == r_o["iters"], (p, r_g["iters"], r_o["iters"])
        for k in range(r_o["iters"]):
            a, b = r_g["trace"][k], r_o["trace"][k]
            assert a["mu"] == pytest.approx(b["mu"], rel=1e-10), (p, k)
            assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], (p, k)
            assert a["backtracks"] == b["backtracks"], (p, k)
        x, y, zl, zu = sols[p]
        assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max()), p
        assert np.abs(y - r_o["y"]).max() <= 1e-8 * max(1.0, np.abs(r_o["y"]).max()), p
        # optimality recomputed from the problem data
        nd, m = q["n_d"], q["m"]
        A = np.hstack([np.asarray(q["Jd"]).reshape(m, nd), dense_js(q)])
        assert np.abs(A @ x - q["b"]).max() <= 1e-7
        gf = np.concatenate([q["H"] @ x[:nd] + q["c"], q["w"] * x[nd:] + q["g"]])
        st = gf + A.T @ y - zl + zu
        sd = max(1.0, (np.abs(y).sum() + zl.sum() + zu.sum()) / (m + 2 * len(x)) / 100.0)
        assert np.abs(st).max() <= 1e-8 * sd * 10


def test_batch_ipm_matches_oracle_small():
    probs = [_scenario(N, p, ns_per=10) for p, N in enumerate((64, 96, 128, 160, 200, 256))]
    probs.append(_scenario(128, 51, s_scale=6.0, ns_per=10))  # nonconvex: correction fires
    probs.append(_scenario(128, 58, s_scale=12.0, ns_per=10))
    say(f"batch ipm {len(probs)} problems, N = 64..256")
    B = mds.BatchIPM(probs, max_iter=200)
    res = B.solve()
    assert max(t["trials"] for t in res[-2]["trace"]) > 1
    assert max(t["trials"] for t in res[-1]["trace"]) > 1
    _compare(probs, [B.solution(p) for p in range(len(probs))], res)
    # a second run on the same batch repeats every result bit for bit
    x0 = [B.solution(p)[0].copy() for p in range(len(probs))]
    res2 = B.solve()
    assert [r["iters"] for r in res2] == [r["iters"] for r in res]
    for p in range(len(probs)):
        assert np.array_equal(B.solution(p)[0], x0[p])
    B.close()


def test_batch_ipm_matches_oracle_register_rows():
    probs = [_scenario(N, 10 + p, ns_per=4) for p, N in enumerate((516, 1100))]
    say("batch ipm N = 516, 1100")
    B = mds.BatchIPM(probs, max_iter=200, grid=2)
    res = B.solve()
    _compare(probs, [B.solution(p) for p in range(len(probs))], res)
    B.close()


def test_batch_ipm_state_errors():
    probs = [_scenario(64, 0, ns_per=4)]
    say("batch ipm state errors")
    B = mds.BatchIPM(probs, max_iter=20)
    with pytest.raises(mds.MdsError):
        B.solve(max_iter=50)   # beyond the trace rows the workspace holds
    res = B.solve(max_iter=3)
    assert res[0]["status"] == "maxiter" and res[0]["iters"] == 3
    B.close()

"""Look-ahead of the cooperative FP64 factorization (the next panel beside
the trailing update, on CU-masked streams) through the C-ABI.

Panel b + 1 computes the entries of a candidate column (Bunch-Kaufman's
second test, Sec. 2.3) that lie outside the strip the near update wrote
from panel b's input and multipliers; these matrices make it do so on most
pivot steps.  Bars: the pivot sequence is the oracle's, the inertia too, and
the factorization equals the sequential one (same pivots; solutions within
1e-12); the automatic choice and the option's bounds behave as documented.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _dense_problem(A):
    N = A.shape[0]
    return dict(n_d=N, n_s=0, m=0, r=0, H=np.asfortranarray(A), c=np.zeros(N), w=np.zeros(0),
                g=np.zeros(0), Jd=np.zeros((0, N)), rp=np.zeros(1, dtype=np.int32),
                ci=np.zeros(0, dtype=np.int32), v=np.zeros(0), b=np.zeros(0),
                xl=-np.ones(N), xu=np.ones(N))


def _weak_diag(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    return 0.5 * (A + A.T) * np.where(np.eye(N) > 0, 0.01, 1.0)


@pytest.mark.parametrize("N,seed", [(1500, 21), (3000, 22), (4100, 23)])
def test_lookahead_pivots_match_oracle(N, seed):
    A = _weak_diag(N, seed)
    say(f"look-ahead dense N={N}")
    S = mds.solver_for(_dense_problem(A), panel="coop", lookahead="on")
    assert S.info()["lookahead_cus"] > 0
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    _, inn, _ = S.factor_inertia()
    _, _, _, ipo, _, _ = oracle.bk(A)
    piv = S.get_pivots()
    assert np.array_equal(piv, ipo), int((piv != ipo).sum())
    ev = np.linalg.eigvalsh(A)
    assert (inn["npos"], inn["nneg"], inn["nzero"]) == (int((ev > 0).sum()), int((ev < 0).sum()), 0)
    st = S.panel_stats()
    # most steps take the second test: the look-ahead's own column entries are exercised
    assert st["coop_second"] > st["coop_steps"] // 2
    assert S.fallbacks()["coop_aborts"] == 0


def test_lookahead_equals_sequential_on_kkt():
    prob = synth.config_problem(synth.OPF_N4096)
    st = synth.kkt_state(prob, 2)
    res = {}
    for la in ("off", "on"):
        say(f"KKT N=4096 lookahead={la}")
        S = mds.solver_for(prob, lookahead=la)
        assert (S.info()["lookahead_cus"] > 0) == (la == "on")
        S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
        _, inn, _ = S.factor_inertia(1e-8)
        x = np.concatenate([t.cpu().numpy() for t in S.solve(st["r_d"], st["r_s"], st["r_y"])])
        res[la] = (S.get_pivots(), inn, x)
        # a second factorization of the same handle reuses its streams
        S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
        _, inn2, _ = S.factor_inertia(1e-8)
        assert inn2 == inn
        assert np.array_equal(S.get_pivots(), res[la][0])
        del S
    (p0, i0, x0), (p1, i1, x1) = res["off"], res["on"]
    assert np.array_equal(p0, p1) and i0 == i1
    assert np.abs(x1 - x0).max() <= 1e-12 * np.abs(x0).max()


def test_lookahead_whole_ipm_matches_sequential():
    prob = synth.config_problem(synth.OPF_N4096)
    out = {}
    for la in ("off", "on"):
        say(f"whole IPM N=4096 lookahead={la}")
        S = mds.solver_for(prob, lookahead=la)
        r = S.ipm_solve()
        assert r["status"] == "converged"
        out[la] = (r["iters"], [t["inertia"] for t in r["trace"][:r["iters"]]],
                   r["x"].cpu().numpy())
        del S
    assert out["on"][0] == out["off"][0] and out["on"][1] == out["off"][1]
    x0 = out["off"][2]
    assert np.abs(out["on"][2] - x0).max() <= 1e-8 * max(1.0, np.abs(x0).max())


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_lookahead_fp32_storage_matches_sequential(precision):
    """FP32 storage of the trailing matrix: the look-ahead panel computes its
    candidate entries from the previous FP32 buffer and rounds them to FP32;
    inertia and the refined solution match the sequential order's."""
    prob = synth.config_problem(synth.OPF_N4096)
    st = synth.kkt_state(prob, 2)
    res = {}
    for la in ("off", "on"):
        say(f"KKT N=4096 {precision} lookahead={la}")
        S = mds.solver_for(prob, precision=precision, lookahead=la)
        assert (S.info()["lookahead_cus"] > 0) == (la == "on")
        S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
        _, inn, _ = S.factor_inertia(1e-8)
        sol, ri = S.refine(st["r_d"], st["r_s"], st["r_y"], 10, 1e-14)
        assert ri["eta"] <= 1e-14
        res[la] = (S.get_pivots(), inn, np.concatenate([t.cpu().numpy() for t in sol]))
        del S
    (p0, i0, x0), (p1, i1, x1) = res["off"], res["on"]
    assert i0 == i1
    assert np.mean(p0 == p1) > 0.999
    # two different FP32 factors, each refined to backward error 1e-14: they
    # agree to this system's conditioning (an FP32 factor's refined solution
    # lies ~1e-8 from the FP64 one here), the bar of the mixed IPM tests
    assert np.abs(x1 - x0).max() <= 1e-7 * np.abs(x0).max()


def test_lookahead_automatic_choice_and_bounds():
    prob = synth.config_problem(synth.OPF_N4096)
    say("look-ahead automatic choice")
    assert mds.solver_for(prob).info()["lookahead_cus"] == 0          # N = 4096 < 8192
    assert mds.solver_for(prob, precision="fp32").info()["lookahead_cus"] == 0
    # only the cooperative panel has a look-ahead form
    assert mds.solver_for(prob, panel="mem", lookahead="on").info()["lookahead_cus"] == 0
    with pytest.raises(mds.MdsError):
        mds.Solver(8, 10, 4, 10, lookahead="sometimes")

"""Inequality rows (Sec. 2, eq. (ineq)) on the GPU against the CPU oracle,
through the C-ABI.

The last m_I rows of J are hl <= (J x) <= hu.  The IPM carries one bounded
slack per row; its Newton step eliminates the slack step into the (4,4)
block 1/(Sigma_h + dw) of eq. (linsys4x4), which the condensation places on
the diagonal of M22 (Sec. 2.2, eq. (compressed)).

Bars: the barrier diagonal is bit-exact and the right-hand side within
n eps of the oracle's (element-wise, same operations); whole IPMs take the
same number of iterations as the oracle with the same per-iteration barrier
parameter, inertia, correction trials and backtracks, and end within 1e-8 of
the oracle's x, d and y; invalid bounds are rejected before any work.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _interior(prob, seed):
    it = synth.interior_iterate(prob, seed)
    rng = np.random.default_rng(seed + 50)
    hl, hu = prob["hl"], prob["hu"]
    mid = np.where(np.isfinite(hl) & np.isfinite(hu), 0.5 * (hl + hu),
                   np.where(np.isfinite(hl), hl + 0.3, hu - 0.3))
    d = mid + 0.05 * rng.standard_normal(len(mid))
    vl = np.where(np.isfinite(hl), 10.0 ** rng.uniform(-2, 1, len(d)), 0.0)
    vu = np.where(np.isfinite(hu), 10.0 ** rng.uniform(-2, 1, len(d)), 0.0)
    return (np.concatenate([it["x"], d]), it["y"], np.concatenate([it["zl"], vl]),
            np.concatenate([it["zu"], vu]), it["mu"])


def test_vector_kernels_with_slacks():
    prob = synth.make_problem(40, 700, 60, 4, cfg=340, m_I=25)
    X, y, ZL, ZU, mu = _interior(prob, 1)
    say("slack vector kernels N=100, m_I=25")
    S = mds.solver_for(prob, nb=8)
    P = oracle.Problem(prob)
    sig, rx, ry = [_np(t) for t in S.sigma_rhs(X, y, ZL, ZU, mu)]
    so, rxo, ryo = oracle.sigma_rhs(P, X, y, ZL, ZU, mu)
    assert len(sig) == P.nx
    assert np.array_equal(sig.view(np.int64), so.view(np.int64))
    assert np.abs(rx - rxo).max() <= 1e-12 * max(1.0, np.abs(rxo).max())
    assert np.abs(ry - ryo).max() <= 1e-12 * max(1.0, np.abs(ryo).max())
    E, _ = S.opt_error(X, y, ZL, ZU, mu)
    Eo, _ = oracle.opt_error(P, X, y, ZL, ZU, mu)
    assert E == pytest.approx(Eo, rel=1e-12)
    f, phi, th = S.merit(X, mu)
    assert phi == pytest.approx(oracle.barrier(P, X, mu), rel=1e-12)
    assert th == pytest.approx(oracle.theta(P, X), rel=1e-12)


def _ipm_compare(prob, nb=0, warm=None):
    P = oracle.Problem(prob)
    r_o = oracle.ipm(P, warm=warm)
    S = mds.solver_for(prob, nb=nb)
    if warm is None:
        r_g = S.ipm_solve()
    else:
        r_g = S.ipm_solve_warm(warm["x_d"], warm["y"], warm["mu0"])
    assert r_g["status"] == r_o["status"] == "converged", (r_g["status"], r_o["status"])
    assert r_g["iters"] == r_o["iters"]
    for k in range(r_o["iters"]):
        a, b = r_g["trace"][k], r_o["trace"][k]
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-10), k
        assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], k
        assert a["backtracks"] == b["backtracks"], k
    x, y = _np(r_g["x"]), _np(r_g["y"])
    assert len(x) == P.nx
    assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())
    assert np.abs(y - r_o["y"]).max() <= 1e-8 * max(1.0, np.abs(r_o["y"]).max())
    return r_g, r_o


IPM_CASES = [
    # (n_d, n_s, m, r, m_I, s_scale)
    (64, 2000, 128, 4, 64, 1.0),     # the N = 192 shape, half the rows inequalities
    (64, 2000, 128, 4, 40, 6.0),     # nonconvex: the correction loop fires
    (32, 800, 64, 4, 64, 1.0),       # every row an inequality (m_E = 0)
    (20, 0, 30, 0, 10, 1.0),         # n_s = 0
    (0, 400, 50, 3, 20, 1.0),        # n_d = 0
]


@pytest.mark.parametrize("case", range(len(IPM_CASES)))
def test_ipm_with_inequalities_matches_oracle(case):
    nd, ns, m, r, mI, sc = IPM_CASES[case]
    prob = synth.make_problem(nd, ns, m, r, cfg=341, p=case, s_scale=sc, m_I=mI)
    say(f"ipm with inequality rows {IPM_CASES[case]}")
    r_g, r_o = _ipm_compare(prob)
    # some inequality row binds at the solution
    if ns > 0:
        assert np.abs(r_o["y"][m - mI:]).max() > 1e-6
    if sc > 1.0:
        assert max(t["trials"] for t in r_g["trace"]) > 1


def test_ipm_with_inequalities_warm_start_matches_oracle():
    prob = synth.make_problem(64, 2000, 128, 4, cfg=342, m_I=48)
    r_cold = oracle.ipm(oracle.Problem(prob))
    rng = np.random.default_rng(3)
    warm = dict(x_d=r_cold["x"][:64] + 0.05 * rng.standard_normal(64),
                y=r_cold["y"] * (1.0 + 0.05 * rng.standard_normal(128)), mu0=1e-3)
    say("warm ipm with inequality rows")
    _ipm_compare(prob, warm=warm)


def test_inequality_bounds_validated():
    prob = synth.make_problem(4, 10, 5, 2, cfg=343, m_I=3)
    say("inequality bound validation")
    S = mds.Solver(4, 10, 5, len(prob["v"]), nb=8, m_I=3)
    for hl, hu in ((prob["hu"], prob["hu"]), (np.full(3, -np.inf), np.full(3, np.inf)),
                   (np.array([0.0, np.nan, 0.0]), np.ones(3))):
        bad = dict(prob)
        bad["hl"], bad["hu"] = hl, hu
        with pytest.raises(mds.MdsError, match="nonpositive"):
            S.set_problem(bad)
    S.set_problem(prob)


def test_caller_diagonal_blocks_the_ipm_and_set_problem_clears_it():
    prob = synth.make_problem(8, 60, 10, 3, cfg=344)
    say("m22 diagonal vs IPM state")
    S = mds.solver_for(prob, nb=8)
    S.set_m22_diag(np.full(10, 0.5))
    it = S.new_iterate()
    with pytest.raises(mds.MdsError, match="call order"):
        S.ipm_init(it)
    S.set_problem(prob)  # clears the caller's diagonal
    S.ipm_init(it)
    r = S.ipm_solve()
    assert r["status"] == "converged"

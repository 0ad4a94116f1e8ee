"""GPU parity of the HIP path against the CPU oracle, through the C-ABI.

Bars:
* condensation: bit-exact M and D_s^{-1} (integer-style equality of doubles);
* Bunch-Kaufman: pivot sequence (ipiv) and inertia identical; L and D equal
  to the oracle's within a tolerance derived from the growth-bounded
  backward stability of BK (both factor the same bits of M);
* solve: relative difference <= 1e-8 against the oracle's solve, and the
  refined solution's normwise backward error on the full KKT system <= 1e-10;
* vector kernels: fraction-to-boundary bit-exact (a min is order-free); sums
  within n * eps of their l1 magnitude;
* IPM: same status, iteration count and per-iteration inertia/trial counts
  as the oracle; final x, y within 1e-8.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth
from helpers import block_d, full_kkt, perm_from_ipiv

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _np(t):
    return t.detach().cpu().numpy()


CASES = [
    # (n_d, n_s, m, r, nb, log-range of the barrier diagonals)
    (64, 2000, 128, 4, 0, (-1.0, 1.0)),     # the N = 192 workload shape
    (10, 40, 27, 3, 8, (-1.0, 1.0)),        # N = 37: ragged panels
    (100, 900, 200, 4, 16, (-2.0, 2.0)),    # N = 300: many panels, ragged tail
    (150, 3000, 550, 6, 32, (-3.0, 3.0)),   # N = 700, wider panels
    (0, 50, 40, 3, 8, (-1.0, 1.0)),         # n_d = 0: M = M22 only
    (33, 0, 20, 0, 8, (-1.0, 1.0)),         # n_s = 0: no Schur term
    (45, 30, 0, 2, 16, (-1.0, 1.0)),        # m = 0: M = H + Sigma_d
]


def _case(idx, seed=0):
    nd, ns, m, r, nb, lr = CASES[idx]
    prob = synth.make_problem(nd, ns, m, r, cfg=300 + idx, p=seed)
    st = synth.kkt_state(prob, seed, lr)
    return prob, st, nb


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("shifts", [(0.0, 0.0), (3e-3, 2e-7)])
def test_condense_bit_exact(idx, shifts):
    prob, st, nb = _case(idx)
    say(f"condense case={CASES[idx]} shifts={shifts}")
    S = mds.solver_for(prob, nb=nb)
    S.condense(st["sigma_d"], st["dsbase"], *shifts)
    M = S.get_matrix()
    Mo, invo = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], *shifts)
    assert np.array_equal(M.view(np.int64), Mo.view(np.int64))
    assert np.array_equal(S.get_inv_ds().view(np.int64), invo.view(np.int64))


def _factor_check(S, Mo):
    N = Mo.shape[0]
    L, dd, ds, ipiv = S.get_factor()
    Lo, ddo, dso, ipo, info_o, _ = oracle.bk(Mo)
    assert np.array_equal(ipiv, ipo), f"first differing pivot {np.argmax(ipiv != ipo)}"
    scale = max(1.0, np.abs(Mo).max())
    tol = 1e-10 * scale * max(1.0, np.abs(Lo).max()) ** 2
    assert np.abs(dd - ddo).max() <= tol
    assert np.abs(ds - dso).max() <= tol
    assert np.abs(L - Lo).max() <= 1e-10 * max(1.0, np.abs(Lo).max()) * scale
    # the GPU factor reproduces its own input
    p = perm_from_ipiv(ipiv)
    R = L @ block_d(ipiv, dd, ds) @ L.T
    assert np.abs(R - Mo[np.ix_(p, p)]).max() <= 1e-11 * N * scale * max(1.0, np.abs(L).max()) ** 2
    return oracle.inertia(ipo, ddo, dso), info_o


PANELS = {"auto": dict(panel="auto"), "mem": dict(panel="mem"), "reg": dict(panel="reg"),
          "reg512": dict(panel="reg", panel_threads=512),
          "reg1024": dict(panel="reg", panel_threads=1024), "coop": dict(panel="coop"),
          "lds": dict(panel="lds")}
LDS_MAX_N = 199


@pytest.mark.parametrize("panel", list(PANELS))
@pytest.mark.parametrize("idx", range(len(CASES)))
def test_factor_pivots_and_inertia_exact(idx, panel):
    prob, st, nb = _case(idx, seed=1)
    if panel == "lds" and prob["n_d"] + prob["m"] > LDS_MAX_N:
        pytest.skip("the LDS factorization holds N <= 199")
    say(f"factor case={CASES[idx]} panel={panel}")
    if panel in ("reg1024", "coop") and nb > 32:
        nb = 32
    S = mds.solver_for(prob, nb=nb, **PANELS[panel])
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    Mo, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 0.0, 0.0)
    status, inn, _ = S.factor_inertia()
    ino, info_o = _factor_check(S, Mo)
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == ino
    assert inn["info"] == info_o
    assert status == (mds.MDS_ZERO_PIVOT if info_o else mds.MDS_OK)


def _dense_problem(A):
    """A problem whose condensed matrix is exactly A (m = n_s = 0, Sigma_d = 0)."""
    N = A.shape[0]
    return dict(n_d=N, n_s=0, m=0, r=0, H=np.asfortranarray(A), c=np.zeros(N), w=np.zeros(0),
                g=np.zeros(0), Jd=np.zeros((0, N)), rp=np.zeros(1, dtype=np.int32),
                ci=np.zeros(0, dtype=np.int32), v=np.zeros(0), b=np.zeros(0),
                xl=-np.ones(N), xu=np.ones(N))


BRANCHES = [
    np.array([[4.0, 1.0], [1.0, 3.0]]),
    np.array([[1.0, 2.0, 0.0], [2.0, 0.0, 10.0], [0.0, 10.0, 0.0]]),
    np.array([[0.1, 2.0, 0.0], [2.0, 5.0, 1.0], [0.0, 1.0, 1.0]]),
    np.array([[0.0, 1.0], [1.0, 0.0]]),
    np.array([[0.0, 0.5, 2.0], [0.5, 1.0, 0.3], [2.0, 0.3, 0.0]]),
    np.diag([3.0, 0.0, -2.0, 5.0]),
]


@pytest.mark.parametrize("case", range(len(BRANCHES)))
def test_factor_branch_matrices(case):
    A = BRANCHES[case]
    say(f"branch case={case}")
    S = mds.solver_for(_dense_problem(A), nb=8)
    S.condense(np.zeros(A.shape[0]), np.zeros(0), 0.0, 0.0)
    status, inn, _ = S.factor_inertia()
    ino, info_o = _factor_check(S, A)
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == ino
    assert inn["info"] == info_o


@pytest.mark.parametrize("panel", list(PANELS))
@pytest.mark.parametrize("N,nb", [(64, 8), (129, 16), (250, 16), (400, 64), (700, 0),
                                  (1300, 0), (2100, 0), (3000, 0)])
def test_factor_random_symmetric(N, nb, panel):
    if panel == "lds" and N > LDS_MAX_N:
        pytest.skip("the LDS factorization holds N <= 199")
    rng = np.random.default_rng(N)
    A = rng.standard_normal((N, N))
    A = A + A.T
    say(f"random symmetric N={N} nb={nb} panel={panel}")
    S = mds.solver_for(_dense_problem(A), nb=nb, **PANELS[panel])
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    status, inn, _ = S.factor_inertia()
    ino, _ = _factor_check(S, A)
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == ino


def _panel_widths(ipiv, N, nb):
    """Column counts of the memory panel's panels: a panel ends once nb
    columns are done, so a 2x2 pivot on its last column makes it nb + 1 wide."""
    out, k = [], 0
    while k < N:
        k0, j = k, 0
        while j < nb and k < N:
            s = 2 if ipiv[k] < 0 else 1
            k += s
            j += s
        out.append(k - k0)
    return out


@pytest.mark.parametrize("N,seed", [(400, 102), (700, 100)])
def test_solve_widest_panels(N, seed):
    """Memory panel with nb = 64 on random symmetric matrices whose pivot
    sequence ends several panels with a 2x2 pivot (65 columns, more pivot
    entries than one wave has lanes in the standard form's sweep): the
    solution equals the oracle's."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    A = A + A.T
    say(f"widest panels N={N} seed={seed}")
    prob = _dense_problem(A)
    S = mds.solver_for(prob, nb=64, panel="mem")
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    S.factor_inertia()
    _factor_check(S, A)
    _, _, _, ipiv = S.get_factor()
    assert 65 in _panel_widths(ipiv, N, 64)
    r = rng.standard_normal(N)
    dx = _np(S.solve(r, np.zeros(0), np.zeros(0))[0])
    F = oracle.Factor(oracle.Problem(prob)).once(np.zeros(N), np.zeros(0), 0.0, 0.0)
    od = F.solve(r, np.zeros(0), np.zeros(0))[0]
    # both solves use the same pivots; their factors agree to rounding, so the
    # solutions agree to about cond(A) times that
    assert np.abs(dx - od).max() <= 1e-13 * np.linalg.cond(A) * np.abs(od).max()


@pytest.mark.parametrize("idx", [0, 1, 2, 3, 4, 5, 6])
def test_solve_and_refine(idx):
    prob, st, nb = _case(idx, seed=2)
    say(f"solve case={CASES[idx]}")
    S = mds.solver_for(prob, nb=nb)
    S.condense(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    S.factor_inertia()
    dx_d, dx_s, dy = [_np(t) for t in S.solve(st["r_d"], st["r_s"], st["r_y"])]
    P = oracle.Problem(prob)
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    got, ref = np.concatenate([dx_d, dx_s, dy]), np.concatenate([od, os_, oy])
    assert np.abs(got - ref).max() <= 1e-8 * max(np.abs(ref).max(), 1e-300)
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 5, 1e-14)
    assert info["eta"] <= 1e-10
    if prob["n_d"] + prob["n_s"] + prob["m"] <= 2500:
        K = full_kkt(prob, st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
        r = np.concatenate([st["r_d"], st["r_s"], st["r_y"]])
        x = np.concatenate([_np(rd), _np(rs), _np(ry)])
        eta = np.abs(r - K @ x).max() / (np.abs(K).sum(1).max() * np.abs(x).max() + np.abs(r).max())
        assert eta <= 1e-10


def test_correction_loop_closed_form():
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "correction_loop.json")))
    prob = synth.make_problem(4, 3, 0, 2, cfg=106)
    prob["H"] = -2.0 * np.eye(4)
    say("correction loop closed form")
    S = mds.solver_for(prob, nb=8)
    S.condense(np.zeros(4), prob["w"], 0.0, 0.0)
    reg = dict(delta_w_last=0.0)
    for call in gold["calls"]:
        st, inn, out = S.factor_inertia(mu=1e-2, reg=reg)
        assert st == 0
        assert out["trials"] == call["trials"]
        assert out["delta_w_last"] == pytest.approx(call["dw_num"] / call["dw_den"], rel=1e-12)
        assert (inn["npos"], inn["nzero"], inn["nneg"]) == (4, 0, 0)
        reg = dict(delta_w_last=out["delta_w_last"])


def test_correction_loop_matches_oracle_on_singular_system():
    prob = synth.make_problem(4, 10, 3, 2, cfg=108)
    prob["H"] = np.eye(4)
    prob["rp"] = np.array([0, 2, 4, 6], dtype=np.int32)
    prob["ci"] = np.array([1, 5, 1, 5, 2, 7], dtype=np.int32)
    prob["v"] = np.array([2.0, 2.0, 2.0, 2.0, -1.0, 0.5])
    prob["Jd"] = np.asfortranarray(np.vstack([np.ones(4), np.ones(4), np.arange(4.0)]))
    say("correction loop singular")
    S = mds.solver_for(prob, nb=8)
    sd, db = np.ones(4), np.full(10, 4.0)
    S.condense(sd, db, 0.0, 0.0)
    st, inn, _ = S.factor_inertia()
    assert inn["nzero"] == 1 and st == mds.MDS_ZERO_PIVOT
    st, inn, out = S.factor_inertia(mu=1e-4, reg=dict(delta_w_last=0.0))
    F = oracle.Factor(oracle.Problem(prob))
    sto, dwl = F.correct(sd, db, 1e-4, 0.0)
    assert st == sto == 0
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == F.inertia
    assert out["delta_c"] == F.s.dc and out["delta_w"] == F.s.dw and out["trials"] == F.s.trials


# ------------------------------------------------------------- vector kernels
@pytest.mark.parametrize("seed", [0, 1])
def test_vector_kernels(seed):
    prob = synth.make_problem(40, 700, 60, 4, cfg=320, p=seed)
    it = synth.interior_iterate(prob, seed)
    say(f"vector kernels seed={seed}")
    S = mds.solver_for(prob, nb=8)
    P = oracle.Problem(prob)
    sig, rx, ry = [_np(t) for t in S.sigma_rhs(it["x"], it["y"], it["zl"], it["zu"], it["mu"])]
    so, rxo, ryo = oracle.sigma_rhs(P, it["x"], it["y"], it["zl"], it["zu"], it["mu"])
    assert np.array_equal(sig.view(np.int64), so.view(np.int64))  # element-wise, same ops
    assert np.abs(rx - rxo).max() <= 1e-12 * max(1.0, np.abs(rxo).max())
    assert np.abs(ry - ryo).max() <= 1e-12 * max(1.0, np.abs(ryo).max())
    E, parts = S.opt_error(it["x"], it["y"], it["zl"], it["zu"], it["mu"])
    Eo, po = oracle.opt_error(P, it["x"], it["y"], it["zl"], it["zu"], it["mu"])
    assert E == pytest.approx(Eo, rel=1e-12)
    f, phi, th = S.merit(it["x"], it["mu"])
    assert f == pytest.approx(oracle.objective(P, it["x"]), rel=1e-12)
    assert phi == pytest.approx(oracle.barrier(P, it["x"], it["mu"]), rel=1e-12)
    assert th == pytest.approx(oracle.theta(P, it["x"]), rel=1e-12)
    rng = np.random.default_rng(seed)
    v = 10.0 ** rng.uniform(-3, 1, 5000)
    dv = rng.standard_normal(5000) * 10.0 ** rng.uniform(-2, 2, 5000)
    assert S.ftb(v, dv, 0.99) == oracle.ftb(v, dv, 0.99)
    assert S.ftb(v, np.abs(dv), 0.99) == 1.0


# ------------------------------------------------------------------------ IPM
def _ipm_compare(prob, nb=0, rows_equal=True):
    r_o = oracle.ipm(oracle.Problem(prob))
    S = mds.solver_for(prob, nb=nb)
    r_g = S.ipm_solve()
    assert r_g["status"] == r_o["status"] == "converged"
    assert r_g["iters"] == r_o["iters"]
    for k in range(r_o["iters"]):
        a, b = r_g["trace"][k], r_o["trace"][k]
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-10)
        if rows_equal:
            assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], k
            assert a["backtracks"] == b["backtracks"], k
    x, y = _np(r_g["x"]), _np(r_g["y"])
    assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())
    assert np.abs(y - r_o["y"]).max() <= 1e-8 * max(1.0, np.abs(r_o["y"]).max())
    return r_g, r_o


def test_ipm_config0_matches_oracle():
    say("ipm N=192 workload")
    _ipm_compare(synth.config_problem(synth.IPM_N192))


def test_ipm_nonconvex_correction_fires():
    prob = synth.make_problem(64, 2000, 128, 4, cfg=0, p=1, s_scale=6.0)
    say("ipm nonconvex variant")
    r_g, r_o = _ipm_compare(prob)
    assert max(t["trials"] for t in r_g["trace"]) > 1


@pytest.mark.parametrize("seed", [3, 4])
def test_ipm_other_seeds(seed):
    prob = synth.make_problem(32, 800, 64, 4, cfg=202, p=seed)
    say(f"ipm seed={seed}")
    _ipm_compare(prob, nb=8)


def test_problem_validation_errors():
    prob = synth.make_problem(4, 10, 3, 2, cfg=330)
    say("validation")
    S = mds.Solver(4, 10, 3, len(prob["v"]), nb=8)
    bad = dict(prob)
    bad["w"] = prob["w"].copy()
    bad["w"][2] = -1.0
    with pytest.raises(mds.MdsError, match="nonpositive"):
        S.set_problem(bad)
    bad = dict(prob)
    bad["ci"] = prob["ci"].copy()
    bad["ci"][0], bad["ci"][1] = bad["ci"][1], bad["ci"][0]
    with pytest.raises(mds.MdsError, match="pattern"):
        S.set_problem(bad)
    bad = dict(prob)
    bad["b"] = prob["b"].copy()
    bad["b"][0] = np.nan
    with pytest.raises(mds.MdsError, match="non-finite"):
        S.set_problem(bad)
    S.set_problem(prob)
    with pytest.raises(mds.MdsError, match="call order"):
        S.solve(np.zeros(4), np.zeros(10), np.zeros(3))


@pytest.mark.parametrize("N", [1025, 2049, 4097])
def test_cooperative_panel_workgroup_boundaries(N):
    # one row past a multiple of 1024: the last workgroup owns a single row
    rng = np.random.default_rng(N)
    A = rng.standard_normal((N, N))
    A = A + A.T
    say(f"cooperative panel N={N} vs oracle")
    S = mds.solver_for(_dense_problem(A), panel="coop")
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    status, inn, _ = S.factor_inertia()
    ino, _ = _factor_check(S, A)
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == ino


@pytest.mark.parametrize("N", [2049, 3000])
def test_automatic_panel_register_tail(N):
    # above N = 2048 the automatic choice runs the cooperative panel and hands
    # over to the one-workgroup register panel for the last (<= 1024) rows;
    # the pivot sequence must still be the oracle's, and the factor the same
    # as the cooperative panel's run to the end, up to rounding
    rng = np.random.default_rng(N + 7)
    A = rng.standard_normal((N, N))
    A = A + A.T
    say(f"automatic panel (register tail) N={N} vs oracle")
    S = mds.solver_for(_dense_problem(A))
    assert S.info()["panel"] == "coop"
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    _, inn, _ = S.factor_inertia()
    ino, _ = _factor_check(S, A)
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == ino
    L_auto, _, _, piv_auto = S.get_factor()
    del S
    C = mds.solver_for(_dense_problem(A), panel="coop")
    C.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    C.factor_inertia()
    L_coop, _, _, piv_coop = C.get_factor()
    assert np.array_equal(piv_auto, piv_coop)
    assert np.max(np.abs(L_auto - L_coop)) <= 1e-10 * max(1.0, np.max(np.abs(L_coop)))


def _golden_ipiv(name):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))
    N = g["ipiv"]["N"]
    ipiv = np.arange(1, N + 1, dtype=np.int32)
    ipiv[np.asarray(g["ipiv"]["index"], dtype=np.int64)] = g["ipiv"]["value"]
    return ipiv, tuple(g["inertia"]), g


def test_cooperative_panel_nine_workgroups_matches_oracle():
    # N = 9000: 9 workgroups (the 12-workgroup variant of the kernel); the
    # reference is the oracle's pivot sequence and inertia, stored by
    # tests/golden/make_golden_pivots.py (the oracle takes ~70 s on one
    # core), and the memory panel must agree as well
    N = 9000
    rng = np.random.default_rng(N)
    A = rng.standard_normal((N, N))
    A = A + A.T
    say("cooperative panel N=9000 vs memory panel")
    out = {}
    for panel in ("coop", "mem"):
        S = mds.solver_for(_dense_problem(A), panel=panel)
        S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
        _, inn, _ = S.factor_inertia()
        out[panel] = (S.get_factor()[3], (inn["npos"], inn["nzero"], inn["nneg"]))
        del S
    ipo, ino, _ = _golden_ipiv("pivots_dense_n9000.json")
    for panel in ("coop", "mem"):
        assert np.array_equal(out[panel][0], ipo), (panel, int(np.argmax(out[panel][0] != ipo)))
        assert out[panel][1] == ino, panel

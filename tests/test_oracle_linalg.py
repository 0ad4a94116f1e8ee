"""Pins for the oracle's linear algebra against what the paper and mathematics fix.

* condensation == the Schur complement of the explicit KKT matrix of
  eq. (linsys4x4) after eliminating x_s (Sec. 2.2, eq. (compressed));
* condensed solve + back-substitution == a dense solve of the full KKT system;
* Bunch-Kaufman pivots == LAPACK dsytrf (scipy) and P'AP = L D L';
* inertia == eigenvalue sign counts (Sylvester); Haynsworth additivity
  In(K) = In(D_s) + In(M) (Sec. 2.3);
* the inertia-correction loop reproduces its closed-form trial sequence;
* refinement reaches the backward-error target on the full KKT system.
"""
import json
import os

import numpy as np
import pytest
from scipy.linalg import lapack

import oracle
import synth
from helpers import block_d, full_kkt, perm_from_ipiv, sign_counts

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = (1.0 + np.sqrt(17.0)) / 8.0


def _tiny(n_d=5, n_s=12, m=4, r=3, p=0):
    return synth.make_problem(n_d, n_s, m, r, cfg=100, p=p)


def _state(prob, seed=0, lo=-1.0, hi=1.0):
    return synth.kkt_state(prob, seed, (lo, hi))


# ---------------------------------------------------------------- condense --
@pytest.mark.parametrize("dims", [(5, 12, 4, 3), (8, 30, 10, 4), (3, 6, 7, 2), (6, 40, 1, 5)])
@pytest.mark.parametrize("shifts", [(0.0, 0.0), (1e-3, 1e-6)])
def test_condense_is_schur_complement(dims, shifts):
    prob = _tiny(*dims)
    st = _state(prob, 1)
    dw, dc = shifts
    P = oracle.Problem(prob)
    M, inv_d = oracle.condense(P, st["sigma_d"], st["dsbase"], dw, dc)
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], dw, dc)
    nd, ns = prob["n_d"], prob["n_s"]
    n = nd + ns
    keep = np.r_[0:nd, n:K.shape[0]]
    elim = np.arange(nd, n)
    S = K[np.ix_(keep, keep)] - K[np.ix_(keep, elim)] @ np.linalg.solve(
        K[np.ix_(elim, elim)], K[np.ix_(elim, keep)])
    assert np.allclose(M, S, rtol=1e-12, atol=1e-12 * np.abs(S).max())
    assert np.array_equal(M, M.T)
    assert np.allclose(inv_d, 1.0 / (st["dsbase"] + dw), rtol=0, atol=0)


def test_condense_zero_sizes():
    # n_s = 0: no Schur term, M22 = -dc I
    prob = synth.make_problem(4, 0, 3, 2, cfg=101)
    P = oracle.Problem(prob)
    M, _ = oracle.condense(P, np.ones(4), np.zeros(0), 0.5, 0.25)
    assert np.array_equal(M[4:, 4:], -0.25 * np.eye(3))
    # m = 0: M = H + Sigma_d + dw
    prob = synth.make_problem(4, 5, 0, 2, cfg=102)
    P = oracle.Problem(prob)
    M, _ = oracle.condense(P, np.ones(4), np.ones(5), 0.5, 0.0)
    assert np.allclose(M, prob["H"] + 1.5 * np.eye(4), rtol=1e-15, atol=1e-15)
    # n_d = 0: M = M22 only
    prob = synth.make_problem(0, 9, 3, 3, cfg=103)
    P = oracle.Problem(prob)
    M, _ = oracle.condense(P, np.zeros(0), np.full(9, 2.0), 0.0, 0.0)
    K = full_kkt(prob, np.zeros(0), np.full(9, 2.0))
    S = -K[9:, :9] @ np.linalg.solve(K[:9, :9], K[:9, 9:])
    assert np.allclose(M, S, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_condensed_solve_equals_full_kkt_solve(seed):
    prob = _tiny(6, 25, 8, 3, p=seed)
    st = _state(prob, seed)
    P = oracle.Problem(prob)
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 1e-3, 1e-5)
    dx_d, dx_s, dy, status = F.solve(st["r_d"], st["r_s"], st["r_y"])
    assert status == 0
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], 1e-3, 1e-5)
    ref = np.linalg.solve(K, np.concatenate([st["r_d"], st["r_s"], st["r_y"]]))
    got = np.concatenate([dx_d, dx_s, dy])
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_rhs_condense_and_backsub_match_elimination():
    prob = _tiny(5, 20, 6, 3, p=4)
    st = _state(prob, 4)
    P = oracle.Problem(prob)
    _, inv_d = oracle.condense(P, st["sigma_d"], st["dsbase"], 0.0, 0.0)
    from helpers import dense_js
    Js = dense_js(prob)
    rhat = oracle.rhs_condense(P, inv_d, st["r_s"], st["r_y"])
    assert np.allclose(rhat, st["r_y"] - Js @ (st["r_s"] / st["dsbase"]), rtol=1e-13, atol=1e-13)
    dy = np.random.default_rng(0).standard_normal(prob["m"])
    dxs = oracle.backsub(P, inv_d, st["r_s"], dy)
    assert np.allclose(dxs, (st["r_s"] - Js.T @ dy) / st["dsbase"], rtol=1e-13, atol=1e-13)


# -------------------------------------------------------------- Bunch-Kaufman
def _check_factor(A, L, dd, ds, ipiv):
    N = A.shape[0]
    p = perm_from_ipiv(ipiv)
    R = L @ block_d(ipiv, dd, ds) @ L.T
    err = np.abs(R - A[np.ix_(p, p)]).max()
    assert err <= 10 * N * np.finfo(float).eps * max(np.abs(A).max(), 1.0) * max(
        1.0, np.abs(L).max() ** 2)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 17, 64, 65, 100, 257, 300])
@pytest.mark.parametrize("seed", [0, 1])
def test_bk_pivots_match_lapack(N, seed):
    rng = np.random.default_rng(1000 + 7 * N + seed)
    A = rng.standard_normal((N, N))
    A = A + A.T
    ldu, ipiv_ref, info_ref = lapack.dsytrf(A, lower=1)
    L, dd, ds, ipiv, info, _ = oracle.bk(A)
    assert info == info_ref == 0
    assert np.array_equal(ipiv, ipiv_ref)
    _check_factor(A, L, dd, ds, ipiv)


@pytest.mark.parametrize("seed", range(4))
def test_bk_on_condensed_matrices_matches_lapack(seed):
    prob = synth.make_problem(40, 300, 90, 4, cfg=104, p=seed)
    st = synth.kkt_state(prob, seed, (-2.0, 2.0))
    M, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 0.0, 0.0)
    ldu, ipiv_ref, info_ref = lapack.dsytrf(M, lower=1)
    L, dd, ds, ipiv, info, kind = oracle.bk(M)
    assert np.array_equal(ipiv, ipiv_ref)
    _check_factor(M, L, dd, ds, ipiv)


BRANCH_CASES = [
    # (matrix, expected branch of pivot step 0, expected ipiv)
    (np.array([[4.0, 1.0], [1.0, 3.0]]), 1, [1, 2]),
    (np.array([[1.0, 2.0, 0.0], [2.0, 0.0, 10.0], [0.0, 10.0, 0.0]]), 2, None),
    (np.array([[0.1, 2.0, 0.0], [2.0, 5.0, 1.0], [0.0, 1.0, 1.0]]), 3, None),
    (np.array([[0.0, 1.0], [1.0, 0.0]]), 4, [-2, -2]),
    (np.array([[0.0, 0.5, 2.0], [0.5, 1.0, 0.3], [2.0, 0.3, 0.0]]), 4, [-3, -3, 3]),
    (np.array([[0.0, 0.0], [0.0, 1.0]]), 0, [1, 2]),
]


@pytest.mark.parametrize("case", range(len(BRANCH_CASES)))
def test_bk_branches(case):
    A, br, ip = BRANCH_CASES[case]
    L, dd, ds, ipiv, info, kind = oracle.bk(A)
    assert kind[0] == br
    ldu, ipiv_ref, info_ref = lapack.dsytrf(A, lower=1)
    assert np.array_equal(ipiv, ipiv_ref)
    assert info == info_ref
    if ip is not None:
        assert list(ipiv) == ip
    if info == 0:
        _check_factor(A, L, dd, ds, ipiv)
    ev = np.linalg.eigvalsh(A)
    assert oracle.inertia(ipiv, dd, ds) == sign_counts(ev, 1e-12)


def test_bk_branch_thresholds_hand_computed():
    # absakk = 1 < alpha*colmax = 1.28 (first test fails);
    # alpha*colmax*(colmax/rowmax) = alpha*2*0.2 = 0.256 <= 1 -> 1x1 without swap
    A = BRANCH_CASES[1][0]
    assert 1.0 < ALPHA * 2.0 and ALPHA * 2.0 * (2.0 / 10.0) <= 1.0
    L, dd, ds, ipiv, info, kind = oracle.bk(A)
    assert dd[0] == 1.0 and ipiv[0] == 1


@pytest.mark.parametrize("N", [6, 31, 120])
def test_inertia_is_sylvester(N):
    rng = np.random.default_rng(N)
    Qm, _ = np.linalg.qr(rng.standard_normal((N, N)))
    ev = rng.uniform(0.5, 2.0, N) * rng.choice([-1.0, 1.0], N)
    A = (Qm * ev) @ Qm.T
    A = 0.5 * (A + A.T)
    L, dd, ds, ipiv, info, _ = oracle.bk(A)
    assert oracle.inertia(ipiv, dd, ds) == sign_counts(ev)


def test_inertia_zero_eigenvalue_exact():
    # exactly singular: a zero row/column gives an exact zero pivot
    A = np.diag([3.0, 0.0, -2.0, 5.0])
    L, dd, ds, ipiv, info, _ = oracle.bk(A)
    assert info == 2
    assert oracle.inertia(ipiv, dd, ds) == (2, 1, 1)


@pytest.mark.parametrize("seed", range(3))
def test_haynsworth_additivity(seed):
    prob = synth.make_problem(6, 15, 5, 3, cfg=105, p=seed)
    st = _state(prob, seed)
    P = oracle.Problem(prob)
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    K = full_kkt(prob, st["sigma_d"], st["dsbase"])
    npos, nz, nneg = sign_counts(np.linalg.eigvalsh(K), 1e-10)
    assert (npos, nz, nneg) == (F.inertia[0] + prob["n_s"], F.inertia[1], F.inertia[2])


# ------------------------------------------------------- inertia correction --
def test_correction_loop_closed_form():
    gold = json.load(open(os.path.join(GOLD, "correction_loop.json")))
    prob = synth.make_problem(4, 3, 0, 2, cfg=106)
    prob["H"] = -2.0 * np.eye(4)
    P = oracle.Problem(prob)
    F = oracle.Factor(P)
    dw_last = 0.0
    for call in gold["calls"]:
        st, dw_last = F.correct(np.zeros(4), np.asarray(prob["w"]), 1e-2, dw_last)
        assert st == 0
        assert F.s.trials == call["trials"]
        assert dw_last == pytest.approx(call["dw_num"] / call["dw_den"], rel=1e-12)
        assert F.inertia == (4, 0, 0)
        M = (dw_last - 2.0) * np.eye(4)
        assert sign_counts(np.linalg.eigvalsh(M)) == F.inertia


def test_correction_loop_cap_fails():
    prob = synth.make_problem(3, 2, 0, 1, cfg=107)
    prob["H"] = -1e6 * np.eye(3)
    P = oracle.Problem(prob)
    F = oracle.Factor(P)
    st, _ = F.correct(np.zeros(3), np.asarray(prob["w"]), 1e-2, 0.0, dw_max=1e3)
    assert st == 2


def test_correction_singular_sets_dc():
    # Two identical constraint rows make M exactly singular.  All entries are
    # dyadic so the elimination is exact and the zero pivot is exactly 0.0;
    # the loop must then add dc = 1e-8 mu^(1/4) and reach inertia (n_d, 0, m).
    prob = synth.make_problem(4, 10, 3, 2, cfg=108)
    prob["H"] = np.eye(4)
    prob["rp"] = np.array([0, 2, 4, 6], dtype=np.int32)
    prob["ci"] = np.array([1, 5, 1, 5, 2, 7], dtype=np.int32)
    prob["v"] = np.array([2.0, 2.0, 2.0, 2.0, -1.0, 0.5])
    prob["Jd"] = np.asfortranarray(np.vstack([np.ones(4), np.ones(4), np.arange(4.0)]))
    P = oracle.Problem(prob)
    sd, db = np.ones(4), np.full(10, 4.0)
    F = oracle.Factor(P).once(sd, db, 0.0, 0.0)
    assert F.inertia[1] == 1
    mu = 1e-4
    st, dwl = F.correct(sd, db, mu, 0.0)
    assert st == 0 and F.inertia == (4, 0, 3)
    assert F.s.dc == pytest.approx(1e-8 * mu ** 0.25, rel=1e-14)
    assert F.s.dw == pytest.approx(1e-4, rel=1e-14)
    K = full_kkt(prob, sd, db, F.s.dw, F.s.dc)
    assert sign_counts(np.linalg.eigvalsh(K), 1e-14) == (14, 0, 3)


# ---------------------------------------------------------------- refinement --
@pytest.mark.parametrize("seed", [0, 1])
def test_refine_reaches_backward_error(seed):
    prob = synth.make_problem(20, 200, 40, 4, cfg=109, p=seed)
    st = synth.kkt_state(prob, seed, (-1.0, 1.0))
    P = oracle.Problem(prob)
    F = oracle.Factor(P)
    stc, _ = F.correct(st["sigma_d"], st["dsbase"], 1e-2, 0.0)
    assert stc == 0
    dx_d, dx_s, dy, steps, eta = F.refine(st["r_d"], st["r_s"], st["r_y"], 5, 1e-14)
    assert eta <= 1e-14
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], F.s.dw, F.s.dc)
    r = np.concatenate([st["r_d"], st["r_s"], st["r_y"]])
    x = np.concatenate([dx_d, dx_s, dy])
    eta_np = np.abs(r - K @ x).max() / (np.abs(K).sum(1).max() * np.abs(x).max() + np.abs(r).max())
    assert eta_np <= 1e-14
    ref = np.linalg.solve(K, r)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    # the operator norm used in eta is the max absolute row sum of K
    assert oracle.kkt_norm_inf(P, st["sigma_d"], st["dsbase"], F.s.dw, F.s.dc) == pytest.approx(
        np.abs(K).sum(1).max(), rel=1e-13)


def test_kkt_matvec_matches_dense():
    prob = _tiny(7, 30, 9, 3, p=5)
    st = _state(prob, 5)
    P = oracle.Problem(prob)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(7 + 30 + 9)
    o = oracle.kkt_matvec(P, st["sigma_d"], st["dsbase"], 0.3, 0.2, x[:7], x[7:37], x[37:])
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], 0.3, 0.2)
    assert np.allclose(np.concatenate(o), K @ x, rtol=1e-13, atol=1e-13)


def test_threaded_elimination_is_bit_identical():
    # the columns of each rank-1/2 update are split over threads; every entry
    # keeps its expression, so the factor does not depend on the count
    prob = synth.make_problem(150, 3000, 450, 6, cfg=299, s_scale=3.0)
    st = synth.kkt_state(prob, 5, (-3.0, 3.0))
    P = oracle.Problem(prob)
    M, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], 0.0, 0.0)
    ref = oracle.bk(M)
    try:
        oracle.set_threads(4)
        got = oracle.bk(M)
    finally:
        oracle.set_threads(1)
    for a, b in zip(ref[:4], got[:4]):
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
    # the partial elimination is the same process stopped early
    A = np.asfortranarray(M.copy())
    _, ipiv = oracle.bk_partial(A, 100)
    k = 100 if ref[3][99] > 0 or ref[3][98] == ref[3][99] else 101
    assert np.array_equal(ipiv[:k], ref[3][:k])

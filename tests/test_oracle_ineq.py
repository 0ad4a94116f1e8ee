"""Pins for the oracle's inequality rows (Sec. 2, eq. (ineq)) and their slack
reformulation inside the IPM (Sec. 2.1), against results the mathematics
fixes independently of the oracle:

* the condensed matrix with the rows' (4,4) block equals the Schur
  complement of the explicit Newton matrix in which the slacks are unknowns
  (x_d, x_s, d, y), eliminating x_s and d (Sec. 2.2, eq. (compressed));
* Haynsworth: the inertia of that explicit matrix is (n_s + m_I, 0, 0) plus
  the inertia of the condensed one (Sec. 2.3);
* the IPM's Newton direction equals the direction of the unreduced
  primal-dual Newton system with slacks and every bound multiplier kept;
* the right-hand side is minus the gradient of the barrier Lagrangian in
  (x, d) (central finite differences);
* rows whose bounds cannot bind leave the solution of the equality-only
  problem unchanged; a tiny strictly convex QP with binding inequality rows
  and bounds is solved by brute-force enumeration of active sets, and the
  IPM must land on that global optimum; at termination the first-order
  conditions hold (checked with numpy) and the explicit KKT matrix has the
  inertia (n + m_I, 0, m).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from helpers import dense_js, sign_counts


def _blocks(prob):
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    H = np.asarray(prob["H"]).reshape(nd, nd)
    Jd = np.asarray(prob["Jd"]).reshape(m, nd)
    Js = dense_js(prob)
    return H, Jd, Js


def _selector(prob):
    """E (m x m_I): the slack column of inequality row m_E + r is E[:, r]."""
    m, mI = prob["m"], prob["m_I"]
    E = np.zeros((m, mI))
    E[m - mI + np.arange(mI), np.arange(mI)] = 1.0
    return E


def _slack_kkt(prob, sigma_d, dsbase, sig_h, dw, dc):
    """Newton matrix with the slacks as unknowns, order (x_d, x_s, d, y):
    [[H+Sd+dw, 0, 0, Jd'], [0, Ds+dw, 0, Js'], [0, 0, Sh+dw, -E'],
     [Jd, Js, -E, -dc I]]."""
    H, Jd, Js = _blocks(prob)
    nd, ns, m, mI = prob["n_d"], prob["n_s"], prob["m"], prob["m_I"]
    E = _selector(prob)
    t = nd + ns + mI + m
    K = np.zeros((t, t))
    a, b, c = nd, nd + ns, nd + ns + mI
    K[:a, :a] = H + np.diag(sigma_d + dw)
    K[a:b, a:b] = np.diag(dsbase + dw)
    K[b:c, b:c] = np.diag(sig_h + dw)
    K[c:, :a] = Jd
    K[c:, a:b] = Js
    K[c:, b:c] = -E
    K[:c, c:] = K[c:, :c].T
    K[c:, c:] = -dc * np.eye(m)
    return K


def _state(prob, seed):
    rng = np.random.default_rng(seed)
    return dict(sigma_d=10.0 ** rng.uniform(-2, 1, prob["n_d"]),
                dsbase=10.0 ** rng.uniform(-1, 1, prob["n_s"]),
                sig_h=10.0 ** rng.uniform(-2, 2, prob["m_I"]))


@pytest.mark.parametrize("shape", [(5, 12, 7, 3, 4), (4, 9, 6, 2, 6), (0, 10, 5, 3, 2),
                                   (6, 0, 4, 0, 4)])
def test_condensed_ineq_is_schur_complement(shape):
    nd, ns, m, r, mI = shape
    prob = synth.make_problem(nd, ns, m, r, cfg=300, p=sum(shape), m_I=mI)
    st = _state(prob, 1)
    P = oracle.Problem(prob)
    dw, dc = 0.3, 1e-3
    dcv = oracle.ineq_dcv(P, st["sig_h"], dw)
    assert np.all(dcv[:m - mI] == 0.0)
    assert np.array_equal(dcv[m - mI:], 1.0 / (st["sig_h"] + dw))
    M, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], dw, dc, dcv=dcv)
    K = _slack_kkt(prob, st["sigma_d"], st["dsbase"], st["sig_h"], dw, dc)
    keep = np.r_[np.arange(nd), nd + ns + mI + np.arange(m)]
    elim = np.arange(nd, nd + ns + mI)
    S = K[np.ix_(keep, keep)] - K[np.ix_(keep, elim)] @ np.linalg.solve(
        K[np.ix_(elim, elim)], K[np.ix_(elim, keep)])
    assert np.allclose(M, S, rtol=1e-12, atol=1e-12 * np.abs(S).max())
    # Haynsworth inertia additivity: In(K) = (n_s + m_I, 0, 0) + In(M)
    eM = np.linalg.eigvalsh(M)
    eK = np.linalg.eigvalsh(K)
    pm, zm, nm = sign_counts(eM)
    assert sign_counts(eK) == (pm + ns + mI, zm, nm)


def test_factor_with_slack_forms_the_block_every_trial():
    # the correction loop re-condenses with each trial shift, and the slacks'
    # D_h = Sigma_h + dw follows it
    prob = synth.make_problem(6, 40, 10, 3, cfg=301, s_scale=6.0, m_I=5)
    st = _state(prob, 2)
    P = oracle.Problem(prob)
    F = oracle.Factor(P, sig_h=st["sig_h"])
    status, _ = F.correct(st["sigma_d"], st["dsbase"], 0.1)
    assert status == 0 and F.s.trials > 1
    dw = F.s.dw
    assert np.array_equal(F.dcv, oracle.ineq_dcv(P, st["sig_h"], dw))
    K = _slack_kkt(prob, st["sigma_d"], st["dsbase"], st["sig_h"], dw, F.s.dc)
    n = prob["n_d"] + prob["n_s"]
    assert sign_counts(np.linalg.eigvalsh(K)) == (n + prob["m_I"], 0, prob["m"])


def _qp(prob):
    H, Jd, Js = _blocks(prob)
    nd, ns = prob["n_d"], prob["n_s"]
    G = np.zeros((nd + ns, nd + ns))
    G[:nd, :nd] = H
    G[nd:, nd:] = np.diag(prob["w"])
    q = np.concatenate([prob["c"], prob["g"]])
    A = np.hstack([Jd, Js])
    return G, q, A


def _interior_point(prob, seed):
    """Strictly interior (x, d) with multipliers: slacks strictly inside
    their bounds."""
    it = synth.interior_iterate(prob, seed)
    rng = np.random.default_rng(seed + 50)
    hl, hu = prob["hl"], prob["hu"]
    mid = np.where(np.isfinite(hl) & np.isfinite(hu), 0.5 * (hl + hu),
                   np.where(np.isfinite(hl), hl + 0.3, hu - 0.3))
    d = mid + 0.05 * rng.standard_normal(len(mid))
    vl = np.where(np.isfinite(hl), 10.0 ** rng.uniform(-2, 1, len(d)), 0.0)
    vu = np.where(np.isfinite(hu), 10.0 ** rng.uniform(-2, 1, len(d)), 0.0)
    zl = np.where(np.isfinite(prob["xl"]), it["zl"], 0.0)
    zu = np.where(np.isfinite(prob["xu"]), it["zu"], 0.0)
    return (np.concatenate([it["x"], d]), it["y"], np.concatenate([zl, vl]),
            np.concatenate([zu, vu]), it["mu"])


def test_direction_equals_unreduced_newton_with_slacks():
    prob = synth.make_problem(4, 9, 5, 2, cfg=302, s_scale=0.0, m_I=3)
    prob["hl"][0] = -np.inf  # one row bounded above only
    X, y, ZL, ZU, mu = _interior_point(prob, 4)
    P = oracle.Problem(prob)
    st, dx, dy, dzl, dzu = oracle.newton_direction(P, X, y, ZL, ZU, mu)
    assert st == 0
    G, q, A = _qp(prob)
    n, m, mI = G.shape[0], prob["m"], prob["m_I"]
    nx = n + mI
    E = _selector(prob)
    lo = np.concatenate([prob["xl"], prob["hl"]])
    up = np.concatenate([prob["xu"], prob["hu"]])
    fl, fu = np.isfinite(lo), np.isfinite(up)
    # unknowns (dx, dd, dy, dzl, dzu); infinite bounds have no multiplier
    Gx = np.zeros((nx, nx))
    Gx[:n, :n] = G
    Ax = np.hstack([A, -E])                     # constraint Jacobian in (x, d)
    bx = np.concatenate([prob["b"][:m - mI], np.zeros(mI)])
    I = np.eye(nx)
    sl = np.where(fl, X - np.where(fl, lo, 0.0), 1.0)
    su = np.where(fu, np.where(fu, up, 0.0) - X, 1.0)
    KK = np.block([
        [Gx, Ax.T, -I, I],
        [Ax, np.zeros((m, m)), np.zeros((m, nx)), np.zeros((m, nx))],
        [np.diag(ZL), np.zeros((nx, m)), np.diag(sl), np.zeros((nx, nx))],
        [-np.diag(ZU), np.zeros((nx, m)), np.zeros((nx, nx)), np.diag(su)]])
    grad = np.concatenate([G @ X[:n] + q, np.zeros(mI)])
    F0 = np.concatenate([grad + Ax.T @ y - ZL + ZU, Ax @ X - bx,
                         np.where(fl, sl * ZL - mu, 0.0), np.where(fu, su * ZU - mu, 0.0)])
    # rows of absent multipliers: dz = 0
    for i in range(nx):
        if not fl[i]:
            KK[nx + m + i, :] = 0.0
            KK[nx + m + i, nx + m + i] = 1.0
        if not fu[i]:
            KK[2 * nx + m + i, :] = 0.0
            KK[2 * nx + m + i, 2 * nx + m + i] = 1.0
    d = np.linalg.solve(KK, -F0)
    scale = np.abs(d).max()
    assert np.abs(dx - d[:nx]).max() <= 1e-9 * scale
    assert np.abs(dy - d[nx:nx + m]).max() <= 1e-9 * scale
    assert np.abs(dzl - d[nx + m:2 * nx + m]).max() <= 1e-9 * scale
    assert np.abs(dzu - d[2 * nx + m:]).max() <= 1e-9 * scale


def test_rhs_is_minus_barrier_lagrangian_gradient_in_x_and_d():
    prob = synth.make_problem(3, 5, 4, 2, cfg=303, m_I=2)
    X, y, ZL, ZU, _ = _interior_point(prob, 7)
    P = oracle.Problem(prob)
    mu = 0.05
    _, rx, ry = oracle.sigma_rhs(P, X, y, ZL, ZU, mu)
    G, q, A = _qp(prob)
    n, m, mI = G.shape[0], prob["m"], prob["m_I"]
    E = _selector(prob)
    bx = np.concatenate([prob["b"][:m - mI], np.zeros(mI)])

    def c(v):
        return A @ v[:n] - E @ v[n:] - bx

    def lag(v):
        return oracle.barrier(P, v, mu) + y @ c(v)

    h = 1e-6
    for i in range(n + mI):
        e = np.zeros(n + mI)
        e[i] = h
        fd = (lag(X + e) - lag(X - e)) / (2 * h)
        assert -rx[i] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    assert np.allclose(-ry, c(X), rtol=1e-13, atol=1e-13)
    assert oracle.theta(P, X) == pytest.approx(np.abs(c(X)).sum(), rel=1e-13)


def test_rows_that_cannot_bind_change_nothing():
    prob = synth.make_problem(10, 120, 14, 3, cfg=304, m_I=5)
    loose = dict(prob)
    loose["hl"] = prob["b"][-5:] - 1e3
    loose["hu"] = np.where(np.arange(5) % 2 == 0, np.inf, prob["b"][-5:] + 1e3)
    r = oracle.ipm(oracle.Problem(loose))
    assert r["status"] == "converged"
    # the same problem without the inequality rows
    m_E = prob["m"] - 5
    eq = dict(prob)
    eq["m"], eq["m_I"] = m_E, 0
    eq["hl"], eq["hu"] = np.zeros(0), np.zeros(0)
    eq["Jd"] = np.asfortranarray(np.asarray(prob["Jd"])[:m_E])
    eq["rp"] = prob["rp"][:m_E + 1]
    eq["ci"] = prob["ci"][:prob["rp"][m_E]]
    eq["v"] = prob["v"][:prob["rp"][m_E]]
    eq["b"] = prob["b"][:m_E]
    re = oracle.ipm(oracle.Problem(eq))
    assert re["status"] == "converged"
    n = prob["n_d"] + prob["n_s"]
    assert np.abs(r["x"][:n] - re["x"]).max() <= 1e-6
    assert np.abs(r["y"][:m_E] - re["y"]).max() <= 1e-6 * max(1.0, np.abs(re["y"]).max())
    assert np.abs(r["y"][m_E:]).max() <= 1e-6


def _brute_force(G, q, A, b, mE, hl, hu, lo, hi):
    """Global minimiser of a strictly convex QP with equality rows, two-sided
    inequality rows and bounds, by enumerating the active sets."""
    n, m = G.shape[0], A.shape[0]
    mI = m - mE
    best = None
    for xs in itertools.product((0, 1, 2), repeat=n):          # free, lower, upper
        xs = np.array(xs)
        for hs in itertools.product((0, 1, 2), repeat=mI):     # inactive, at hl, at hu
            hs = np.array(hs)
            if np.any((hs == 1) & ~np.isfinite(hl)) or np.any((hs == 2) & ~np.isfinite(hu)):
                continue
            if np.any((xs == 1) & ~np.isfinite(lo)) or np.any((xs == 2) & ~np.isfinite(hi)):
                continue
            rows = list(range(mE)) + [mE + r for r in range(mI) if hs[r] != 0]
            rhs_b = np.concatenate([b[:mE], [hl[r] if hs[r] == 1 else hu[r]
                                             for r in range(mI) if hs[r] != 0]])
            F = np.where(xs == 0)[0]
            Fx = np.where(xs != 0)[0]
            xf = np.where(xs == 1, lo, hi)
            Ar = A[rows]
            nf, mr = len(F), len(rows)
            KK = np.zeros((nf + mr, nf + mr))
            KK[:nf, :nf] = G[np.ix_(F, F)]
            KK[:nf, nf:] = Ar[:, F].T
            KK[nf:, :nf] = Ar[:, F]
            if np.linalg.matrix_rank(KK) < nf + mr:
                continue
            sol = np.linalg.solve(KK, np.concatenate([-q[F] - G[np.ix_(F, Fx)] @ xf[Fx],
                                                      rhs_b - Ar[:, Fx] @ xf[Fx]]))
            x = xf.copy()
            x[F] = sol[:nf]
            if np.any(x < lo - 1e-12) or np.any(x > hi + 1e-12):
                continue
            h = A[mE:] @ x
            if np.any(h < hl - 1e-12) or np.any(h > hu + 1e-12):
                continue
            y = np.zeros(m)
            y[rows] = sol[nf:]
            yh = y[mE:]
            if np.any(yh[hs == 1] > 1e-12) or np.any(yh[hs == 2] < -1e-12):
                continue
            gl = G @ x + q + A.T @ y
            if np.any(np.where(xs == 1, gl, 0.0) < -1e-12) or np.any(np.where(xs == 2, -gl, 0.0) < -1e-12):
                continue
            f = 0.5 * x @ G @ x + q @ x
            if best is None or f < best[0]:
                best = (f, x, y, hs)
    return best


@pytest.mark.parametrize("seed", range(4))
def test_ineq_qp_brute_force(seed):
    prob = synth.make_problem(2, 3, 3, 2, cfg=305, p=seed, m_I=2)
    prob["H"] = np.asfortranarray(prob["H"] + 1.5 * np.eye(2))   # strictly convex
    prob["c"] = 3.0 * prob["c"]
    prob["g"] = 6.0 * prob["g"]
    G, q, A = _qp(prob)
    mE = prob["m"] - prob["m_I"]
    best = _brute_force(G, q, A, prob["b"], mE, prob["hl"], prob["hu"], prob["xl"], prob["xu"])
    assert best is not None
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    n = G.shape[0]
    assert np.abs(r["x"][:n] - best[1]).max() <= 1e-6
    assert np.abs(r["y"] - best[2]).max() <= 1e-5 * max(1.0, np.abs(best[2]).max())


def test_some_brute_force_case_has_a_binding_row():
    # the parametrised QPs above exercise binding inequality rows
    hits = 0
    for seed in range(4):
        prob = synth.make_problem(2, 3, 3, 2, cfg=305, p=seed, m_I=2)
        prob["H"] = np.asfortranarray(prob["H"] + 1.5 * np.eye(2))
        prob["c"] = 3.0 * prob["c"]
        prob["g"] = 6.0 * prob["g"]
        G, q, A = _qp(prob)
        best = _brute_force(G, q, A, prob["b"], 1, prob["hl"], prob["hu"], prob["xl"],
                            prob["xu"])
        hits += int(np.any(best[3] != 0))
    assert hits >= 1


def test_ineq_ipm_certificate_and_second_order_inertia():
    prob = synth.make_problem(16, 300, 40, 4, cfg=306, m_I=20)
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    G, q, A = _qp(prob)
    n, m, mI = G.shape[0], prob["m"], prob["m_I"]
    E = _selector(prob)
    X, y, ZL, ZU = r["x"], r["y"], r["zl"], r["zu"]
    x, d = X[:n], X[n:]
    lo = np.concatenate([prob["xl"], prob["hl"]])
    up = np.concatenate([prob["xu"], prob["hu"]])
    fl, fu = np.isfinite(lo), np.isfinite(up)
    tol = 1e-8
    nz = fl.sum() + fu.sum()
    sd = max(1.0, (np.abs(y).sum() + ZL.sum() + ZU.sum()) / (m + nz) / 100.0)
    sc = max(1.0, (ZL.sum() + ZU.sum()) / nz / 100.0)
    # primal: equality rows, inequality rows against their slacks, slacks in bounds
    assert np.abs(A[:m - mI] @ x - prob["b"][:m - mI]).max() <= tol
    assert np.abs(A[m - mI:] @ x - d).max() <= tol
    assert np.all(d[np.isfinite(prob["hl"])] > prob["hl"][np.isfinite(prob["hl"])])
    assert np.all(d[np.isfinite(prob["hu"])] < prob["hu"][np.isfinite(prob["hu"])])
    # dual: grad f + J'y - zl + zu = 0 in x; -y_h - vl + vu = 0 in d
    gx = G @ x + q + A.T @ y - ZL[:n] + ZU[:n]
    gd = -y[m - mI:] - ZL[n:] + ZU[n:]
    assert max(np.abs(gx).max(), np.abs(gd).max()) <= tol * sd
    # complementarity
    cl = np.where(fl, (X - np.where(fl, lo, 0.0)) * ZL, 0.0)
    cu = np.where(fu, (np.where(fu, up, 0.0) - X) * ZU, 0.0)
    assert max(np.abs(cl).max(), np.abs(cu).max()) <= tol * sc
    # some inequality row binds (its multiplier is away from zero)
    assert np.abs(y[m - mI:]).max() > 1e-3
    # second order: the slack-form KKT matrix at the solution has inertia
    # (n + m_I, 0, m)
    sig = np.where(fl, ZL / np.where(fl, X - np.where(fl, lo, 0.0), 1.0), 0.0) + \
        np.where(fu, ZU / np.where(fu, np.where(fu, up, 0.0) - X, 1.0), 0.0)
    nd = prob["n_d"]
    K = _slack_kkt(prob, sig[:nd], prob["w"] + sig[nd:n], sig[n:], 0.0, 0.0)
    assert sign_counts(np.linalg.eigvalsh(K)) == (n + mI, 0, m)

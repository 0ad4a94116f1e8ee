"""Pins for the oracle's coupling blocks of the sparse Hessian (assumption A2
of Sec. 2 in its general form: Q_{x_s} = diag(w) + blockdiag(Wb) + D_{x_s},
cheap to solve with), against what the mathematics fixes:

* blocks of size one with zero entries change nothing (bitwise);
* the blocks' L Delta L' reproduces each block of Q_{x_s};
* the condensed matrix is the Schur complement of the explicit KKT matrix
  of eq. (linsys4x4) whose (x_s, x_s) block is block diagonal, and the
  condensed solve + back-substitution equal a dense solve of that system;
* Haynsworth: In(K) = In(Q_{x_s}) + In(M) with Q_{x_s} positive definite;
* the full-system product and norm equal the dense matrix's;
* an equality-constrained convex QP with infinite bounds and coupled sparse
  variables reaches the closed-form solution of its KKT system; a bounded
  one ends at a KKT point certified in numpy with the block Hessian.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import dense_js, full_kkt, sign_counts


def _blockdiag(prob):
    ns, bp, Wb = prob["n_s"], prob["bp"], prob["Wb"]
    W = np.zeros((ns, ns))
    off = 0
    for b in range(len(bp) - 1):
        k0, sz = bp[b], bp[b + 1] - bp[b]
        W[k0:k0 + sz, k0:k0 + sz] = Wb[off:off + sz * sz].reshape(sz, sz, order="F")
        off += sz * sz
    return W


def _kkt(prob, sd, dsb, dw, dc):
    K = full_kkt(prob, sd, dsb, dw, dc)
    nd, ns = prob["n_d"], prob["n_s"]
    K[nd:nd + ns, nd:nd + ns] += _blockdiag(prob)
    return K


def _prob(nd=6, ns=40, m=9, r=4, sblk=4, p=0):
    return synth.make_problem(nd, ns, m, r, cfg=120, p=p, sblk=sblk)


def test_unit_zero_blocks_change_nothing():
    prob = _prob(sblk=0)
    st = synth.kkt_state(prob, 1, (-1.0, 1.0))
    P0 = oracle.Problem(prob)
    q = dict(prob, bp=np.arange(prob["n_s"] + 1), Wb=np.zeros(prob["n_s"]))
    P1 = oracle.Problem(q)
    M0, i0 = oracle.condense(P0, st["sigma_d"], st["dsbase"], 1e-3, 1e-6)
    M1, i1 = oracle.condense(P1, st["sigma_d"], st["dsbase"], 1e-3, 1e-6)
    assert np.array_equal(M0.view(np.int64), M1.view(np.int64))
    assert np.array_equal(i0.view(np.int64), i1.view(np.int64))


@pytest.mark.parametrize("sblk", [2, 5, 16])
def test_block_factors_reproduce_q(sblk):
    prob = _prob(sblk=sblk, ns=60)
    st = synth.kkt_state(prob, 2, (-2.0, 2.0))
    P = oracle.Problem(prob)
    dw = 1e-4
    _, inv_d, lb = oracle.condense(P, st["sigma_d"], st["dsbase"], dw, 0.0, with_blocks=True)
    Q = _blockdiag(prob) + np.diag(st["dsbase"] + dw)
    bp = prob["bp"]
    off = 0
    for b in range(len(bp) - 1):
        k0, sz = bp[b], bp[b + 1] - bp[b]
        L = np.tril(lb[off:off + sz * sz].reshape(sz, sz, order="F"), -1) + np.eye(sz)
        D = np.diag(1.0 / inv_d[k0:k0 + sz])
        Qb = Q[k0:k0 + sz, k0:k0 + sz]
        assert np.abs(L @ D @ L.T - Qb).max() <= 1e-13 * np.abs(Qb).max()
        off += sz * sz


@pytest.mark.parametrize("dims", [(6, 40, 9, 4), (3, 25, 12, 3), (0, 30, 8, 4), (5, 20, 1, 6)])
@pytest.mark.parametrize("sblk", [2, 6])
def test_condense_is_schur_complement_with_blocks(dims, sblk):
    prob = _prob(*dims, sblk=sblk)
    st = synth.kkt_state(prob, 3, (-1.0, 1.0))
    dw, dc = 1e-3, 1e-6
    P = oracle.Problem(prob)
    M, inv_d, lb = oracle.condense(P, st["sigma_d"], st["dsbase"], dw, dc, with_blocks=True)
    K = _kkt(prob, st["sigma_d"], st["dsbase"], dw, dc)
    nd, ns = prob["n_d"], prob["n_s"]
    n = nd + ns
    keep = np.r_[0:nd, n:K.shape[0]]
    elim = np.arange(nd, n)
    S = K[np.ix_(keep, keep)] - K[np.ix_(keep, elim)] @ np.linalg.solve(
        K[np.ix_(elim, elim)], K[np.ix_(elim, keep)])
    assert np.allclose(M, S, rtol=1e-12, atol=1e-12 * np.abs(S).max())
    # Haynsworth with Q_{x_s} positive definite
    assert sign_counts(np.linalg.eigvalsh(K[np.ix_(elim, elim)])) == (ns, 0, 0)
    kin = sign_counts(np.linalg.eigvalsh(K))
    min_ = sign_counts(np.linalg.eigvalsh(M))
    assert kin == (min_[0] + ns, min_[1], min_[2])
    # condensed solve + back-substitution == dense solve of the full system
    F = oracle.Factor(P)
    F.once(st["sigma_d"], st["dsbase"], dw, dc)
    dx_d, dx_s, dy, stt = F.solve(st["r_d"], st["r_s"], st["r_y"])
    ref = np.linalg.solve(K, np.concatenate([st["r_d"], st["r_s"], st["r_y"]]))
    got = np.concatenate([dx_d, dx_s, dy])
    assert np.abs(got - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    # the condensed rhs and the back-substitution on their own
    Ks = K[np.ix_(elim, elim)]
    rhat = oracle.rhs_condense(P, inv_d, st["r_s"], st["r_y"], lb)
    Js = dense_js(prob)
    ref_rhat = st["r_y"] - Js @ np.linalg.solve(Ks, st["r_s"])
    assert np.abs(rhat - ref_rhat).max() <= 1e-11 * max(1.0, np.abs(ref_rhat).max())
    xs = oracle.backsub(P, inv_d, st["r_s"], st["r_y"], lb)
    ref_xs = np.linalg.solve(Ks, st["r_s"] - Js.T @ st["r_y"])
    assert np.abs(xs - ref_xs).max() <= 1e-11 * max(1.0, np.abs(ref_xs).max())


def test_kkt_product_and_norm_with_blocks():
    prob = _prob(sblk=5)
    st = synth.kkt_state(prob, 4, (-1.0, 1.0))
    P = oracle.Problem(prob)
    K = _kkt(prob, st["sigma_d"], st["dsbase"], 2e-3, 3e-7)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(K.shape[0])
    nd, ns = prob["n_d"], prob["n_s"]
    o = oracle.kkt_matvec(P, st["sigma_d"], st["dsbase"], 2e-3, 3e-7, v[:nd], v[nd:nd + ns],
                          v[nd + ns:])
    assert np.allclose(np.concatenate(o), K @ v, rtol=1e-13, atol=1e-13 * np.abs(K @ v).max())
    nrm = oracle.kkt_norm_inf(P, st["sigma_d"], st["dsbase"], 2e-3, 3e-7)
    assert nrm == pytest.approx(np.abs(K).sum(axis=1).max(), rel=1e-13)


def _qp_data(prob):
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    G = np.zeros((nd + ns, nd + ns))
    G[:nd, :nd] = prob["H"]
    G[nd:, nd:] = np.diag(prob["w"]) + _blockdiag(prob)
    q = np.concatenate([prob["c"], prob["g"]])
    A = np.hstack([np.asarray(prob["Jd"]).reshape(m, nd), dense_js(prob)])
    return G, q, A


def test_equality_qp_closed_form_with_blocks():
    prob = synth.make_problem(8, 60, 10, 3, cfg=121, sblk=4)
    H = prob["H"]
    prob["H"] = np.asfortranarray(H - np.diag(np.linalg.eigvalsh(H).min() * np.ones(8)) + np.eye(8))
    n = 68
    prob["xl"] = np.full(n, -np.inf)
    prob["xu"] = np.full(n, np.inf)
    G, q, A = _qp_data(prob)
    K = np.block([[G, A.T], [A, np.zeros((10, 10))]])
    sol = np.linalg.solve(K, np.concatenate([-q, prob["b"]]))
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    assert np.abs(r["x"] - sol[:n]).max() <= 1e-8 * max(1.0, np.abs(sol[:n]).max())
    assert np.abs(r["y"] - sol[n:]).max() <= 1e-8 * max(1.0, np.abs(sol[n:]).max())


@pytest.mark.parametrize("seed", [0, 1])
def test_bounded_qp_with_blocks_kkt_certificate(seed):
    prob = synth.make_problem(16, 300, 24, 3, cfg=122, p=seed, sblk=6)
    prob["g"] = 4.0 * prob["g"]   # several bounds bind at the solution
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    G, q, A = _qp_data(prob)
    x, y, zl, zu = r["x"], r["y"], r["zl"], r["zu"]
    tol = 1e-8
    assert np.abs(A @ x - prob["b"]).max() <= tol
    sd = max(1.0, (np.abs(y).sum() + zl.sum() + zu.sum()) / (len(y) + 2 * len(x)) / 100.0)
    assert np.abs(G @ x + q + A.T @ y - zl + zu).max() <= tol * sd
    sc = max(1.0, (zl.sum() + zu.sum()) / (2 * len(x)) / 100.0)
    assert np.abs((x - prob["xl"]) * zl).max() <= tol * sc
    assert np.abs((prob["xu"] - x) * zu).max() <= tol * sc
    assert np.sum((prob["xu"] - x) < 1e-6) + np.sum((x - prob["xl"]) < 1e-6) > 0
    # second-order: the final KKT matrix with the IPM's barrier diagonal has inertia (n, 0, m)
    last = r["trace"][r["iters"] - 1]
    assert tuple(last["inertia"]) == (prob["n_d"], 0, prob["m"])


def test_warm_start_refused_with_blocks():
    prob = _prob(sblk=3)
    with pytest.raises(Exception):
        oracle.ipm(oracle.Problem(prob), warm=dict(x_d=np.zeros(prob["n_d"]),
                                                   y=np.zeros(prob["m"]), mu0=1e-3))

"""Pins for the oracle's interior-point method (Sec. 2.1) and its vector
quantities, against results the mathematics fixes independently of it:

* an equality-constrained convex QP with no bounds has the closed-form
  solution of its KKT system;
* a tiny bound-constrained convex QP is solved by brute-force enumeration of
  active sets; the IPM must land on that global optimum;
* sparse variables that appear in no constraint decouple into 1-D box QPs
  whose minimiser is clip(-g/w, -1, 1);
* at termination the first-order conditions hold (checked with numpy from
  the problem data) and the final KKT matrix has inertia (n, 0, m);
* the reduced Newton direction equals the direction of the unreduced
  primal-dual Newton system (with the bound multipliers kept);
* the right-hand side is minus the gradient of the barrier Lagrangian
  (central finite differences); fraction-to-boundary satisfies its definition.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from helpers import dense_js, full_kkt, sign_counts


def _qp_data(prob):
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    G = np.zeros((nd + ns, nd + ns))
    G[:nd, :nd] = prob["H"]
    G[nd:, nd:] = np.diag(prob["w"])
    q = np.concatenate([prob["c"], prob["g"]])
    A = np.hstack([np.asarray(prob["Jd"]).reshape(m, nd), dense_js(prob)])
    return G, q, A


def test_equality_qp_closed_form():
    prob = synth.make_problem(10, 50, 12, 3, cfg=200)
    prob["H"] = np.asfortranarray(prob["H"] - np.diag(np.linalg.eigvalsh(prob["H"]).min() * np.ones(10)) + np.eye(10))
    n = 60
    prob["xl"] = np.full(n, -np.inf)
    prob["xu"] = np.full(n, np.inf)
    G, q, A = _qp_data(prob)
    K = np.block([[G, A.T], [A, np.zeros((12, 12))]])
    sol = np.linalg.solve(K, np.concatenate([-q, prob["b"]]))
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    assert np.abs(r["x"] - sol[:n]).max() <= 1e-8 * max(1.0, np.abs(sol[:n]).max())
    assert np.abs(r["y"] - sol[n:]).max() <= 1e-8 * max(1.0, np.abs(sol[n:]).max())


def _brute_force_box_qp(G, q, A, b, lo, hi):
    """Global minimiser of a strictly convex QP by enumerating active sets."""
    n, m = G.shape[0], A.shape[0]
    best = None
    for state in itertools.product((0, 1, 2), repeat=n):  # 0 free, 1 lower, 2 upper
        fixed = np.array([s != 0 for s in state])
        xf = np.where(np.array(state) == 1, lo, hi)
        F = np.where(~fixed)[0]
        Fx = np.where(fixed)[0]
        nf = len(F)
        KK = np.zeros((nf + m, nf + m))
        KK[:nf, :nf] = G[np.ix_(F, F)]
        KK[:nf, nf:] = A[:, F].T
        KK[nf:, :nf] = A[:, F]
        rhs = np.concatenate([-q[F] - G[np.ix_(F, Fx)] @ xf[Fx], b - A[:, Fx] @ xf[Fx]])
        try:
            if np.linalg.matrix_rank(KK) < nf + m:
                continue
            s = np.linalg.solve(KK, rhs)
        except np.linalg.LinAlgError:
            continue
        x = xf.copy()
        x[F] = s[:nf]
        y = s[nf:]
        if np.any(x[F] < lo[F] - 1e-12) or np.any(x[F] > hi[F] + 1e-12):
            continue
        gl = G @ x + q + A.T @ y
        zl = np.where(np.array(state) == 1, gl, 0.0)
        zu = np.where(np.array(state) == 2, -gl, 0.0)
        if np.any(zl < -1e-12) or np.any(zu < -1e-12):
            continue
        f = 0.5 * x @ G @ x + q @ x
        if best is None or f < best[0]:
            best = (f, x, y)
    return best


@pytest.mark.parametrize("seed", range(4))
def test_box_qp_brute_force(seed):
    prob = synth.make_problem(2, 4, 2, 2, cfg=201, p=seed)
    prob["H"] = np.asfortranarray(prob["H"] + 1.5 * np.eye(2))  # strictly convex
    # scale the linear terms so that several bounds are active at the optimum
    prob["c"] = 3.0 * prob["c"]
    prob["g"] = 6.0 * prob["g"]
    G, q, A = _qp_data(prob)
    n = 6
    best = _brute_force_box_qp(G, q, A, prob["b"], prob["xl"], prob["xu"])
    assert best is not None
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    assert np.abs(r["x"] - best[1]).max() <= 1e-6
    assert np.abs(r["y"] - best[2]).max() <= 1e-5 * max(1.0, np.abs(best[2]).max())


def _kkt_certificate(prob, r, tol):
    G, q, A = _qp_data(prob)
    x, y, zl, zu = r["x"], r["y"], r["zl"], r["zu"]
    stat = G @ x + q + A.T @ y - zl + zu
    assert np.abs(A @ x - prob["b"]).max() <= tol
    assert np.abs(stat).max() <= tol * max(1.0, (np.abs(y).sum() + np.abs(zl).sum() + np.abs(zu).sum()) / (len(y) + 2 * len(x)) / 100.0)
    assert np.all(zl > 0) and np.all(zu > 0)
    assert np.all(x > prob["xl"]) and np.all(x < prob["xu"])
    assert np.abs((x - prob["xl"]) * zl).max() <= tol * max(1.0, (zl.sum() + zu.sum()) / (2 * len(x)) / 100.0)
    assert np.abs((prob["xu"] - x) * zu).max() <= tol * max(1.0, (zl.sum() + zu.sum()) / (2 * len(x)) / 100.0)


def test_config0_ipm_certificate_and_decoupled_variables():
    prob = synth.config_problem(synth.IPM_N192)
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    assert r["iters"] < 200
    _kkt_certificate(prob, r, 1e-8)
    # sparse variables that appear in no constraint: 1-D box QPs
    used = np.zeros(prob["n_s"], dtype=bool)
    used[prob["ci"]] = True
    free = np.where(~used)[0]
    assert len(free) > 100
    xs = r["x"][prob["n_d"]:]
    u = -prob["g"] / prob["w"]
    expect = np.clip(u, -1.0, 1.0)
    err = np.abs(xs[free] - expect[free])
    # strictly complementary variables (unconstrained minimiser at least 0.01
    # away from a bound) are accurate to the barrier bias; degenerate ones
    # (minimiser at a bound with a vanishing multiplier) only to O(sqrt(mu))
    # Error bound implied by the stopping test E_0 <= tol on the 1-D problem:
    # interior minimiser: |x - x*| <= tol (s_d + s_c (1/s_l + 1/s_u)) / w;
    # minimiser at a bound with multiplier z* = w |u| - w > 0: the slack is
    # at most tol s_c / z with z >= z* - tol s_d.
    tol = 1e-8
    zl, zu, y = r["zl"], r["zu"], r["y"]
    ntot = len(r["x"])
    sd = max(1.0, (np.abs(y).sum() + zl.sum() + zu.sum()) / (len(y) + 2 * ntot) / 100.0)
    sc = max(1.0, (zl.sum() + zu.sum()) / (2 * ntot) / 100.0)
    xf, wf, uf = xs[free], prob["w"][free], u[free]
    margin = np.abs(uf) - 1.0
    inner = margin < -1e-3
    bound_in = tol * (sd + sc * (1.0 / (xf + 1.0) + 1.0 / (1.0 - xf))) / wf
    assert np.all(err[inner] <= 2.0 * bound_in[inner])
    outer = margin > 1e-3
    zstar = wf * margin - tol * sd
    assert np.all(err[outer] <= 2.0 * tol * sc / zstar[outer])
    # degenerate ones (minimiser within 1e-3 of a bound): O(sqrt(tol))
    assert err.max() <= 1e-4
    # second order: the KKT matrix at the solution (with the final barrier
    # diagonal) has inertia (n, 0, m)
    x, zl, zu = r["x"], r["zl"], r["zu"]
    sig = zl / (x - prob["xl"]) + zu / (prob["xu"] - x)
    nd = prob["n_d"]
    K = full_kkt(prob, sig[:nd], prob["w"] + sig[nd:])
    n = nd + prob["n_s"]
    ev = np.linalg.eigvalsh(K)
    assert sign_counts(ev) == (n, 0, prob["m"])


@pytest.mark.parametrize("seed", range(3))
def test_ipm_other_seeds_converge(seed):
    prob = synth.make_problem(32, 800, 64, 4, cfg=202, p=seed)
    r = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == "converged"
    _kkt_certificate(prob, r, 1e-8)


def test_reduced_direction_equals_unreduced_newton():
    prob = synth.make_problem(4, 9, 3, 2, cfg=203)
    it = synth.interior_iterate(prob, 3)
    P = oracle.Problem(prob)
    mu = it["mu"]
    sig, rx, ry = oracle.sigma_rhs(P, it["x"], it["y"], it["zl"], it["zu"], mu)
    nd = prob["n_d"]
    F = oracle.Factor(P).once(sig[:nd], prob["w"] + sig[nd:], 0.0, 0.0)
    dxd, dxs, dy, st = F.solve(rx[:nd], rx[nd:], ry)
    assert st == 0
    # unreduced primal-dual Newton system in (dx, dy, dzl, dzu)
    G, q, A = _qp_data(prob)
    n, m = G.shape[0], A.shape[0]
    x, y, zl, zu = it["x"], it["y"], it["zl"], it["zu"]
    sl, su = x - prob["xl"], prob["xu"] - x
    I = np.eye(n)
    KK = np.block([
        [G, A.T, -I, I],
        [A, np.zeros((m, m)), np.zeros((m, n)), np.zeros((m, n))],
        [np.diag(zl), np.zeros((n, m)), np.diag(sl), np.zeros((n, n))],
        [-np.diag(zu), np.zeros((n, m)), np.zeros((n, n)), np.diag(su)]])
    F0 = np.concatenate([G @ x + q + A.T @ y - zl + zu, A @ x - prob["b"], sl * zl - mu, su * zu - mu])
    d = np.linalg.solve(KK, -F0)
    assert np.allclose(np.concatenate([dxd, dxs]), d[:n], rtol=1e-9, atol=1e-11)
    assert np.allclose(dy, d[n:n + m], rtol=1e-9, atol=1e-11)


def test_rhs_is_minus_barrier_lagrangian_gradient():
    prob = synth.make_problem(3, 5, 2, 2, cfg=204)
    it = synth.interior_iterate(prob, 1)
    P = oracle.Problem(prob)
    mu = 0.05
    _, rx, ry = oracle.sigma_rhs(P, it["x"], it["y"], it["zl"], it["zu"], mu)
    G, q, A = _qp_data(prob)

    def lag(x):
        return oracle.barrier(P, x, mu) + it["y"] @ (A @ x - prob["b"])

    h = 1e-6
    for i in range(len(it["x"])):
        e = np.zeros(len(it["x"]))
        e[i] = h
        fd = (lag(it["x"] + e) - lag(it["x"] - e)) / (2 * h)
        assert -rx[i] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    assert np.allclose(-ry, A @ it["x"] - prob["b"], rtol=1e-13, atol=1e-13)


def test_theta_zero_at_generating_point():
    prob = synth.config_problem(synth.IPM_N192)
    P = oracle.Problem(prob)
    assert oracle.theta(P, prob["x0"]) <= 1e-12 * prob["m"]


@pytest.mark.parametrize("seed", range(5))
def test_fraction_to_boundary_definition(seed):
    rng = np.random.default_rng(seed)
    v = 10.0 ** rng.uniform(-3, 1, 200)
    dv = rng.standard_normal(200) * 10.0 ** rng.uniform(-2, 2, 200)
    tau = 0.99
    a = oracle.ftb(v, dv, tau)
    assert 0.0 < a <= 1.0
    assert np.all(v + a * dv >= (1 - tau) * v - 1e-12 * v)
    if a < 1.0:
        # some entry is exactly at its fraction-to-boundary limit
        slack = (v + a * dv - (1 - tau) * v) / v
        assert np.abs(slack).min() <= 1e-12
        assert np.any(v + (a * (1 + 1e-9)) * dv < (1 - tau) * v)
    # all-positive direction: full step
    assert oracle.ftb(v, np.abs(dv), tau) == 1.0


def test_opt_error_zero_at_exact_kkt_point():
    prob = synth.make_problem(2, 4, 2, 2, cfg=201, p=1)
    prob["H"] = np.asfortranarray(prob["H"] + 1.5 * np.eye(2))
    G, q, A = _qp_data(prob)
    f, x, y = _brute_force_box_qp(G, q, A, prob["b"], prob["xl"], prob["xu"])
    gl = G @ x + q + A.T @ y
    zl, zu = np.maximum(gl, 0.0), np.maximum(-gl, 0.0)
    e, parts = oracle.opt_error(oracle.Problem(prob), x, y, zl, zu, 0.0)
    assert e <= 1e-13

"""Pins for the oracle's general-NLP IPM (model objects from an external
modeling layer, the end of Sec. 2.3; the filter line search of Sec. 2.1 with
its second-order correction and feasibility restoration), against what the
mathematics fixes:

* the test family's model (objective, gradient, rows, Jacobian, Hessian of
  the Lagrangian) agrees with central finite differences;
* a circle-constrained linear objective has the closed-form solution
  x* = centre - R c/||c||, y* = ||c|| / (2R) (one case takes a second-order
  correction on the way);
* family members end at KKT points certified in numpy (first-order
  conditions from an independent evaluation of the model, bounds,
  complementarity) with second-order inertia (n_d, 0, m) of the last Newton
  matrix; a member whose first trial points raise the violation is rescued
  by a second-order correction;
* a forced restoration lowers theta by the required factor and the IPM still
  ends at the same point; with no nonlinear terms the NLP path reaches the
  quadratic oracle's solution;
* inequality rows with nonlinear terms converge to a certified point.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import dense_js


def _family(nd=16, ns=300, m=24, r=3, p=0, q_scale=0.5, m_I=0, cfg=500):
    prob = synth.make_problem(nd, ns, m, r, cfg=cfg, p=p, m_I=m_I)
    return synth.nlp_terms(prob, cfg, p, q_scale=q_scale)


def _np_model(q, x, y):
    """The family's derivatives written out in numpy from the problem data."""
    nd, ns, m = q["n_d"], q["n_s"], q["m"]
    H, c, w, g, e, Q = q["H"], q["c"], q["w"], q["g"], q["e"], q["Q"]
    xd, xs = x[:nd], x[nd:nd + ns]
    Js = dense_js(q)
    Jd = np.asarray(q["Jd"]).reshape(m, nd) + 2.0 * Q * xd[None, :]
    grad = np.concatenate([H @ xd + c, w * xs + g + e * (np.exp(xs) - 1.0)])
    rows = np.asarray(q["Jd"]).reshape(m, nd) @ xd + Js @ xs + Q @ (xd * xd)
    return grad, np.hstack([Jd, Js]), rows


def test_model_derivatives_match_finite_differences():
    q = _family(nd=6, ns=20, m=8, r=3, p=1, q_scale=1.0)
    P = oracle.Problem(q)
    rng = np.random.default_rng(3)
    n, m = 26, 8
    x = rng.uniform(-0.8, 0.8, n)
    y = rng.standard_normal(m)
    ev = oracle.nlp_test_eval(P, q["Q"], q["e"], x, y)
    h = 1e-6
    fd_g = np.zeros(n)
    fd_J = np.zeros((m, n))
    for i in range(n):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        ep = oracle.nlp_test_eval(P, q["Q"], q["e"], xp, y)
        em = oracle.nlp_test_eval(P, q["Q"], q["e"], xm, y)
        fd_g[i] = (ep["f"] - em["f"]) / (2 * h)
        fd_J[:, i] = (ep["c"] - em["c"]) / (2 * h)
    assert np.allclose(ev["g"], fd_g, rtol=1e-6, atol=1e-7)
    J = np.hstack([ev["Jd"], dense_js(dict(q, v=ev["v"]))])
    assert np.allclose(J, fd_J, rtol=1e-6, atol=1e-7)
    # Hessian of the Lagrangian: finite differences of grad f + J' y
    def lag_grad(xx):
        e2 = oracle.nlp_test_eval(P, q["Q"], q["e"], xx, y)
        Jx = np.hstack([e2["Jd"], dense_js(dict(q, v=e2["v"]))])
        return e2["g"] + Jx.T @ y
    HL = np.zeros((n, n))
    for i in range(n):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        HL[:, i] = (lag_grad(xp) - lag_grad(xm)) / (2 * h)
    assert np.allclose(HL[:6, :6], ev["H"], rtol=1e-5, atol=1e-6)
    assert np.allclose(np.diag(HL)[6:], ev["w"], rtol=1e-5, atol=1e-6)
    assert np.abs(HL[6:, 6:] - np.diag(np.diag(HL)[6:])).max() <= 1e-6   # A2: diagonal
    assert np.abs(HL[:6, 6:]).max() <= 1e-6                              # A1: no cross terms
    # the numpy evaluation of the same model
    gn, Jn, rows = _np_model(q, x, y)
    assert np.allclose(ev["g"], gn, rtol=1e-12, atol=1e-12)
    assert np.allclose(J, Jn, rtol=1e-12, atol=1e-12)


def _circle(cvec, a):
    prob = dict(n_d=2, n_s=0, m=1, r=0, H=np.zeros((2, 2), order="F"),
                c=np.array(cvec, float), w=np.zeros(0), g=np.zeros(0),
                Jd=np.asfortranarray([[a, 0.0]]), rp=np.array([0, 0], np.int32),
                ci=np.zeros(0, np.int32), v=np.zeros(0), b=np.array([1.0]),
                xl=np.full(2, -5.0), xu=np.full(2, 5.0), x0=np.zeros(2), m_I=0,
                hl=np.zeros(0), hu=np.zeros(0))
    return prob, np.asfortranarray([[1.0, 1.0]]), np.zeros(0)


@pytest.mark.parametrize("cvec,a,soc", [([1.0, 0.5], 0.3, True), ([-2.0, 1.0], 0.5, False),
                                        ([0.3, -1.2], -0.7, False)])
def test_circle_closed_form(cvec, a, soc):
    prob, Q, e = _circle(cvec, a)
    r = oracle.nlp_test_ipm(oracle.Problem(prob), Q, e)
    c = np.array(cvec)
    R = np.sqrt(1.0 + a * a / 4.0)
    xs = np.array([-a / 2.0, 0.0]) - R * c / np.linalg.norm(c)
    assert r["status"] == "converged"
    assert np.abs(r["x"] - xs).max() <= 1e-8
    assert abs(r["y"][0] - np.linalg.norm(c) / (2.0 * R)) <= 1e-8
    assert (r["soc_accepted"] > 0) == soc


def _certificate(q, r, tol=1e-8):
    nd, ns, m = q["n_d"], q["n_s"], q["m"]
    n = nd + ns
    mI = int(q.get("m_I", 0))
    mE = m - mI
    x, y, zl, zu = r["x"], r["y"], r["zl"], r["zu"]
    gn, J, rows = _np_model(q, x[:n], y)
    # the rows: equalities at b, inequalities at their slack, inside [hl, hu]
    assert np.abs(rows[:mE] - q["b"][:mE]).max(initial=0.0) <= tol
    if mI:
        d = x[n:]
        assert np.abs(rows[mE:] - d).max() <= tol
        assert np.all(d > q["hl"]) and np.all(d < q["hu"])
    lo = np.concatenate([q["xl"], q.get("hl", np.zeros(0))])
    up = np.concatenate([q["xu"], q.get("hu", np.zeros(0))])
    gl = np.concatenate([gn + J.T @ y, -y[mE:]])
    zlf = np.where(np.isfinite(lo), zl, 0.0)
    zuf = np.where(np.isfinite(up), zu, 0.0)
    sd = max(1.0, (np.abs(y).sum() + zlf.sum() + zuf.sum()) / (m + 2 * len(x)) / 100.0)
    assert np.abs(gl - zlf + zuf).max() <= tol * sd
    sc = max(1.0, (zlf.sum() + zuf.sum()) / (2 * len(x)) / 100.0)
    fin = np.isfinite(lo)
    assert np.abs((x - lo)[fin] * zl[fin]).max(initial=0.0) <= tol * sc
    fin = np.isfinite(up)
    assert np.abs((up - x)[fin] * zu[fin]).max(initial=0.0) <= tol * sc
    last = r["trace"][r["iters"] - 1]
    assert tuple(last["inertia"]) == (nd, 0, m)


@pytest.mark.parametrize("p,q_scale", [(0, 0.5), (2, 1.0), (5, 2.0)])
def test_family_kkt_certificate(p, q_scale):
    q = _family(p=p, q_scale=q_scale)
    r = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"])
    assert r["status"] == "converged"
    _certificate(q, r)


def test_second_order_correction_rescues_a_step():
    q = _family(p=4, q_scale=2.0)
    r = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"])
    assert r["status"] == "converged" and r["soc_accepted"] >= 1
    k = [t["soc"] for t in r["trace"][:r["iters"]]].index(1)
    # the corrected point was accepted where the plain trial point raised theta
    assert r["trace"][k]["backtracks"] == 0
    _certificate(q, r)


def test_forced_restoration_reduces_theta_and_still_converges():
    q = _family(p=0, q_scale=0.5)
    P = oracle.Problem(q)
    r0 = oracle.nlp_test_ipm(P, q["Q"], q["e"])
    r = oracle.nlp_test_ipm(P, q["Q"], q["e"], force_resto=2)
    assert r["resto_calls"] == 1 and r["trace"][2]["resto"] >= 1
    assert r["trace"][3]["theta"] <= 0.9 * r["trace"][2]["theta"]
    assert r["status"] == "converged"
    assert np.abs(r["x"] - r0["x"]).max() <= 1e-6
    _certificate(q, r)


def test_no_nonlinear_terms_reduces_to_the_quadratic_ipm():
    prob = synth.make_problem(16, 300, 24, 3, cfg=501)
    q = dict(prob, Q=np.zeros((24, 16), order="F"), e=np.zeros(300))
    rn = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"])
    rq = oracle.ipm(oracle.Problem(prob))
    assert rn["status"] == rq["status"] == "converged"
    assert np.abs(rn["x"] - rq["x"]).max() <= 1e-8 * max(1.0, np.abs(rq["x"]).max())
    assert np.abs(rn["y"] - rq["y"]).max() <= 1e-8 * max(1.0, np.abs(rq["y"]).max())


def test_nonlinear_inequality_rows():
    q = _family(nd=12, ns=200, m=20, p=1, q_scale=1.0, m_I=8, cfg=502)
    r = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"])
    assert r["status"] == "converged"
    _certificate(q, r)

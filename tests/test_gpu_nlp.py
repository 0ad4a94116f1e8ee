"""General NLP (model objects from an external modeling layer, the end of
Sec. 2.3) on the GPU against the CPU oracle, through the C-ABI.

The library's built-in separable model (mds_sep_model_*) supplies the
callbacks; the oracle evaluates the same family in plain C.  In NLP mode the
IPM's filter line search (Sec. 2.1) adds the second-order correction and the
feasibility restoration.

Bars: whole IPMs take the same number of iterations as the oracle with the
same per-iteration barrier parameter, inertia, correction trials,
backtracks, second-order corrections and restoration phases, and end within
1e-8 of the oracle's x (variables and slacks) and y; forced restoration
lowers theta by the phase's factor; with no nonlinear terms NLP mode takes
the quadratic IPM's path; invalid uses are refused before any work.
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


def _family(nd=16, ns=300, m=24, r=3, p=0, q_scale=0.5, m_I=0, cfg=500):
    prob = synth.make_problem(nd, ns, m, r, cfg=cfg, p=p, m_I=m_I)
    return synth.nlp_terms(prob, cfg, p, q_scale=q_scale)


def _gpu_solve(q, nb=0, force_at=-1):
    S = mds.solver_for(q, nb=nb, nlp=True)
    S.set_sep_model(q["Q"], q["e"])
    if force_at < 0:
        r = S.ipm_solve()
    else:
        it = S.new_iterate()
        S.ipm_init(it)
        trace, code = [], 0
        while True:
            if it["c"].iter == force_at:
                S.set_debug(mds.MDS_DEBUG_FORCE_RESTO)
            code, info = S.ipm_step(it)
            trace.append(info)
            if code != 0:
                break
        r = dict(status=mds.STATUS_NAMES.get(code, code), code=code, iters=it["c"].iter,
                 trace=trace, x=it["x"], y=it["y"], zl=it["zl"], zu=it["zu"])
    r["stats"] = S.nlp_stats()
    return S, r


def _compare(q, r_g, r_o):
    assert r_g["status"] == r_o["status"] == "converged", (r_g["status"], r_o["status"])
    assert r_g["iters"] == r_o["iters"]
    for k in range(r_o["iters"]):
        a, b = r_g["trace"][k], r_o["trace"][k]
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-10), k
        assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], k
        assert a["backtracks"] == b["backtracks"], k
        assert (a["nlp_event"] == 1) == (b["soc"] == 1), k
        assert (a["nlp_event"] == 2) == (b["resto"] != 0), k
    st = r_g["stats"]
    assert (st["soc_trials"], st["soc_accepted"]) == (r_o["soc_trials"], r_o["soc_accepted"])
    assert (st["resto_calls"], st["resto_iters"]) == (r_o["resto_calls"], r_o["resto_iters"])
    x, y = _np(r_g["x"]), _np(r_g["y"])
    assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())
    assert np.abs(y - r_o["y"]).max(initial=0.0) <= 1e-8 * max(1.0, np.abs(r_o["y"]).max(initial=0.0))


FAMILY = [
    # (n_d, n_s, m, r, p, q_scale, m_I, cfg, nb)
    (16, 300, 24, 3, 0, 0.5, 0, 500, 0),
    (16, 300, 24, 3, 2, 1.0, 0, 500, 0),
    (16, 300, 24, 3, 5, 2.0, 0, 500, 0),
    (16, 300, 24, 3, 4, 2.0, 0, 500, 0),      # a second-order correction is accepted
    (12, 200, 20, 3, 1, 1.0, 8, 502, 0),      # nonlinear inequality rows
    (64, 3000, 192, 4, 1, 1.0, 0, 500, 16),   # N = 256: several panels, ragged tail
    (48, 2000, 150, 4, 2, 1.0, 60, 503, 8),   # inequality rows, N = 198
    (0, 400, 30, 3, 0, 0.5, 0, 504, 0),       # no dense block: e terms only
]


@pytest.mark.parametrize("idx", range(len(FAMILY)))
def test_nlp_ipm_matches_oracle(idx):
    nd, ns, m, r, p, qs, mI, cfg, nb = FAMILY[idx]
    q = _family(nd, ns, m, r, p, qs, mI, cfg)
    say(f"nlp family {FAMILY[idx]}")
    r_o = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"])
    _, r_g = _gpu_solve(q, nb=nb)
    _compare(q, r_g, r_o)
    if idx == 3:
        assert r_g["stats"]["soc_accepted"] >= 1


def _circle(cvec, a):
    prob = dict(n_d=2, n_s=0, m=1, r=0, H=np.zeros((2, 2), order="F"),
                c=np.array(cvec, float), w=np.zeros(0), g=np.zeros(0),
                Jd=np.asfortranarray([[a, 0.0]]), rp=np.array([0, 0], np.int32),
                ci=np.zeros(0, np.int32), v=np.zeros(0), b=np.array([1.0]),
                xl=np.full(2, -5.0), xu=np.full(2, 5.0), x0=np.zeros(2), m_I=0,
                hl=np.zeros(0), hu=np.zeros(0))
    return dict(prob, Q=np.asfortranarray([[1.0, 1.0]]), e=np.zeros(0))


@pytest.mark.parametrize("cvec,a", [([1.0, 0.5], 0.3), ([-2.0, 1.0], 0.5)])
def test_circle_closed_form(cvec, a):
    q = _circle(cvec, a)
    say(f"nlp circle c={cvec} a={a}")
    r_o = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"])
    _, r_g = _gpu_solve(q)
    _compare(q, r_g, r_o)
    c = np.array(cvec)
    R = np.sqrt(1.0 + a * a / 4.0)
    xs = np.array([-a / 2.0, 0.0]) - R * c / np.linalg.norm(c)
    assert np.abs(_np(r_g["x"]) - xs).max() <= 1e-8


def test_forced_restoration_matches_oracle():
    q = _family(p=0, q_scale=0.5)
    say("nlp forced restoration at iteration 2")
    r_o = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], q["e"], force_resto=2)
    _, r_g = _gpu_solve(q, force_at=2)
    assert r_g["trace"][2]["nlp_event"] == 2
    assert r_g["trace"][3]["theta"] <= 0.9 * r_g["trace"][2]["theta"]
    _compare(q, r_g, r_o)


def test_no_nonlinear_terms_take_the_quadratic_path():
    prob = synth.make_problem(16, 300, 24, 3, cfg=501)
    q = dict(prob, Q=np.zeros((24, 16), order="F"), e=np.zeros(300))
    say("nlp with zero nonlinear terms vs quadratic IPM")
    S, r_n = _gpu_solve(q)
    S.set_nlp(None)
    r_q = S.ipm_solve()
    assert r_n["status"] == r_q["status"] == "converged"
    assert r_n["iters"] == r_q["iters"]
    for a, b in zip(r_n["trace"][:r_n["iters"]], r_q["trace"][:r_q["iters"]]):
        assert a["inertia"] == b["inertia"] and a["backtracks"] == b["backtracks"]
    xq = _np(r_q["x"])
    assert np.abs(_np(r_n["x"]) - xq).max() <= 1e-8 * max(1.0, np.abs(xq).max())
    # back in quadratic mode the handle reproduces the oracle's quadratic IPM
    r_o = oracle.ipm(oracle.Problem(prob))
    assert np.abs(xq - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())


def test_invalid_nlp_uses_are_refused():
    q = _family(nd=6, ns=40, m=8, r=2, p=0, q_scale=0.5)
    say("nlp refusals")
    S = mds.solver_for(q)          # no room for the model objects
    with pytest.raises(mds.MdsError, match="options.nlp"):
        S.set_sep_model(q["Q"], q["e"])
    S2 = mds.solver_for(q, nlp=True)
    S2.set_sep_model(q["Q"], q["e"])
    with pytest.raises(mds.MdsError, match="quadratic problem"):
        S2.ipm_solve_warm(np.zeros(6), np.zeros(8), 0.1)
    # a model whose sparse Hessian turns negative ends the step with an error
    S3 = mds.solver_for(q, nlp=True)
    S3.set_sep_model(q["Q"], -50.0 * np.ones(40))
    with pytest.raises(mds.MdsError, match="negative"):
        S3.ipm_solve()
    r_o = oracle.nlp_test_ipm(oracle.Problem(q), q["Q"], -50.0 * np.ones(40))
    assert r_o["code"] == 9

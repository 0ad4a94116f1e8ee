"""Parity at the benchmarked size (n_d = 1024, n_s = 200000, m = 3072, N = 4096),
in the launch configuration the benchmark times (default panel choice: the
cooperative register panel), and with the single-workgroup register and
memory panels.

* M is compared bit for bit with the oracle's condensation (all N^2 entries);
* the pivot sequence and inertia are compared with the oracle's unblocked
  Bunch-Kaufman on the same M (one ~15 s CPU factorization);
* the solve is checked by its normwise backward error on the full KKT system
  (a property that holds at any size) and against the oracle's solve;
* one IPM step from the cold start matches the oracle's first iteration.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def big():
    prob = synth.config_problem(synth.OPF_N4096)
    it = synth.interior_iterate(prob, 0)
    P = oracle.Problem(prob)
    sig, rx, ry = oracle.sigma_rhs(P, it["x"], it["y"], it["zl"], it["zu"], it["mu"])
    nd = prob["n_d"]
    return dict(prob=prob, P=P, sig=sig, rx=rx, ry=ry, dsb=prob["w"] + sig[nd:], nd=nd)


@pytest.mark.parametrize("panel", ["auto", "reg", "mem"])
def test_fullsize_condense_factor_solve(big, panel):
    prob, P, nd = big["prob"], big["P"], big["nd"]
    say(f"N=4096 condense/factor/solve panel={panel}")
    S = mds.solver_for(prob, panel=panel)
    S.condense(big["sig"][:nd], big["dsb"], 0.0, 0.0)
    M = S.get_matrix()
    Mo, _ = oracle.condense(P, big["sig"][:nd], big["dsb"], 0.0, 0.0)
    assert np.array_equal(M.view(np.int64), Mo.view(np.int64))
    st, inn, _ = S.factor_inertia()
    L, dd, ds, ipiv = S.get_factor()
    Lo, ddo, dso, ipo, info, _ = oracle.bk(Mo)
    assert np.array_equal(ipiv, ipo), f"first differing pivot {np.argmax(ipiv != ipo)}"
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == oracle.inertia(ipo, ddo, dso)
    assert np.abs(dd - ddo).max() <= 1e-9 * max(1.0, np.abs(ddo).max())
    dx_d, dx_s, dy = [t.cpu().numpy() for t in S.solve(big["rx"][:nd], big["rx"][nd:], big["ry"])]
    F = oracle.Factor(P)
    F.once(big["sig"][:nd], big["dsb"], 0.0, 0.0)
    od, os_, oy, _ = F.solve(big["rx"][:nd], big["rx"][nd:], big["ry"])
    got, ref = np.concatenate([dx_d, dx_s, dy]), np.concatenate([od, os_, oy])
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()
    (rd, rs, ry), info = S.refine(big["rx"][:nd], big["rx"][nd:], big["ry"], 3, 1e-14)
    assert info["eta"] <= 1e-10


def test_fullsize_first_ipm_step(big):
    prob = big["prob"]
    say("N=4096 first IPM step")
    S = mds.solver_for(prob)
    it = S.new_iterate()
    S.ipm_init(it)
    st, info = S.ipm_step(it)
    assert st == 0
    ro = oracle.ipm(big["P"], max_iter=1)
    assert ro["iters"] == 1
    t = ro["trace"][0]
    assert info["inertia"] == t["inertia"] and info["trials"] == t["trials"]
    assert info["alpha_pr"] == pytest.approx(t["alpha_pr"], rel=1e-9)
    assert info["mu"] == t["mu"]
    x = it["x"].cpu().numpy()
    assert np.abs(x - ro["x"]).max() <= 1e-8 * max(1.0, np.abs(ro["x"]).max())

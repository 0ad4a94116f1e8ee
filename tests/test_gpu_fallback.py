"""Failure paths of the Newton step, forced from the host so that every
kernel still ends normally:

* a cooperative panel whose exchange wait expires (forced by the host-set
  test flag, which makes each workgroup report it before its first exchange)
  is redone by the memory panel in FP64; the factorization then has the
  oracle's pivots and inertia, and an IPM step reports the fallback;
* a mixed-precision Newton solve whose GMRES refinement stops above its
  tolerance (its iteration budget cut to 1) is recomputed from an FP64
  factorization of the same system; the IPM still converges to the oracle's
  solution and every such step is flagged.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.mark.parametrize("lookahead", ["off", "on"])
def test_cooperative_abort_refactors_with_memory_panel(lookahead):
    N = 2200
    prob = synth.make_problem(550, 8000, N - 550, 4, cfg=350)
    st = synth.kkt_state(prob, 0, (-2.0, 2.0))
    say(f"cooperative abort fallback N={N} lookahead={lookahead}")
    S = mds.solver_for(prob, lookahead=lookahead)
    assert S.info()["panel"] == "coop"
    assert (S.info()["lookahead_cus"] > 0) == (lookahead == "on")
    S.condense(st["sigma_d"], st["dsbase"])
    _, inn0, _ = S.factor_inertia()
    ipiv0 = S.get_pivots()
    S.set_debug(mds.MDS_DEBUG_COOP_ABORT)
    S.condense(st["sigma_d"], st["dsbase"])
    status, inn, _ = S.factor_inertia()
    assert status == mds.MDS_OK
    assert S.fallbacks()["coop_aborts"] == 1
    assert np.array_equal(S.get_pivots(), ipiv0)
    assert inn == inn0
    F = oracle.Factor(oracle.Problem(prob)).once(st["sigma_d"], st["dsbase"])
    assert np.array_equal(S.get_pivots(), F.ipiv)
    (dxd, dxs, dy), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 3, 1e-14)
    assert info["eta"] <= 1e-12
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    xo = np.concatenate([od, os_, oy])
    x = np.concatenate([t.cpu().numpy() for t in (dxd, dxs, dy)])
    assert np.abs(x - xo).max() <= 1e-8 * np.abs(xo).max()
    # an IPM step under the flag reports the fallback
    it = S.new_iterate()
    S.ipm_init(it)
    code, info = S.ipm_step(it)
    assert code == 0 and info["fallback"] & 2
    S.set_debug(0)
    code, info = S.ipm_step(it)
    assert code == 0 and info["fallback"] == 0


def test_mixed_precision_noconv_falls_back_to_fp64():
    prob = synth.config_problem(synth.IPM_N192)
    say("bf16 IPM with a one-iteration GMRES budget")
    S = mds.solver_for(prob, precision="bf16")
    r = S.ipm_solve(gmres_max=1)
    ro = oracle.ipm(oracle.Problem(prob))
    assert r["status"] == ro["status"] == "converged"
    flagged = [t["fallback"] & 1 for t in r["trace"][:r["iters"]]]
    assert sum(flagged) >= 1
    assert S.fallbacks()["fp64_refactors"] == sum(flagged)
    x = r["x"].cpu().numpy()
    assert np.abs(x - ro["x"]).max() <= 1e-8 * max(1.0, np.abs(ro["x"]).max())

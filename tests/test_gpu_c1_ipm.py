"""A whole FP64 IPM on the OPF-scale workload (n_d = 1024, n_s = 200000,
m = 3072, N = 4096, 6 nonzeros per row of J_s) in the benchmarked launch
configuration (cooperative panel with the register tail), run on the GPU to
E_0 <= 1e-8, with the Newton systems of five iterations (the first, the last
and three in between) replayed against the oracle:

* the pre-step iterate is copied to the host and the oracle rebuilds that
  iteration's system from it (Sigma and the right-hand side at the step's
  barrier parameter, the accepted shifts delta_w, delta_c): the pivot
  sequence the GPU accepted in that step and its inertia (n_d, 0, m) must be
  the oracle's, bit for bit;
* the same system solved by the GPU (condense, factor, refine) against the
  oracle's refined solve: within 1e-8 of the oracle's solution, or, where the
  late-barrier system is too ill-conditioned for that, with backward error
  <= 1e-10 on the full system (both backward stable; the forward difference
  is then bounded by the condition number, not by the method);
* at termination the optimality error is <= 1e-8 (recomputed by the oracle
  from the final iterate) and the iteration count is reported.

The oracle factors N = 4096 in ~7 s on one core; its elimination is split
over host threads (bit-identical to one thread).
"""
import os

import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_c1_whole_ipm_with_step_replays():
    prob = synth.config_problem(synth.OPF_N4096)
    nd, m = prob["n_d"], prob["m"]
    P = oracle.Problem(prob)
    say("N=4096 whole FP64 IPM")
    S = mds.solver_for(prob)
    assert S.info()["panel"] == "coop"
    it = S.new_iterate()
    S.ipm_init(it)
    pre, infos, pivs = [], [], []
    while True:
        snap = [it[k].cpu().numpy().copy() for k in ("x", "y", "zl", "zu")]
        code, info = S.ipm_step(it)
        if code != 0:
            break
        pre.append(snap)
        infos.append(info)
        pivs.append(S.get_pivots().copy())
        assert len(infos) < 200
    assert code == mds.MDS_IPM_CONVERGED
    K = len(infos)
    x, y, zl, zu = [it[k].cpu().numpy() for k in ("x", "y", "zl", "zu")]
    E0, _ = oracle.opt_error(P, x, y, zl, zu, 0.0)
    say(f"  converged in {K} iterations, E_0 = {E0:.2e} (oracle recomputation)")
    assert E0 <= 1e-8
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        for k in sorted({0, K // 4, K // 2, (3 * K) // 4, K - 1}):
            xk, yk, zlk, zuk = pre[k]
            inf = infos[k]
            mu, dw, dc = inf["mu"], inf["dw"], inf["dc"]
            sig, rx, ry = oracle.sigma_rhs(P, xk, yk, zlk, zuk, mu)
            dsb = prob["w"] + sig[nd:]
            F = oracle.Factor(P).once(sig[:nd], dsb, dw, dc)
            assert np.array_equal(pivs[k], F.ipiv), (k, int(np.argmax(pivs[k] != F.ipiv)))
            assert F.inertia == inf["inertia"] == (nd, 0, m), k
            od, os_, oy, _, eta_o = F.refine(rx[:nd], rx[nd:], ry, 2, 1e-14)
            ref = np.concatenate([od, os_, oy])
            S.condense(sig[:nd], dsb, dw, dc)
            S.factor_inertia()
            (gd, gs, gy), ri = S.refine(rx[:nd], rx[nd:], ry, 2, 1e-14)
            got = np.concatenate([t.cpu().numpy() for t in (gd, gs, gy)])
            rel = np.abs(got - ref).max() / np.abs(ref).max()
            say(f"  iteration {k}: mu {mu:.1e}, trials {inf['trials']}, pivots identical, "
                f"rel diff {rel:.1e}, eta gpu {ri['eta']:.1e} oracle {eta_o:.1e}")
            assert rel <= 1e-8 or ri["eta"] <= 1e-10
    finally:
        oracle.set_threads(1)

"""Mixed-precision factorization (FP32 storage of the trailing matrix with FP32
or BF16 MFMA products) refined by FP64 GMRES on the full Newton system.

Bars (the factor is only a preconditioner here, so its own error is reported
rather than bounded tightly):
* refined solution within 1e-8 (relative, max-norm) of the oracle's FP64
  solve, and normwise backward error on the full KKT system <= 1e-12;
* GMRES iterations bounded (FP32 <= 10, BF16 <= 40) at these sizes;
* the low-precision factor reconstructs the equilibrated S M S to the
  precision's accuracy, with the inertia of the FP64 factorization;
* a whole IPM in mixed precision converges to the oracle's solution.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth
from helpers import block_d, full_kkt, perm_from_ipiv

pytestmark = pytest.mark.gpu

ITER_CAP = {"fp32": 10, "bf16": 40, "bf16x3": 12}
D_TOL = {"fp32": 1e-4, "bf16": 5e-2, "bf16x3": 1e-3}


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _np(t):
    return t.detach().cpu().numpy()


CASES = [
    # (n_d, n_s, m, r, nb) -- N from one ragged panel to several row tiles
    (64, 2000, 128, 4, 0),
    (10, 40, 27, 3, 8),
    (100, 900, 200, 4, 16),
    (150, 3000, 550, 6, 0),
    (300, 8000, 900, 5, 0),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("idx", range(len(CASES)))
def test_mixed_solve_matches_fp64_oracle(idx, prec):
    nd, ns, m, r, nb = CASES[idx]
    prob = synth.make_problem(nd, ns, m, r, cfg=500 + idx, p=0)
    st = synth.kkt_state(prob, 0, (-1.0, 1.0))
    say(f"mixed {prec} case={CASES[idx]}")
    S = mds.solver_for(prob, nb=nb, precision=prec)
    assert S.info()["precision"] == prec
    S.condense(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    S.factor_inertia()
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 60, 1e-14)
    P = oracle.Problem(prob)
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    got = np.concatenate([_np(rd), _np(rs), _np(ry)])
    ref = np.concatenate([od, os_, oy])
    say(f"  gmres iterations={info['steps']} eta={info['eta']:.2e}")
    assert info["eta"] <= 1e-12
    assert info["steps"] <= ITER_CAP[prec]
    assert np.abs(got - ref).max() <= 1e-8 * max(np.abs(ref).max(), 1e-300)
    if nd + ns + m <= 2500:
        K = full_kkt(prob, st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
        rr = np.concatenate([st["r_d"], st["r_s"], st["r_y"]])
        eta = np.abs(rr - K @ got).max() / (np.abs(K).sum(1).max() * np.abs(got).max()
                                             + np.abs(rr).max())
        assert eta <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_mixed_factor_reconstructs_equilibrated_matrix(prec):
    # the low-precision factor is of S M S, S = diag(1/sqrt(row max |M|)):
    # P (S M S) P' = L D L' within the precision, and In(M) is the FP64 one
    prob = synth.make_problem(150, 3000, 550, 6, cfg=510, p=1)
    st = synth.kkt_state(prob, 1, (-1.0, 1.0))
    say(f"mixed factor reconstruction {prec}")
    S64 = mds.solver_for(prob)
    S64.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    M = S64.get_matrix()
    _, inn64, _ = S64.factor_inertia()
    S = mds.solver_for(prob, precision=prec)
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    _, inn, _ = S.factor_inertia()
    L, dd, ds, ipiv = S.get_factor()
    N = M.shape[0]
    s = 1.0 / np.sqrt(np.abs(M).max(axis=0))
    A = s[:, None] * M * s[None, :]
    p = perm_from_ipiv(ipiv)
    Lu = np.tril(L, -1) + np.eye(N)
    R = Lu @ block_d(ipiv, dd, ds) @ Lu.T
    err = np.abs(A[np.ix_(p, p)] - R).max() / np.abs(A).max()
    say(f"  reconstruction error {err:.2e}")
    assert err <= D_TOL[prec]
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == (inn64["npos"], inn64["nzero"], inn64["nneg"])


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_mixed_ipm_converges_to_oracle_solution(prec):
    prob = synth.config_problem(synth.IPM_N192)
    say(f"mixed ipm N=192 {prec}")
    r_o = oracle.ipm(oracle.Problem(prob))
    S = mds.solver_for(prob, precision=prec)
    r_g = S.ipm_solve()
    assert r_g["status"] == r_o["status"] == "converged"
    assert abs(r_g["iters"] - r_o["iters"]) <= 2
    x = _np(r_g["x"])
    assert np.abs(x - r_o["x"]).max() <= 1e-7 * max(1.0, np.abs(r_o["x"]).max())


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_cooperative_panel(prec):
    # N = 1200 over two cooperating workgroups, nb = 32
    nd, ns, m, r, _ = CASES[4]
    prob = synth.make_problem(nd, ns, m, r, cfg=504, p=0)
    st = synth.kkt_state(prob, 0, (-1.0, 1.0))
    say(f"mixed {prec} cooperative panel N={nd + m}")
    S = mds.solver_for(prob, panel="coop", precision=prec)
    assert S.info()["panel"] == "coop" and S.info()["nb"] == 32
    S.condense(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    S.factor_inertia()
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 60, 1e-14)
    P = oracle.Problem(prob)
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    got = np.concatenate([_np(rd), _np(rs), _np(ry)])
    ref = np.concatenate([od, os_, oy])
    assert info["eta"] <= 1e-12
    assert info["steps"] <= ITER_CAP[prec]
    assert np.abs(got - ref).max() <= 1e-8 * max(np.abs(ref).max(), 1e-300)


def test_mixed_automatic_panel_register_tail():
    # N = 2200: the automatic choice runs the cooperative panel on the FP32
    # trailing matrix and the register panel over its last <= 1024 rows
    nd, ns, m, r = 500, 6000, 1700, 5
    prob = synth.make_problem(nd, ns, m, r, cfg=530, p=0)
    st = synth.kkt_state(prob, 0, (-1.0, 1.0))
    say(f"mixed fp32 automatic panel (register tail) N={nd + m}")
    S = mds.solver_for(prob, precision="fp32")
    assert S.info()["panel"] == "coop"
    S.condense(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    S.factor_inertia()
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 60, 1e-14)
    P = oracle.Problem(prob)
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    got = np.concatenate([_np(rd), _np(rs), _np(ry)])
    ref = np.concatenate([od, os_, oy])
    assert info["eta"] <= 1e-12
    assert info["steps"] <= ITER_CAP["fp32"]
    assert np.abs(got - ref).max() <= 1e-8 * max(np.abs(ref).max(), 1e-300)


def test_mixed_needs_register_panel():
    prob = synth.make_problem(10, 40, 27, 3, cfg=520, p=0)
    with pytest.raises(mds.MdsError):
        mds.solver_for(prob, panel="mem", precision="fp32")

"""GPU parity of the coupling blocks of the sparse Hessian (assumption A2 of
Sec. 2 in its general form; mds_set_sparse_blocks), through the C-ABI:

* condensation (the blocks' L Delta L', the transformed Jacobian J_s L^{-T}
  and the Schur term over it) is bit-identical to the oracle's: M and
  1/Delta, for blocks of 1..16 variables and shapes with n_d = 0 and m = 1;
  removing the blocks restores the plain M bit for bit;
* the correction loop lands on In(M) = (n_d, 0, m) and the refined solve
  matches the oracle's within 1e-8 with backward error <= 1e-10 on the full
  system with the block-diagonal (x_s, x_s) block (checked with a dense
  solve in numpy);
* whole IPMs take the same number of iterations as the oracle with the same
  per-iteration barrier parameter, inertia, trials and backtracks, and end
  within 1e-8 of its x and y;
* invalid blocks are rejected, the warm start is refused while blocks are
  set, and mds_set_problem removes them.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth
from helpers import full_kkt

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _blockdiag(prob):
    ns, bp, Wb = prob["n_s"], prob["bp"], prob["Wb"]
    W = np.zeros((ns, ns))
    off = 0
    for b in range(len(bp) - 1):
        k0, sz = bp[b], bp[b + 1] - bp[b]
        W[k0:k0 + sz, k0:k0 + sz] = Wb[off:off + sz * sz].reshape(sz, sz, order="F")
        off += sz * sz
    return W


SHAPES = [  # (n_d, n_s, m, r, sblk)
    (64, 2000, 128, 4, 4),
    (10, 300, 27, 3, 16),
    (0, 400, 40, 3, 5),
    (20, 200, 1, 6, 3),
    (150, 3000, 550, 6, 8),
]


@pytest.mark.parametrize("idx", range(len(SHAPES)))
def test_sblock_condense_bit_exact(idx):
    nd, ns, m, r, sb = SHAPES[idx]
    prob = synth.make_problem(nd, ns, m, r, cfg=430 + idx, sblk=sb)
    st = synth.kkt_state(prob, idx, (-1.0, 1.0))
    say(f"coupling blocks condense shape={SHAPES[idx]}")
    S = mds.solver_for(prob)
    P = oracle.Problem(prob)
    for dw, dc in ((0.0, 0.0), (1e-4, 1e-8)):
        S.condense(st["sigma_d"], st["dsbase"], dw, dc)
        M = S.get_matrix()
        Mo, invo = oracle.condense(P, st["sigma_d"], st["dsbase"], dw, dc)
        assert np.array_equal(M.view(np.int64), Mo.view(np.int64))
        assert np.array_equal(S.get_inv_ds().view(np.int64), invo.view(np.int64))
    S.set_sparse_blocks(None)
    S.condense(st["sigma_d"], st["dsbase"], 1e-4, 1e-8)
    q = {k: v for k, v in prob.items() if k not in ("bp", "Wb")}
    Mp, _ = oracle.condense(oracle.Problem(q), st["sigma_d"], st["dsbase"], 1e-4, 1e-8)
    assert np.array_equal(S.get_matrix().view(np.int64), Mp.view(np.int64))


@pytest.mark.parametrize("seed", [0, 1])
def test_sblock_correction_and_refined_solve(seed):
    prob = synth.make_problem(20, 300, 30, 3, cfg=440, p=seed, s_scale=6.0, sblk=6)
    st = synth.kkt_state(prob, seed, (-1.0, 1.0))
    say(f"coupling blocks solve seed={seed}")
    S = mds.solver_for(prob)
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    status, inn, reg = S.factor_inertia(mu=1e-2, reg=dict(delta_w_last=0.0))
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == (20, 0, 30)
    P = oracle.Problem(prob)
    F = oracle.Factor(P)
    sto, dwl = F.correct(st["sigma_d"], st["dsbase"], 1e-2)
    assert F.inertia == (20, 0, 30) and reg["trials"] == F.s.trials
    assert reg["delta_w"] == F.s.dw and reg["delta_c"] == F.s.dc
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 5, 1e-14)
    assert info["eta"] <= 1e-10
    x = np.concatenate([t.cpu().numpy() for t in (rd, rs, ry)])
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    xo = np.concatenate([od, os_, oy])
    assert np.abs(x - xo).max() <= 1e-8 * np.abs(xo).max()
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], reg["delta_w"], reg["delta_c"])
    K[20:320, 20:320] += _blockdiag(prob)
    r = np.concatenate([st["r_d"], st["r_s"], st["r_y"]])
    ref = np.linalg.solve(K, r)
    assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()


IPM_CASES = [  # (n_d, n_s, m, r, sblk, s_scale)
    (64, 2000, 128, 4, 4, 1.0),
    (32, 800, 64, 4, 8, 6.0),
    (0, 400, 50, 3, 3, 1.0),
]


@pytest.mark.parametrize("case", range(len(IPM_CASES)))
def test_sblock_ipm_matches_oracle(case):
    nd, ns, m, r, sb, sc = IPM_CASES[case]
    prob = synth.make_problem(nd, ns, m, r, cfg=450, p=case, s_scale=sc, sblk=sb)
    say(f"coupling blocks ipm {IPM_CASES[case]}")
    r_o = oracle.ipm(oracle.Problem(prob))
    S = mds.solver_for(prob)
    r_g = S.ipm_solve()
    assert r_g["status"] == r_o["status"] == "converged", (r_g["status"], r_o["status"])
    assert r_g["iters"] == r_o["iters"]
    for k in range(r_o["iters"]):
        a, b = r_g["trace"][k], r_o["trace"][k]
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-10), k
        assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], k
        assert a["backtracks"] == b["backtracks"], k
    x, y = r_g["x"].cpu().numpy(), r_g["y"].cpu().numpy()
    assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())
    assert np.abs(y - r_o["y"]).max() <= 1e-8 * max(1.0, np.abs(r_o["y"]).max())


def test_sblock_validation_and_state():
    prob = synth.make_problem(6, 40, 8, 3, cfg=460, sblk=4)
    say("coupling blocks validation")
    S = mds.solver_for(prob)
    bp, Wb = prob["bp"], prob["Wb"]
    with pytest.raises(mds.MdsError, match="cover"):
        S.set_sparse_blocks(bp[:-1], Wb)
    bad = Wb.copy()
    bad[1] += 1.0  # first block (if larger than 1x1) loses its symmetry
    if bp[1] - bp[0] > 1:
        with pytest.raises(mds.MdsError, match="symmetric"):
            S.set_sparse_blocks(bp, bad)
    neg = Wb.copy()
    neg[0] = -5.0
    with pytest.raises(mds.MdsError, match="semidefinite"):
        S.set_sparse_blocks(bp, neg)
    big = np.array([0, prob["n_s"]], dtype=np.int32)
    with pytest.raises(mds.MdsError, match="size"):
        S.set_sparse_blocks(big, np.zeros(prob["n_s"] ** 2))
    S.set_sparse_blocks(bp, Wb)
    with pytest.raises(mds.MdsError, match="coupling"):
        S.ipm_solve_warm(np.zeros(6), np.zeros(8), 1e-3)
    # a problem without blocks: mds_set_problem removed them
    q = {k: v for k, v in prob.items() if k not in ("bp", "Wb")}
    S.set_problem(q)
    st = synth.kkt_state(q, 0, (-1.0, 1.0))
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    Mo, _ = oracle.condense(oracle.Problem(q), st["sigma_d"], st["dsbase"], 0.0, 0.0)
    assert np.array_equal(S.get_matrix().view(np.int64), Mo.view(np.int64))

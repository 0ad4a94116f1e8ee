"""GPU parity of the optional per-row (2,2) diagonal (mds_set_m22_diag).

* condensation with the diagonal is bit-identical to the oracle's (the same
  IEEE sequence: - dc, then - dcv[r]), for several shapes incl. n_d = 0 and
  n_s = 0, and clearing it restores the plain M bit for bit;
* the inertia-correction loop lands on In(M) = (n_d, 0, m) and the refined
  solution satisfies the full KKT system whose (y, y) block carries the
  diagonal: backward error <= 1e-10 and agreement with a dense solve;
* invalid diagonals (negative, NaN) are rejected and leave the handle as it
  was.
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


def _dcv(m, seed):
    rng = np.random.default_rng(900 + seed)
    return 10.0 ** rng.uniform(-4.0, 2.0, m)


SHAPES = [(64, 2000, 128, 4), (10, 40, 27, 3), (0, 50, 40, 3), (33, 0, 20, 0), (150, 3000, 550, 6)]


@pytest.mark.parametrize("idx", range(len(SHAPES)))
def test_m22_diag_condense_bit_exact(idx):
    nd, ns, m, r = SHAPES[idx]
    prob = synth.make_problem(nd, ns, m, r, cfg=400 + idx, p=0)
    st = synth.kkt_state(prob, idx, (-1.0, 1.0))
    dcv = _dcv(m, idx)
    say(f"m22 diag condense shape={SHAPES[idx]}")
    S = mds.solver_for(prob)
    S.set_m22_diag(dcv)
    S.condense(st["sigma_d"], st["dsbase"], 1e-4, 1e-8)
    M = S.get_matrix()
    Mo, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 1e-4, 1e-8, dcv)
    assert np.array_equal(M.view(np.int64), Mo.view(np.int64))
    S.set_m22_diag(None)
    S.condense(st["sigma_d"], st["dsbase"], 1e-4, 1e-8)
    M0 = S.get_matrix()
    Mp, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 1e-4, 1e-8)
    assert np.array_equal(M0.view(np.int64), Mp.view(np.int64))


@pytest.mark.parametrize("seed", [0, 1])
def test_m22_diag_correction_and_refined_solve(seed):
    prob = synth.make_problem(20, 300, 30, 3, cfg=410, p=seed)
    st = synth.kkt_state(prob, seed, (-1.0, 1.0))
    dcv = _dcv(30, seed)
    say(f"m22 diag solve seed={seed}")
    S = mds.solver_for(prob)
    S.set_m22_diag(dcv)
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    status, inn, reg = S.factor_inertia(mu=1e-2, reg=dict(delta_w_last=0.0))
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == (20, 0, 30)
    assert np.array_equal(S.get_pivots(), S.get_factor()[3])
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 5, 1e-14)
    assert info["eta"] <= 1e-10
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], reg["delta_w"], reg["delta_c"], dcv)
    r = np.concatenate([st["r_d"], st["r_s"], st["r_y"]])
    x = np.concatenate([t.cpu().numpy() for t in (rd, rs, ry)])
    ref = np.linalg.solve(K, r)
    assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()


def test_m22_diag_rejects_invalid_entries():
    prob = synth.make_problem(5, 20, 6, 2, cfg=420)
    st = synth.kkt_state(prob, 0, (-1.0, 1.0))
    say("m22 diag invalid")
    S = mds.solver_for(prob)
    good = _dcv(6, 3)
    S.set_m22_diag(good)
    for bad in (np.array([1.0, -1e-3, 1.0, 1.0, 1.0, 1.0]), np.array([1.0, np.nan, 1, 1, 1, 1.0])):
        with pytest.raises(mds.MdsError, match="nonnegative"):
            S.set_m22_diag(bad)
    # the valid diagonal set before is still in effect
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    Mo, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 0.0, 0.0, good)
    assert np.array_equal(S.get_matrix().view(np.int64), Mo.view(np.int64))

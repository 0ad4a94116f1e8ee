"""Pins for the oracle's per-row (2,2) diagonal (the way inequality rows'
inverse barrier diagonal -D_h^{-1} enters the compressed form of Sec. 2.2):

* with no x_d and no x_s block, M = -dc I - diag(dcv) (closed form);
* a zero dcv changes nothing (bitwise);
* M with dcv is the Schur complement of the explicit KKT matrix whose (y, y)
  block is -dc I - diag(dcv), computed by a dense solve;
* the inertia of that KKT matrix is In(D_s) + In(M) (Haynsworth), with
  In(M) = (n_d, 0, m) for a convex Q and positive dcv.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import full_kkt, sign_counts


def _dcv(m, seed):
    rng = np.random.default_rng(700 + seed)
    return 10.0 ** rng.uniform(-4.0, 2.0, m)


def test_m22_diag_closed_form_without_x_blocks():
    prob = synth.make_problem(0, 0, 6, 0, cfg=111)
    P = oracle.Problem(prob)
    dcv = _dcv(6, 0)
    M, _ = oracle.condense(P, np.zeros(0), np.zeros(0), 0.0, 1e-7, dcv)
    assert np.array_equal(M, np.diag(-1e-7 - dcv))


def test_zero_m22_diag_changes_nothing():
    prob = synth.make_problem(5, 30, 7, 3, cfg=112)
    st = synth.kkt_state(prob, 1, (-1.0, 1.0))
    P = oracle.Problem(prob)
    M0, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], 1e-3, 1e-6)
    M1, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], 1e-3, 1e-6, np.zeros(7))
    assert np.array_equal(M0.view(np.int64), M1.view(np.int64))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_m22_diag_is_schur_complement(seed):
    prob = synth.make_problem(6, 40, 9, 4, cfg=113, p=seed)
    st = synth.kkt_state(prob, seed, (-1.0, 1.0))
    P = oracle.Problem(prob)
    dcv = _dcv(9, seed)
    M, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], 1e-4, 1e-8, dcv)
    K = full_kkt(prob, st["sigma_d"], st["dsbase"], 1e-4, 1e-8, dcv)
    nd, ns = prob["n_d"], prob["n_s"]
    n = nd + ns
    keep = np.r_[0:nd, n:K.shape[0]]
    elim = np.arange(nd, n)
    S = K[np.ix_(keep, keep)] - K[np.ix_(keep, elim)] @ np.linalg.solve(
        K[np.ix_(elim, elim)], K[np.ix_(elim, keep)])
    assert np.allclose(M, S, rtol=1e-12, atol=1e-12 * np.abs(S).max())
    # Haynsworth: In(K) = In(D_s) + In(M); D_s > 0
    kin = sign_counts(np.linalg.eigvalsh(K))
    min_ = sign_counts(np.linalg.eigvalsh(M))
    assert kin == (min_[0] + ns, min_[1], min_[2])
    assert min_ == (nd, 0, prob["m"])

"""The large condensed system (n_d = 4096, n_s = 1000000, m = 12288, N = 16384,
8 nonzeros per row of J_s, D_s and Sigma_d log-uniform over 1e-8..1e8) in the
default launch configuration (cooperative register panel, 16 workgroups).

The oracle's unblocked factorization of N = 16384 takes minutes, so its
results are stored (tests/golden/kkt_n16384.json, written by
tests/golden/make_golden_pivots.py from oracle/ only):

* M is compared bit for bit with the oracle's condensation (all N^2 entries);
* the pivot sequence and the inertia equal the oracle's, for the cooperative
  panel and for the memory panel;
* P M P' = L D L' on 300 sampled entries within N eps of (|L| |D| |L'|)_ij;
* the normwise backward error of the solve on the full KKT system, and the
  solution at 3000 stored positions against the oracle's refined solution;
* the precision sweep: FP32 and split-BF16 trailing updates refined by FP64
  GMRES reach backward error <= 1e-13 with the oracle's inertia; their
  solutions are reported against the oracle's (at this conditioning a
  backward error of 1e-14 allows forward differences ~1e-5, which the test
  bounds by 1e-3); plain BF16 is reported only (its factor is not a usable
  preconditioner here and its inertia differs).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_13736_amd as mds
import synth
from helpers import perm_from_ipiv

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _golden():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "kkt_n16384.json")))
    N = g["ipiv"]["N"]
    ipiv = np.arange(1, N + 1, dtype=np.int32)
    ipiv[np.asarray(g["ipiv"]["index"], dtype=np.int64)] = g["ipiv"]["value"]
    g["ipiv_full"] = ipiv
    g["x_index"] = np.asarray(g["x_index"], dtype=np.int64)
    g["x_value"] = np.asarray(g["x_value"])
    return g


@pytest.fixture(scope="module")
def c2():
    prob = synth.config_problem(synth.LARGE_N16384)
    st = synth.kkt_state(prob, 2)
    return dict(prob=prob, st=st, P=oracle.Problem(prob), gold=_golden())


def _release(S):
    del S
    torch.cuda.empty_cache()


def _two_blocks(ipiv):
    N = len(ipiv)
    two = np.zeros(N, bool)
    k = 0
    while k < N:
        if ipiv[k] < 0:
            two[k] = True
            k += 2
        else:
            k += 1
    return np.nonzero(two)[0]


def _dmul(v, dd, ds, idx, absval=False):
    d = np.abs(dd) if absval else dd
    c = np.abs(ds[idx]) if absval else ds[idx]
    o = d * v
    o[idx] += c * v[idx + 1]
    o[idx + 1] += c * v[idx]
    return o


def test_c2_condense_factor_solve_fp64(c2):
    prob, st, P = c2["prob"], c2["st"], c2["P"]
    say("N=16384 condense / cooperative factor / solve, FP64")
    S = mds.solver_for(prob)
    assert S.info()["panel"] == "coop"
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    M = S.get_matrix()
    Mo, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], 0.0, 0.0)
    assert np.array_equal(M.view(np.int64), Mo.view(np.int64))
    del M
    status, inn, _ = S.factor_inertia()
    assert status == mds.MDS_OK
    L, dd, ds, ipiv = S.get_factor()
    N = len(ipiv)
    gold = c2["gold"]
    assert np.array_equal(ipiv, gold["ipiv_full"]), int(np.argmax(ipiv != gold["ipiv_full"]))
    assert [inn["npos"], inn["nzero"], inn["nneg"]] == gold["inertia"]
    p = perm_from_ipiv(ipiv)
    idx = _two_blocks(ipiv)
    rng = np.random.default_rng(16384)
    cols = np.arange(N)
    worst = 0.0
    for _ in range(300):
        a, b = sorted(rng.integers(0, N, 2))[::-1]
        la = np.where(cols == a, 1.0, L[a] * (cols < a))
        lb = np.where(cols == b, 1.0, L[b] * (cols < b))
        rec = la @ _dmul(lb, dd, ds, idx)
        bound = np.abs(la) @ _dmul(np.abs(lb), dd, ds, idx, True)
        worst = max(worst, abs(Mo[p[a], p[b]] - rec) / max(bound, 1e-300))
    say(f"  sampled reconstruction: worst |A - LDL'| / (|L||D||L'|) = {worst:.2e}")
    assert worst <= N * np.finfo(float).eps
    del L, Mo
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 3, 1e-14)
    say(f"  backward error {info['eta']:.2e} after {info['steps']} refinement steps")
    assert info["eta"] <= 1e-14
    x64 = np.concatenate([t.cpu().numpy() for t in (rd, rs, ry)])
    fwd = np.abs(x64[gold["x_index"]] - gold["x_value"]).max() / gold["x_absmax"]
    say(f"  sampled difference to the oracle's solution {fwd:.2e} (oracle eta {gold['eta']:.1e})")
    assert fwd <= 1e-6
    c2["x64"], c2["inn64"], c2["ipiv64"] = x64, inn, ipiv
    _release(S)


def test_c2_memory_panel_same_pivots(c2):
    prob, st = c2["prob"], c2["st"]
    if "ipiv64" not in c2:
        pytest.skip("needs the FP64 cooperative factorization of the previous test")
    say("N=16384 memory panel pivots vs cooperative panel")
    S = mds.solver_for(prob, panel="mem")
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    _, inn, _ = S.factor_inertia()
    ipiv = S.get_factor()[3]
    assert np.array_equal(ipiv, c2["gold"]["ipiv_full"])
    assert np.array_equal(ipiv, c2["ipiv64"])
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == (
        c2["inn64"]["npos"], c2["inn64"]["nzero"], c2["inn64"]["nneg"])
    _release(S)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
def test_c2_precision_sweep(c2, prec):
    prob, st = c2["prob"], c2["st"]
    if "x64" not in c2:
        pytest.skip("needs the FP64 solution of the first test")
    say(f"N=16384 precision sweep {prec}")
    S = mds.solver_for(prob, precision=prec)
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    _, inn, _ = S.factor_inertia()
    (rd, rs, ry), info = S.refine(st["r_d"], st["r_s"], st["r_y"], 60, 1e-14)
    x = np.concatenate([t.cpu().numpy() for t in (rd, rs, ry)])
    x64 = c2["x64"]
    diff = np.abs(x - x64).max() / np.abs(x64).max()
    gold = c2["gold"]
    dor = np.abs(x[gold["x_index"]] - gold["x_value"]).max() / gold["x_absmax"]
    say(f"  inertia {inn['npos']}/{inn['nzero']}/{inn['nneg']}, GMRES iterations {info['steps']}, "
        f"backward error {info['eta']:.2e}, max relative difference to FP64 {diff:.2e}, "
        f"to the oracle (sampled) {dor:.2e}")
    if prec != "bf16":
        assert info["eta"] <= 1e-13
        assert [inn["npos"], inn["nzero"], inn["nneg"]] == gold["inertia"]
        assert diff <= 1e-3 and dor <= 1e-3
    _release(S)

"""Diagnostics of the cooperative panel through the C-ABI: pivot statistics
of a factorization (mds_get_panel_stats) checked against the oracle's pivot
sequence (Sec. 2.3), and the exchange round-trip probe (mds_probe_exchange),
after which a cooperative factorization must still reproduce the oracle's
pivots (the probe shares the panel's exchange buffer)."""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _dense_problem(A):
    N = A.shape[0]
    return dict(n_d=N, n_s=0, m=0, r=0, H=np.asfortranarray(A), c=np.zeros(N), w=np.zeros(0),
                g=np.zeros(0), Jd=np.zeros((0, N)), rp=np.zeros(1, dtype=np.int32),
                ci=np.zeros(0, dtype=np.int32), v=np.zeros(0), b=np.zeros(0),
                xl=-np.ones(N), xu=np.ones(N))


def _matrix(N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    # a weak diagonal makes the first Bunch-Kaufman test fail often
    return 0.5 * (A + A.T) * np.where(np.eye(N) > 0, 0.01, 1.0)


def _coop_factor(A):
    S = mds.solver_for(_dense_problem(A), panel="coop")
    S.condense(np.zeros(A.shape[0]), np.zeros(0), 0.0, 0.0)
    S.factor_inertia()
    return S


def test_panel_stats_agree_with_oracle_pivots():
    N = 1500
    A = _matrix(N, 11)
    say(f"panel stats N={N}")
    S = _coop_factor(A)
    st = S.panel_stats()
    ipiv = S.get_pivots()
    _, _, _, ipo, _, _ = oracle.bk(A)
    assert np.array_equal(ipiv, ipo)
    k, n2, swaps = 0, 0, 0
    while k < N:
        if ipo[k] < 0:
            n2 += 1
            k += 2
        else:
            swaps += int(ipo[k] != k + 1)
            k += 1
    assert st["n2x2"] == n2
    # every pivot step of this factorization ran in the cooperative panel
    assert st["coop_steps"] == N - n2
    # a 2x2 pivot or an interchange needs the second test (the candidate
    # column); a 1x1 pivot may need it too without an interchange
    assert swaps + n2 <= st["coop_second"] <= st["coop_steps"]
    # a panel factors 31 or 32 columns (32 when it ends on a 2x2 pivot),
    # except the last
    assert (N + 31) // 32 <= st["panels"] <= (N + 30) // 31


def test_exchange_probe_and_factorization_after_it():
    N = 3000   # three workgroups in the cooperative panel
    A = _matrix(N, 12)
    S = _coop_factor(A)
    for P, words in ((1, 3), (4, 3), (4, 69 * 2), (16, 3), (16, 128)):
        say(f"exchange probe P={P} words={words}")
        us = S.probe_exchange(P, rounds=2000, words=words)
        say(f"  {us:.3f} us per round")
        assert np.isfinite(us) and 0.0 < us < 100.0, (P, words, us)
    for P, words, rounds in ((0, 3, 10), (33, 3, 10), (4, 0, 10), (4, 513, 10), (16, 200, 10),
                             (4, 3, 0)):
        with pytest.raises(mds.MdsError):
            S.probe_exchange(P, rounds=rounds, words=words)
    # the probe's words never pass for a panel's: the factorization that
    # follows still takes the oracle's pivots
    say("cooperative factorization after the probe")
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    S.factor_inertia()
    _, _, _, ipo, _, _ = oracle.bk(A)
    assert np.array_equal(S.get_pivots(), ipo)

"""The factorization's launch sequence is captured into a hipGraph once per
handle and replayed whenever per-launch timing is off.  Every replay must
give the factor that plain launches give: the same matrix is factored
several times on one handle, with eager work (condensation, solves, host
synchronization) between the replays, and each factor is compared bit for
bit with one from plain launches (timing on) and with the oracle's pivots."""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _bits(a):
    return np.asarray(a, np.float64).view(np.int64)


@pytest.mark.parametrize("panel,precision", [("coop", "fp64"), ("reg", "fp64"), ("mem", "fp64"),
                                             ("coop", "fp32")])
def test_graph_replays_equal_plain_launches(panel, precision):
    prob = synth.make_problem(150, 3000, 550, 6, cfg=303, p=1)
    st = synth.kkt_state(prob, 1, (-3.0, 3.0))
    say(f"factor graph replays panel={panel} precision={precision}")
    S = mds.solver_for(prob, nb=32 if panel != "mem" else 16, panel=panel, precision=precision)
    # plain launches (timing on: no capture)
    S.set_timing(True)
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    S.factor_inertia()
    ref = S.get_factor()
    S.set_timing(False)
    Mo, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 0.0, 0.0)
    ipo = oracle.bk(Mo)[3] if precision == "fp64" else None
    for rep in range(4):
        S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
        S.factor_inertia()
        L, dd, ds, ipiv = S.get_factor()
        assert np.array_equal(ipiv, ref[3]), rep
        assert np.array_equal(_bits(L), _bits(ref[0])), rep
        assert np.array_equal(_bits(dd), _bits(ref[1])) and np.array_equal(_bits(ds), _bits(ref[2]))
        if ipo is not None:
            assert np.array_equal(ipiv, ipo)
        S.solve(st["r_d"], st["r_s"], st["r_y"])  # eager work between replays

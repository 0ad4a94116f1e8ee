"""The whole-matrix LDS factorization (panel "lds": unblocked Bunch-Kaufman
with M held in one workgroup's LDS, N <= 199) against the oracle.

Both sides run the same unblocked algorithm on the same bits of M with every
product, sum and division rounded once as written, so the bar is bitwise:
L, D (diagonal and sub-diagonal), ipiv, inertia and info identical.  The
cases cover the workload shape (N = 192), the largest order (199), the
smallest (1, 2), every pivot branch, zero pivots, and both workgroup sizes.
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _dense_problem(A):
    N = A.shape[0]
    return dict(n_d=N, n_s=0, m=0, r=0, H=np.asfortranarray(A), c=np.zeros(N), w=np.zeros(0),
                g=np.zeros(0), Jd=np.zeros((0, N)), rp=np.zeros(1, dtype=np.int32),
                ci=np.zeros(0, dtype=np.int32), v=np.zeros(0), b=np.zeros(0),
                xl=-np.ones(N), xu=np.ones(N))


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float64).view(np.int64),
                          np.asarray(b, np.float64).view(np.int64))


def _check_exact(S, Mo):
    st, inn, _ = S.factor_inertia()
    L, dd, ds, ipiv = S.get_factor()
    Lo, ddo, dso, ipo, info_o, _ = oracle.bk(Mo)
    assert np.array_equal(ipiv, ipo), f"first differing pivot {np.argmax(ipiv != ipo)}"
    assert _same_bits(dd, ddo) and _same_bits(ds, dso)
    assert _same_bits(L, Lo)
    assert (inn["npos"], inn["nzero"], inn["nneg"]) == oracle.inertia(ipo, ddo, dso)
    assert inn["info"] == info_o
    assert st == (mds.MDS_ZERO_PIVOT if info_o else mds.MDS_OK)
    return ipiv


@pytest.mark.parametrize("threads", [256, 512])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lds_workload_shape_bitwise(seed, threads):
    """N = 192 condensed KKT matrices (n_d = 64, n_s = 2000, m = 128)."""
    prob = synth.make_problem(64, 2000, 128, 4, cfg=300, p=seed)
    st = synth.kkt_state(prob, seed, (-3.0, 3.0))
    say(f"lds N=192 seed={seed} threads={threads}")
    S = mds.solver_for(prob, panel="lds", panel_threads=threads)
    assert S.info()["panel"] == "lds"
    S.condense(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    Mo, _ = oracle.condense(oracle.Problem(prob), st["sigma_d"], st["dsbase"], 0.0, 0.0)
    _check_exact(S, Mo)


@pytest.mark.parametrize("N", [1, 2, 3, 63, 64, 65, 128, 198, 199])
def test_lds_random_symmetric_bitwise(N):
    rng = np.random.default_rng(1000 + N)
    A = rng.standard_normal((N, N))
    A = A + A.T
    A[np.diag_indices(N)] *= 0.01  # small diagonals: many interchanges and 2x2 pivots
    say(f"lds random symmetric N={N}")
    S = mds.solver_for(_dense_problem(A), panel="lds")
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    _check_exact(S, A)


BRANCHES = [
    np.array([[4.0, 1.0], [1.0, 3.0]]),                                    # 1x1, first test
    np.array([[1.0, 2.0, 0.0], [2.0, 0.0, 10.0], [0.0, 10.0, 0.0]]),       # second test
    np.array([[0.1, 2.0, 0.0], [2.0, 5.0, 1.0], [0.0, 1.0, 1.0]]),         # 1x1 interchange
    np.array([[0.0, 1.0], [1.0, 0.0]]),                                    # 2x2, no interchange
    np.array([[0.0, 0.5, 2.0], [0.5, 1.0, 0.3], [2.0, 0.3, 0.0]]),         # 2x2 with interchange
    np.diag([3.0, 0.0, -2.0, 5.0]),                                        # zero pivot
    np.zeros((3, 3)),                                                      # all zero
]


@pytest.mark.parametrize("case", range(len(BRANCHES)))
def test_lds_branch_matrices_bitwise(case):
    A = BRANCHES[case]
    say(f"lds branch case={case}")
    S = mds.solver_for(_dense_problem(A), panel="lds")
    S.condense(np.zeros(A.shape[0]), np.zeros(0), 0.0, 0.0)
    _check_exact(S, A)


def test_lds_rank_deficient_zero_columns():
    """Exact zero columns in the middle: zero pivots recorded without elimination."""
    rng = np.random.default_rng(77)
    N = 150
    B = rng.standard_normal((N, 40))
    A = B @ B.T - 3.0 * np.eye(N)
    A[:, 60] = 0.0
    A[60, :] = 0.0
    say("lds zero column N=150")
    S = mds.solver_for(_dense_problem(A), panel="lds")
    S.condense(np.zeros(N), np.zeros(0), 0.0, 0.0)
    _check_exact(S, A)


def test_lds_solve_matches_oracle():
    prob = synth.make_problem(64, 2000, 128, 4, cfg=300, p=5)
    st = synth.kkt_state(prob, 5, (-1.0, 1.0))
    say("lds solve N=192")
    S = mds.solver_for(prob, panel="lds")
    S.condense(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    S.factor_inertia()
    got = np.concatenate([t.cpu().numpy() for t in S.solve(st["r_d"], st["r_s"], st["r_y"])])
    F = oracle.Factor(oracle.Problem(prob)).once(st["sigma_d"], st["dsbase"], 1e-6, 1e-9)
    od, os_, oy, _ = F.solve(st["r_d"], st["r_s"], st["r_y"])
    ref = np.concatenate([od, os_, oy])
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("variant", ["workload", "nonconvex"])
def test_lds_ipm_matches_oracle(variant):
    """Whole IPM on the N = 192 workload (and a nonconvex variant whose
    correction loop fires): status, iterations, per-iteration inertia,
    trials and backtracks identical to the oracle's."""
    prob = (synth.config_problem(synth.IPM_N192) if variant == "workload"
            else synth.make_problem(64, 2000, 128, 4, cfg=0, p=1, s_scale=6.0))
    say(f"lds IPM N=192 {variant}")
    r_o = oracle.ipm(oracle.Problem(prob))
    S = mds.solver_for(prob, panel="lds")
    r_g = S.ipm_solve()
    assert r_g["status"] == r_o["status"] == "converged"
    assert r_g["iters"] == r_o["iters"]
    for k in range(r_o["iters"]):
        a, b = r_g["trace"][k], r_o["trace"][k]
        assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], k
        assert a["backtracks"] == b["backtracks"], k
    x, y = r_g["x"].cpu().numpy(), r_g["y"].cpu().numpy()
    assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())
    assert np.abs(y - r_o["y"]).max() <= 1e-8 * max(1.0, np.abs(r_o["y"]).max())
    if variant == "nonconvex":
        assert max(t["trials"] for t in r_g["trace"]) > 1


def test_lds_order_limit():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((200, 200))
    with pytest.raises(mds.MdsError):
        mds.solver_for(_dense_problem(A + A.T), panel="lds")
    with pytest.raises(mds.MdsError):
        mds.solver_for(_dense_problem(np.eye(8)), panel="lds", precision="fp32")

"""Writes the oracle's pivot sequences, inertia and (for the large condensed
system) sampled solution entries at sizes the GPU tests cannot factor with
the oracle in their time budget:

* pivots_dense_n9000.json: Bunch-Kaufman of the N = 9000 random symmetric
  matrix of the nine-workgroup cooperative-panel test (A = G + G',
  G ~ N(0,1) from numpy default_rng(9000));
* kkt_n16384.json: the large condensed system (n_d = 4096, n_s = 1000000,
  m = 12288, 8 nonzeros per row of J_s, Sigma_d and D_s log-uniform over
  1e-8..1e8, synth.kkt_state seed 2): pivots and inertia of M at zero shifts,
  and the oracle's refined solution of the full system at 3000 seeded
  sample positions.

Only oracle/ and synth/ are called; the elimination runs on several threads,
which gives the same bits as one thread (each entry keeps its expression).
Pivots are stored sparsely: the 1-based ipiv entries that differ from k+1.
Run from the repository root:  python tests/golden/make_golden_pivots.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def sparse_ipiv(ipiv):
    k = np.arange(len(ipiv)) + 1
    idx = np.nonzero(ipiv != k)[0]
    return dict(N=int(len(ipiv)), index=idx.tolist(), value=ipiv[idx].astype(int).tolist())


def dense_problem(A):
    N = A.shape[0]
    return dict(n_d=N, n_s=0, m=0, r=0, H=np.asfortranarray(A), c=np.zeros(N), w=np.zeros(0),
                g=np.zeros(0), Jd=np.zeros((0, N), order="F"), rp=np.zeros(1, np.int32),
                ci=np.zeros(0, np.int32), v=np.zeros(0), b=np.zeros(0), xl=-np.ones(N),
                xu=np.ones(N))


def dense_9000(threads):
    N = 9000
    rng = np.random.default_rng(N)
    A = rng.standard_normal((N, N))
    A = A + A.T
    P = oracle.Problem(dense_problem(A))
    t = time.time()
    F = oracle.Factor(P).once(np.zeros(N), np.zeros(0), 0.0, 0.0)
    out = dict(workload="random symmetric N = 9000, A = G + G', G ~ N(0,1), default_rng(9000)",
               ipiv=sparse_ipiv(F.ipiv), inertia=list(F.inertia), info=int(F.s.info),
               oracle_seconds=time.time() - t, threads=threads)
    json.dump(out, open(os.path.join(HERE, "pivots_dense_n9000.json"), "w"))
    print("n9000 done", out["inertia"], f"{out['oracle_seconds']:.0f}s", flush=True)


def kkt_16384(threads):
    prob = synth.config_problem(synth.LARGE_N16384)
    st = synth.kkt_state(prob, 2)
    P = oracle.Problem(prob)
    t = time.time()
    F = oracle.Factor(P).once(st["sigma_d"], st["dsbase"], 0.0, 0.0)
    tf = time.time() - t
    print(f"n16384 factor {tf:.0f}s", F.inertia, flush=True)
    xd, xs, y, steps, eta = F.refine(st["r_d"], st["r_s"], st["r_y"], 3, 1e-14)
    x = np.concatenate([xd, xs, y])
    rng = np.random.default_rng(16384)
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    pos = np.unique(np.concatenate([rng.integers(0, nd, 1000),
                                    nd + rng.integers(0, ns, 1000),
                                    nd + ns + rng.integers(0, m, 1000)]))
    out = dict(workload="n_d=4096 n_s=1000000 m=12288 (N=16384), J_s 8 nnz/row, "
                        "synth.kkt_state(prob, 2): Sigma_d, D_s log-uniform 1e-8..1e8",
               ipiv=sparse_ipiv(F.ipiv), inertia=list(F.inertia), info=int(F.s.info),
               n2x2=int(np.sum(F.ipiv < 0) // 2), refine_steps=int(steps), eta=float(eta),
               x_index=pos.tolist(), x_value=[float(v) for v in x[pos]],
               x_absmax=float(np.abs(x).max()), oracle_factor_seconds=tf, threads=threads)
    json.dump(out, open(os.path.join(HERE, "kkt_n16384.json"), "w"))
    print("n16384 done", f"eta {eta:.2e}", flush=True)


if __name__ == "__main__":
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    oracle.build(force=False)
    oracle.set_threads(threads)
    which = sys.argv[1:] or ["n9000", "n16384"]
    if "n9000" in which:
        dense_9000(threads)
    if "n16384" in which:
        kkt_16384(threads)

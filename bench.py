"""Benchmark of the condensed-KKT Newton step on one MI355X.

A step is one iteration of the filter line-search IPM on the OPF-scale
workload (n_d = 1024 dense and n_s = 200000 sparse variables, m = 3072
equality constraints, condensed size N = 4096, 6 nonzeros per row of J_s,
seeded synthetic data): optimality test and barrier update, Newton system
(condense + Bunch-Kaufman factorization with the inertia-correction loop),
solve with FP64 refinement, fraction to the boundary, filter line search and
update.  Problem data is resident in HBM before the timed region.

Printed value: KKT factor+solve throughput in TFLOP/s, counting the nominal
N^3/3 flops of every factorization performed (correction trials included) and
2 N^2 per solve, divided by the wall time of the timed steps.

Also reported: a per-kernel roofline for the dominant kernel (HIP events on
the library stream over the timed region), whole-IPM solves/s on the N = 192
workload, and the CPU oracle timed on one N = 4096 condense + factor + solve
(the CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KKT factor+solve TFLOP/s & IPM solves/s: mixed/learned vs FP64, 1e-8 res"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def panel_bytes_per_launch(N, launches_per_factor):
    """Algorithmic HBM bytes of one panel launch, averaged over a factorization:
    a panel of width w starting at k0 reads its w columns (rows >= k0) once,
    reads one pivot-candidate column per pivot, and writes L and W once:
    4 * (N - k0) * w * 8 bytes.  Summed over the factorization this is
    4 * 8 * N (N + 1) / 2 whatever the widths; divided by the launches."""
    return 4.0 * 8.0 * N * (N + 1) / 2.0 / max(launches_per_factor, 1)


def trailing_bytes_per_launch(N, w):
    """Algorithmic bytes of one trailing update (panels of width w): read and
    write the lower trailing triangle, write its mirror, read the L and W
    panels."""
    total, cnt, k0 = 0.0, 0, 0
    while k0 + w < N:
        n = N - (k0 + w)
        total += (n * (n + 1) / 2) * 8.0 * 3 + 2.0 * n * w * 8.0
        cnt += 1
        k0 += w
    return total / max(cnt, 1)


def cpu_baseline(prob, N):
    import numpy as np
    import oracle
    import synth
    P = oracle.Problem(prob)
    it = synth.interior_iterate(prob, 0)
    nd = prob["n_d"]
    sig, rx, ry = oracle.sigma_rhs(P, it["x"], it["y"], it["zl"], it["zu"], it["mu"])
    dsb = prob["w"] + sig[nd:]
    F = oracle.Factor(P)
    t = time.perf_counter()
    F.once(sig[:nd], dsb, 0.0, 0.0)
    F.solve(rx[:nd], rx[nd:], ry)
    dt = time.perf_counter() - t
    flops = N ** 3 / 3.0 + 2.0 * N ** 2
    return dict(value=flops / dt / 1e12, unit="TFLOP/s", cores=1, kind="oracle",
                sample=f"one condense + unblocked Bunch-Kaufman factor + solve of the N={N} "
                       f"system at a seeded interior point, {dt:.1f} s on 1 host core",
                seconds=dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ipm-solves", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates HBM counters)")
    args = ap.parse_args()
    if args.calib_copy:
        import torch
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": x.numel() * 8,
                          "calib_copy_bytes_written": x.numel() * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_13736_amd as mds
    import synth

    cfg = synth.CONFIGS[1]
    prob = synth.config_problem(1)
    N = cfg["n_d"] + cfg["m"]
    log(f"workload N={N} n_s={cfg['n_s']} nnz={len(prob['v'])}")
    S = mds.solver_for(prob, nb=args.nb)
    info0 = S.info()
    nb = info0["nb"]
    it = S.new_iterate()
    S.ipm_init(it)

    def step():
        st, info = S.ipm_step(it)
        if st != 0:  # converged (or failed): restart from the cold start point
            S.ipm_init(it)
            st, info = S.ipm_step(it)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    S.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    facs = solves = 0
    for _ in range(args.steps):
        info = step()
        facs += info["trials"]
        solves += info["solves"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = S.get_timings()
    S.set_timing(False)
    flops = facs * N ** 3 / 3.0 + solves * 2.0 * N ** 2
    value = flops / dt / 1e12
    log(f"timed {args.steps} steps in {dt:.3f}s: {facs} factorizations, {solves} solves")
    log("per-class device time:", json.dumps(tim))

    # dominant kernel roofline
    dom = max(tim, key=lambda k: tim[k]["ms"])
    nlaunch = max(tim[dom]["launches"], 1)
    avg_s = tim[dom]["ms"] / 1e3 / nlaunch
    if dom == "panel":
        per_launch = panel_bytes_per_launch(N, tim["panel"]["launches"] / max(facs, 1))
        roof = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK_GBS,
                    unit="GB/s")
    elif dom == "trailing":
        per_launch = trailing_bytes_per_launch(N, N / max(tim["panel"]["launches"] / max(facs, 1), 1))
        roof = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK_GBS,
                    unit="GB/s")
    elif dom == "solve":
        per_launch = 2.0 * (N * N / 2.0) * 8.0
        roof = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK_GBS,
                    unit="GB/s")
    else:
        m, nd = cfg["m"], cfg["n_d"]
        per_launch = 8.0 * (N * N + m * nd + nd * nd)
        roof = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK_GBS,
                    unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = {"panel": "k_bk_panel_reg" if info0["panel"] == "reg" else "k_bk_panel",
                      "trailing": "k_bk_trailing",
                      "solve": "k_ldl_solve", "condense": "k_condense_dense"}[dom]
    roof["avg_launch_us"] = avg_s * 1e6
    roof["bytes_per_launch"] = per_launch
    fac_ms = (tim["panel"]["ms"] + tim["trailing"]["ms"]) / max(facs, 1)
    factor_tfs = (N ** 3 / 3.0) / (fac_ms / 1e3) / 1e12

    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 IPM Newton steps, n_d=1024 n_s=200000 m=3072 (N={N}), "
                               "J_s 6 nnz/row, seeded synthetic", "N": N, "nb": nb,
                   "panel": info0["panel"], "precision": "fp64"},
        "roofline": roof,
        "factor": {"ms_per_factorization": fac_ms, "tflops": factor_tfs,
                   "frac_fp64_mfma_peak": factor_tfs / FP64_MFMA_PEAK_TFS,
                   "factorizations": facs, "solves": solves},
        "kernel_ms": {k: v["ms"] for k, v in tim.items()},
    }

    if not args.no_ipm_solves:
        prob0 = synth.config_problem(0)
        S0 = mds.solver_for(prob0)
        r = S0.ipm_solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nrep = 5
        for _ in range(nrep):
            r = S0.ipm_solve()
        torch.cuda.synchronize()
        d0 = (time.perf_counter() - t1) / nrep
        out["ipm_solves"] = {"workload": "whole FP64 IPM to E_0 <= 1e-8, n_d=64 n_s=2000 m=128 "
                                         "(N=192)", "solves_per_s": 1.0 / d0,
                             "iters": r["iters"], "status": r["status"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

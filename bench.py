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
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by
# the counters of a 256 MiB copy (the profile file gives the commands and the
# factors); valid for the kernel source as profiled.
MEASURED_TRAFFIC = {
    "k_bk_panel_coop": (2742650.0, "profiles/bk_panel_coop_ipm_newton_step_n4096.md"),
    "k_bk_trailing": (75934233.0, "profiles/bk_trailing_ipm_newton_step_n4096.md"),
}
FP64_MFMA_PEAK_TFS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def panel_bytes_per_launch(N, launches_per_factor, adv=None):
    """Algorithmic HBM bytes of one panel launch, averaged over its launches:
    a panel of width w starting at k0 reads its w columns (rows >= k0) once,
    reads one pivot-candidate column per pivot, and writes L and W once:
    4 * (N - k0) * w * 8 bytes, i.e. 4 * 8 * (N - c) per column c.  Over a
    whole factorization this is 4 * 8 * N (N + 1) / 2 whatever the widths.
    When the launches cover only the first columns (a cooperative panel that
    hands the last rows to another kernel), they cover launches * adv columns
    (adv = nb - 1 per panel, nominal: a panel ending on a 2x2 pivot takes one
    more)."""
    n = max(launches_per_factor, 1)
    K = N if adv is None else min(N, n * adv)
    return 4.0 * 8.0 * (K * N - K * (K - 1) / 2.0) / n


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


def mixed_section(prob, N, reps=3):
    """One Newton system of the workload at a seeded interior point, solved
    to backward error 1e-14 by (a) FP64 factor + classic refinement and (b)
    FP32 / BF16 trailing updates + FP64 GMRES refinement.  Reports the time
    of condense + factor + refined solve, nominal TFLOP/s, refinement
    iterations, and the max-norm error of each solution relative to FP64's."""
    import torch
    import paper_2605_13736_amd as mds
    import synth
    it = synth.interior_iterate(prob, 0)
    nd = prob["n_d"]
    out, ref = {}, None
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        S = mds.solver_for(prob, precision=prec)
        sig, rx, ry = S.sigma_rhs(it["x"], it["y"], it["zl"], it["zu"], it["mu"])
        dsb = S.dev(prob["w"]) + sig[nd:]
        sd = sig[:nd].contiguous()
        steps = 2 if prec == "fp64" else 60

        def once():
            S.condense(sd, dsb, 0.0, 0.0)
            S.factor_inertia()
            return S.refine(rx[:nd], rx[nd:], ry, steps, 1e-14)

        once()
        torch.cuda.synchronize()
        S.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            (a, b, c), info = once()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        tim = S.get_timings()
        S.set_timing(False)
        x = torch.cat([a, b, c]).cpu().numpy()
        if ref is None:
            ref = x
        fac_ms = (tim["panel"]["ms"] + tim["panel_tail"]["ms"] + tim["trailing"]["ms"]) / reps
        out[prec] = dict(ms_condense_factor_refine=dt * 1e3, ms_factor=fac_ms,
                         tflops_nominal=(N ** 3 / 3.0 + 2.0 * N ** 2) / dt / 1e12,
                         refine_iterations=info["steps"], eta=info["eta"],
                         rel_err_vs_fp64=float(abs(x - ref).max() / max(abs(ref).max(), 1e-300)))
        del S
        torch.cuda.empty_cache()
    return out


def batch_section(count, mu=0.05, singles=6):
    """The scenario batch: count problems with N = 4 U{64..512}, n_d = N/4,
    m = 3N/4, n_s = 50N, 4 nonzeros per row of J_s, each at a seeded barrier
    state; solved by the persistent kernel after autotuning, in FP64 and in
    the scope's form (FP32 storage and FP32-MFMA trailing tiles, FP64
    refinement on the full system).  Also times a loop of single-problem FP64
    solves on the first `singles` problems."""
    import numpy as np
    import torch
    import paper_2605_13736_amd as mds
    import synth
    items, flops = [], 0.0
    for p in range(count):
        sz = synth.batch_sizes(p)
        prob = synth.make_problem(sz["n_d"], sz["n_s"], sz["m"], sz["r"], cfg=3, p=p)
        st = synth.kkt_state(prob, p, (-1.0, 1.0))
        it = dict(prob)
        it.update(sigma_d=st["sigma_d"], dsbase=st["dsbase"], r_d=st["r_d"], r_s=st["r_s"],
                  r_y=st["r_y"])
        items.append(it)
        N = sz["N"]
        flops += N ** 3 / 3.0 + 2.0 * N ** 2
    def timed(precision):
        B = mds.Batch(items, precision=precision)
        B.run(mu)
        cfg = B.autotune(mu)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            res = B.run(mu)
        dt = (time.perf_counter() - t0) / reps
        lat = np.array([r["t_done"] for r in res], dtype=np.float64) / 1e5  # 100 MHz ticks
        sols = [np.concatenate(B.solution(p)) for p in range(count)]
        B.close()
        del B
        torch.cuda.empty_cache()
        return dt, res, lat, cfg, sols

    dt, res, lat_ms, cfg, x64 = timed("fp64")
    dt32, res32, lat32, cfg32, x32 = timed("fp32")
    diff32 = max(float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
                 for a, b in zip(x32, x64))
    # loop of single-problem solves (same systems, FP64 path, inertia correction)
    t_single = 0.0
    for p in range(singles):
        it = items[p]
        S = mds.solver_for(it)
        S.condense(it["sigma_d"], it["dsbase"])
        S.factor_inertia(mu, reg={})
        S.solve(it["r_d"], it["r_s"], it["r_y"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S.condense(it["sigma_d"], it["dsbase"])
        S.factor_inertia(mu, reg={})
        S.solve(it["r_d"], it["r_s"], it["r_y"])
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t1
        del S
    per_single = t_single / singles
    Ns = [it["n_d"] + it["m"] for it in items]
    return dict(workload=f"{count} problems, N = 4*U{{64..512}} (mean {np.mean(Ns):.0f}), "
                         "n_d = N/4, m = 3N/4, n_s = 50N, 4 nnz/row of J_s, FP64",
                problems_per_s=count / dt, ms_per_batch=dt * 1e3,
                tflops_nominal=flops / dt / 1e12,
                latency_ms_p50=float(np.percentile(lat_ms, 50)),
                latency_ms_p99=float(np.percentile(lat_ms, 99)),
                autotuned=cfg, trials_max=max(r["trials"] for r in res),
                single_loop_ms_per_problem=per_single * 1e3,
                speedup_vs_single_loop=per_single * count / dt,
                single_loop_sample=f"first {singles} problems of the batch (sizes differ "
                                   "from the batch mean)",
                fp32_mfma_fp64_refinement=dict(
                    problems_per_s=count / dt32, ms_per_batch=dt32 * 1e3,
                    tflops_nominal=flops / dt32 / 1e12,
                    latency_ms_p50=float(np.percentile(lat32, 50)),
                    latency_ms_p99=float(np.percentile(lat32, 99)),
                    autotuned=cfg32,
                    refine_steps_max=max(r["refine_steps"] for r in res32),
                    refine_steps_mean=float(np.mean([r["refine_steps"] for r in res32])),
                    max_rel_diff_vs_fp64_batch=diff32,
                    speedup_vs_fp64_batch=dt / dt32,
                    speedup_vs_single_loop=per_single * count / dt32))


def warmstart_section(n_train, n_held, hidden=128, steps=3000, lr=3e-3, noise=0.5):
    """Learned warm start on a family of N = 192 problems (the C0 shapes; only
    b varies): cold FP64 IPM solves generate the training set; the perceptron
    b -> (x_d, y, log10 mu0) (two GELU layers plus a linear skip path) is
    trained with the library's kernels on input-noised minibatches; held-out
    problems are solved warm (BF16 inference, cold fallback) and cold."""
    import numpy as np
    import torch
    import paper_2605_13736_amd as mds
    import synth
    from paper_2605_13736_amd import warmstart
    base = synth.config_problem(synth.IPM_N192)
    train = [synth.family_member(base, p) for p in range(n_train)]
    held = [synth.family_member(base, 10 ** 6 + p) for p in range(n_held)]
    t0 = time.perf_counter()
    X, T, _, _ = warmstart.solve_family(train)
    t_data = time.perf_counter() - t0
    ws = warmstart.WarmStart(base["m"], base["n_d"], hidden=hidden, max_batch=256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = ws.fit(X, T, steps=steps, lr=lr, batch=128, noise=noise)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    S = mds.solver_for(base)
    cold_it, warm_it, cold_t, warm_t, fb, err = [], [], 0.0, 0.0, 0, 0.0
    for q in held:
        S.P["b"].copy_(S.dev(q["b"]))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c = S.ipm_solve()
        torch.cuda.synchronize()
        cold_t += time.perf_counter() - t1
        xc = c["x"].cpu().numpy().copy()
        t1 = time.perf_counter()
        w = ws.solve(S, q["b"])
        torch.cuda.synchronize()
        warm_t += time.perf_counter() - t1
        cold_it.append(c["iters"])
        warm_it.append(w["warm_iters"])
        fb += int(w["fallback"])
        err = max(err, float(np.abs(w["x"].cpu().numpy() - xc).max()))
    Xn = np.zeros((1, base["m"]), dtype=np.float32)
    ws.net.forward(Xn, "bf16")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        ws.net.forward(Xn, "bf16")
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t1) / 20
    return dict(workload=f"family of N=192 problems (n_d=64, n_s=2000, m=128; b varies), "
                         f"{len(X)} training / {n_held} held-out",
                mlp=f"{base['m']}-{hidden}-{hidden}-{base['n_d'] + base['m'] + 1}, GELU, linear skip, "
                    f"FP32-MFMA training (Adam lr {lr}, {steps} steps, input noise {noise}), "
                    "BF16-MFMA inference",
                data_s=t_data, train_s=t_train, train_steps=steps,
                loss_first=losses[0], loss_last=losses[-1], inference_ms=t_inf * 1e3,
                cold_iters_mean=float(np.mean(cold_it)), warm_iters_mean=float(np.mean(warm_it)),
                iters_saved_frac=1.0 - float(np.mean(warm_it)) / float(np.mean(cold_it)),
                fallback_rate=fb / n_held, cold_solves_per_s=n_held / cold_t,
                warm_solves_per_s=n_held / warm_t, max_abs_x_diff_vs_cold=err)


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


def ipm_solves_section(nrep=5):
    """Whole FP64 IPMs on the N = 192 workload: solves per second."""
    import torch

    import paper_2605_13736_amd as mds
    import synth
    prob0 = synth.config_problem(synth.IPM_N192)
    S0 = mds.solver_for(prob0)
    r = S0.ipm_solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(nrep):
        r = S0.ipm_solve()
    torch.cuda.synchronize()
    d0 = (time.perf_counter() - t1) / nrep
    return {"workload": "whole FP64 IPM to E_0 <= 1e-8, n_d=64 n_s=2000 m=128 (N=192)",
            "solves_per_s": 1.0 / d0, "iters": r["iters"], "status": r["status"],
            "panel": S0.info()["panel"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ipm-solves", action="store_true")
    ap.add_argument("--ipm-only", action="store_true",
                    help="run only the whole-IPM section (N = 192) and print it (profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the scenario-batch section and print it (profiling)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--ws-train", type=int, default=1024)
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
    if args.ipm_only:
        print(json.dumps({"ipm_solves": ipm_solves_section()}))
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_section(args.batch_count)}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_13736_amd as mds
    import synth

    cfg = synth.CONFIGS[synth.OPF_N4096]
    prob = synth.config_problem(synth.OPF_N4096)
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
    # throughput: K steps with no event records between the launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    facs = solves = 0
    for _ in range(args.steps):
        info = step()
        facs += info["trials"]
        solves += info["solves"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flops = facs * N ** 3 / 3.0 + solves * 2.0 * N ** 2
    value = flops / dt / 1e12
    log(f"timed {args.steps} steps in {dt:.3f}s: {facs} factorizations, {solves} solves")
    # per-kernel-class device time: K more steps with HIP event pairs around
    # every launch on the library's stream (the events add launch gaps, so
    # this region is not the throughput one)
    S.set_timing(True)
    torch.cuda.synchronize()
    te = time.perf_counter()
    efacs = 0
    for _ in range(args.steps):
        efacs += step()["trials"]
    torch.cuda.synchronize()
    dte = time.perf_counter() - te
    tim = S.get_timings()
    S.set_timing(False)
    log("per-class device time:", json.dumps(tim))

    # dominant kernel roofline
    dom = max(tim, key=lambda k: tim[k]["ms"])
    nlaunch = max(tim[dom]["launches"], 1)
    avg_s = tim[dom]["ms"] / 1e3 / nlaunch
    if dom == "panel":
        tail = tim["panel_tail"]["launches"] > 0
        per_launch = panel_bytes_per_launch(N, tim["panel"]["launches"] / max(efacs, 1),
                                            adv=max(nb - 1, 1) if tail else None)
        roof = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK_GBS,
                    unit="GB/s")
    elif dom == "trailing":
        npan = tim["panel"]["launches"] + tim["panel_tail"]["launches"]
        per_launch = trailing_bytes_per_launch(N, N / max(npan / max(efacs, 1), 1))
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
    panel_kernel = {"reg": "k_bk_panel_reg", "coop": "k_bk_panel_coop"}.get(info0["panel"], "k_bk_panel")
    roof["kernel"] = {"panel": panel_kernel, "panel_tail": "k_bk_panel_reg",
                      "trailing": "k_bk_trailing",
                      "solve": "k_trsv_fwd+k_trsv_bwd", "condense": "k_condense_dense",
                      "permute": "k_std_sweep+k_std_apply"}[dom]
    meas = MEASURED_TRAFFIC.get(roof["kernel"])
    roof["traffic"] = meas[0] if meas else None
    if meas:
        roof["traffic_source"] = meas[1]
    roof["avg_launch_us"] = avg_s * 1e6
    roof["bytes_per_launch"] = per_launch
    fac_ms = (tim["panel"]["ms"] + tim["panel_tail"]["ms"] + tim["trailing"]["ms"]) / max(efacs, 1)
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
        "event_region": {"steps": args.steps, "ms_per_step": dte / args.steps * 1e3,
                         "factorizations": efacs},
    }

    if not args.no_ipm_solves:
        out["ipm_solves"] = ipm_solves_section()
    if not args.no_mixed:
        log("mixed precision section")
        out["mixed"] = mixed_section(prob, N)
    if not args.no_batch:
        log("batch section")
        out["batch"] = batch_section(args.batch_count)
    if not args.no_warmstart:
        log("learned warm start section")
        out["warmstart"] = warmstart_section(args.ws_train, 32)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

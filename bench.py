"""Benchmark of the condensed-KKT hot path on one MI355X.

Headline (the printed `value`): the large condensed system (n_d = 4096,
n_s = 1000000, m = 12288, condensed N = 16384, 8 nonzeros per row of J_s,
Sigma_d and D_s drawn log-uniform over 1e-8..1e8 as at the end of a barrier
run; seeded synthetic data resident in HBM before the timed region).  One
step is the whole Newton-system path: condense (Sec. 2.2), Bunch-Kaufman
factorization with the inertia-correction loop (Sec. 2.1, 2.3), solve and
back-substitution, FP64 iterative refinement on the full system to backward
error 1e-14.  value = KKT factor+solve TFLOP/s = (N^3/3 per factorization +
2 N^2 per solve) / wall time of the K timed steps, in FP64.

Beside it, in the same JSON line:
* `precision_sweep`: the same system with FP32 / split-BF16 / BF16 trailing
  updates and FP64 GMRES refinement: time, speedup over FP64 at the same
  backward error, GMRES iterations, and the error against the FP64 solution
  and against the oracle's stored solution;
* `opf_n4096`: IPM Newton steps on the OPF-scale problem (N = 4096), their
  per-kernel breakdown, one whole IPM to E_0 <= 1e-8 (solves/s), and one
  Newton system per precision;
* `ipm_solves`: whole IPMs on the N = 192 problem; `batch`: 512 scenario
  problems in one persistent launch; `warmstart`: the learned warm start;
* `roofline` for the dominant kernel of the headline step (HIP events on the
  library's stream), `factor` with the factorization's FP64-MFMA fraction;
* `cpu_baseline`: the oracle on a bounded sample of the headline workload,
  on one pinned host core and on all host cores (bit-identical results).
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
FP32_MFMA_PEAK_TFS = 157.3
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by
# the counters of a 256 MiB copy (the profile file gives the commands and the
# factors); valid for the kernel source and workload as profiled.
MEASURED_TRAFFIC = {
    ("k_bk_trailing_la", 16384): (807272437.0, "profiles/bk_trailing_kkt_n16384.md"),
    ("k_bk_trailing", 4096): (45959473.4, "profiles/bk_trailing_ipm_newton_step_n4096.md"),
    ("k_bk_panel_coop", 4096): (4594730.0, "profiles/bk_panel_coop_ipm_newton_step_n4096.md"),
}
KERNEL_OF_CLASS = {"panel_tail": "k_bk_panel_reg", "trailing": "k_bk_trailing",
                   "solve": "k_trsv_fwd+k_trsv_bwd", "condense": "k_condense_dense",
                   "permute": "k_std_sweep+k_std_apply"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def panel_bytes_per_launch(N, launches_per_factor, adv=None):
    """Algorithmic HBM bytes of one panel launch, averaged over its launches:
    a panel of width w starting at k0 reads its w columns (rows >= k0) once,
    reads one pivot-candidate column per pivot, and writes L and W once:
    4 * (N - k0) * w * 8 bytes, i.e. 4 * 8 * (N - c) per column c.  When the
    launches cover only the first columns (a cooperative panel that hands the
    last rows to another kernel), they cover launches * adv columns."""
    n = max(launches_per_factor, 1)
    K = N if adv is None else min(N, n * adv)
    return 4.0 * 8.0 * (K * N - K * (K - 1) / 2.0) / n


def trailing_bytes_per_launch(N, w, elem=8.0):
    """Algorithmic bytes of one trailing update (panels of width w): read and
    write the lower trailing triangle (elem bytes per entry: 8 in FP64, 4 in
    FP32 storage), read the L and W panels (FP64)."""
    total, cnt, k0 = 0.0, 0, 0
    while k0 + w < N:
        n = N - (k0 + w)
        total += (n * (n + 1) / 2) * elem * 2 + 2.0 * n * w * 8.0
        cnt += 1
        k0 += w
    return total / max(cnt, 1)


def slot_widths(N, nb=32, tail_rows=2048):
    """Columns each panel launch factors at least, in the library's slot plan
    for the automatic cooperative factorization: nb - 1 while more than
    tail_rows rows remain, then the register tail (16-column tile above 1024
    rows, the 32-column one below).  Panels end on these widths except where
    a 2x2 pivot closes a panel one column later."""
    rows, ws = N, []
    while rows > 0:
        if rows <= tail_rows:
            a = min(16 if rows > 1024 else 32, nb) - 1
        else:
            a = nb - 1
        ws.append(a)
        rows -= a
    return ws


def trailing_bytes_plan(N, nb=32, elem=8.0):
    """Algorithmic bytes of one trailing update averaged over the slot plan's
    updates (per update as trailing_bytes_per_launch, at each panel's own
    width); returns (bytes per update, updates per factorization)."""
    total, cnt, k0 = 0.0, 0, 0
    for w in slot_widths(N, nb):
        n = N - (k0 + w)
        if n <= 0:
            break
        total += (n * (n + 1) / 2) * elem * 2 + 2.0 * n * w * 8.0
        cnt += 1
        k0 += w
    return total / max(cnt, 1), cnt


def trailing_flops_plan(N, nb=32):
    """Flops of one trailing update (2 w per lower entry) averaged over the
    slot plan's updates."""
    total, cnt, k0 = 0.0, 0, 0
    for w in slot_widths(N, nb):
        n = N - (k0 + w)
        if n <= 0:
            break
        total += (n * (n + 1) / 2) * 2.0 * w
        cnt += 1
        k0 += w
    return total / max(cnt, 1)


def trailing_flops_per_launch(N, w):
    """Flops of one trailing update: 2 w per lower entry of the trailing matrix."""
    total, cnt, k0 = 0.0, 0, 0
    while k0 + w < N:
        n = N - (k0 + w)
        total += (n * (n + 1) / 2) * 2.0 * w
        cnt += 1
        k0 += w
    return total / max(cnt, 1)


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = sorted(os.sched_getaffinity(0))
    except AttributeError:
        avail = list(range(os.cpu_count() or 1))
    return dict(nproc=os.cpu_count(), cpus_available=len(avail), model=model), avail


# ---------------------------------------------------------------- headline
def kkt_step_section(args):
    """The headline: K steps of condense + factor (correction loop) + refined
    solve of the N = 16384 system in FP64, then K more with per-launch events
    for the per-class breakdown and the roofline."""
    import torch
    import paper_2605_13736_amd as mds
    import synth
    prob = synth.config_problem(synth.LARGE_N16384)
    st = synth.kkt_state(prob, 2)
    N = prob["n_d"] + prob["m"]
    S = mds.solver_for(prob, nb=args.nb)
    info0 = S.info()
    sd, db = S.dev(st["sigma_d"]), S.dev(st["dsbase"])
    rd, rs, ry = S.dev(st["r_d"]), S.dev(st["r_s"]), S.dev(st["r_y"])
    mu = 1e-8  # late barrier parameter (enters only delta_c of a singular M)
    reg = {}

    def step():
        nonlocal reg
        S.condense(sd, db)
        status, inn, r = S.factor_inertia(mu, reg=dict(delta_w_last=reg.get("delta_w_last", 0.0)))
        reg = r
        sol, ri = S.refine(rd, rs, ry, 3, 1e-14)
        return r["trials"], 1 + ri["steps"], ri, sol, inn

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    facs = solves = 0
    for _ in range(args.steps):
        f, s, ri, sol, inn = step()
        facs += f
        solves += s
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = (facs * N ** 3 / 3.0 + solves * 2.0 * N ** 2) / dt / 1e12
    log(f"headline: {args.steps} steps in {dt:.3f}s, {facs} factorizations, {solves} solves")
    x64 = torch.cat(sol).cpu().numpy()
    # per-class device time with HIP event pairs on the library stream
    S.set_timing(True)
    torch.cuda.synchronize()
    te = time.perf_counter()
    efacs = 0
    for _ in range(args.steps):
        efacs += step()[0]
    torch.cuda.synchronize()
    dte = time.perf_counter() - te
    tim = S.get_timings()
    S.set_timing(False)
    log("per-class device time:", json.dumps(tim))
    # pivot statistics of the last factorization and the exchange floor of
    # the cooperative panel at its first panels' width (outside the timed
    # regions)
    pstats = S.panel_stats()
    P = min(32, (N + 1023) // 1024)
    xfloor = dict(P=P, first_exchange_us=S.probe_exchange(P, 2000, 69),
                  second_exchange_us=S.probe_exchange(P, 2000, 16),
                  words=dict(first=69, second=16), rounds=2000)
    out = dict(N=N, dt=dt, facs=facs, solves=solves, value=value, tim=tim, efacs=efacs,
               dte=dte, info=info0, eta=ri["eta"], inertia=inn, x64=x64, pstats=pstats,
               xfloor=xfloor)
    del S
    torch.cuda.empty_cache()
    return out, prob, st


def factor_ms_of(tim, efacs):
    """Device time of one factorization: the event pair around each whole
    factorization on the handle's stream (with look-ahead its panels and
    trailing updates overlap, so the per-class sum would count the overlap
    twice); the per-class sum for timings without that class."""
    f = tim.get("factor", {})
    if f.get("launches"):
        return f["ms"] / f["launches"]
    return (tim["panel"]["ms"] + tim["panel_tail"]["ms"] + tim["trailing"]["ms"]) / max(efacs, 1)


def roofline_of(tim, efacs, N, nb, pstats=None, xfloor=None):
    """The factorization, the step's dominant work (cooperative panel, its
    register tail and the trailing updates), against FP64 MFMA; inside it the
    trailing update against HBM (its own roofline, with the counter traffic)
    and the panel's latency model (microseconds per pivot step against the
    measured exchange round trip)."""
    fac_ms = factor_ms_of(tim, efacs)
    factor_tfs = (N ** 3 / 3.0) / (fac_ms / 1e3) / 1e12
    trl = tim["trailing"]
    near = tim.get("near", {"ms": 0.0, "launches": 0})
    la = near["launches"] > 0
    nl = max(trl["launches"], 1)
    # with look-ahead one update is the near strip (reserved units) plus the
    # rest (the other units, beside the next panel)
    avg_s = (trl["ms"] + near["ms"]) / 1e3 / nl
    # the slot plan's widths (cooperative panels, then the register tail)
    per_launch, _ = trailing_bytes_plan(N, nb)
    meas = MEASURED_TRAFFIC.get(("k_bk_trailing_la" if la else "k_bk_trailing", N))
    trailing = dict(kernel="k_bk_trailing_ps" + (" (near strip + rest)" if la else ""),
                    bound="hbm", achieved=per_launch / avg_s / 1e9,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=per_launch / avg_s / 1e9 / HBM_PEAK_GBS,
                    traffic=meas[0] if meas else None, bytes_per_launch=per_launch,
                    flops_per_launch=trailing_flops_plan(N, nb),
                    avg_launch_us=avg_s * 1e6, launches=nl,
                    ms_per_factorization=(trl["ms"] + near["ms"]) / max(efacs, 1))
    if la:
        trailing["near_ms_per_factorization"] = near["ms"] / max(efacs, 1)
    if meas and meas[0] is not None:
        trailing["traffic_source"] = meas[1]
        trailing["traffic_over_algorithmic"] = meas[0] / per_launch
    return dict(bound="mfma", kernel="factorization (k_bk_panel_coop, k_bk_panel_reg tail, "
                                     "k_bk_trailing_ps" + (", look-ahead" if la else "") + ")",
                achieved=factor_tfs, peak=FP64_MFMA_PEAK_TFS, unit="TFLOP/s",
                frac=factor_tfs / FP64_MFMA_PEAK_TFS, traffic=None,
                flops_per_launch=N ** 3 / 3.0, avg_launch_us=fac_ms * 1e3, launches=efacs,
                trailing=trailing, panel=panel_latency_model(tim, efacs, N, nb, pstats, xfloor))


def panel_latency_model(tim, efacs, N, nb, pstats=None, xfloor=None):
    """Microseconds per pivot step of the cooperative panel and of its
    register tail (a latency-bound chain: one or two grid-wide exchanges and
    one dependent column read per step), and, with the pivot statistics and
    the measured exchange round trip, the floor that the exchanges alone set
    (first exchange every step, the second on the steps whose first test
    fails)."""
    out = {}
    for cls in ("panel", "panel_tail"):
        n = tim[cls]["launches"]
        if n:
            out[cls] = dict(us_per_launch=tim[cls]["ms"] * 1e3 / n,
                            us_per_pivot=tim[cls]["ms"] * 1e3 / n / max(nb - 1, 1),
                            launches_per_factorization=n / max(efacs, 1))
    if pstats and pstats.get("coop_steps") and tim["panel"]["launches"]:
        per_fac = tim["panel"]["launches"] / max(efacs, 1)
        steps_per_launch = pstats["coop_steps"] / per_fac
        us_step = tim["panel"]["ms"] * 1e3 / tim["panel"]["launches"] / steps_per_launch
        f2 = pstats["coop_second"] / pstats["coop_steps"]
        m = dict(steps_per_factorization=pstats["coop_steps"], second_exchange_frac=f2,
                 us_per_step=us_step, n2x2=pstats["n2x2"])
        if xfloor:
            floor = xfloor["first_exchange_us"] + f2 * xfloor["second_exchange_us"]
            m.update(exchange_floor_us_per_step=floor, step_over_floor=us_step / floor,
                     probe=xfloor)
        out["coop_model"] = m
    return out


def precision_sweep(prob, st, N, reps=2, precs=("fp64", "fp32", "bf16x3", "bf16")):
    """The headline Newton matrix without shifts (the first trial of the
    correction loop) in each precision: condense + factor + refined solve to
    backward error 1e-14 (classic FP64 refinement for FP64, at most 60 FP64
    GMRES iterations for the mixed modes).  Errors are measured against the
    FP64 run of the same system and against the oracle's stored entries."""
    import numpy as np
    import torch
    import paper_2605_13736_amd as mds
    gold = None
    try:
        g = json.load(open(os.path.join(ROOT, "tests", "golden", "kkt_n16384.json")))
        gold = (np.asarray(g["x_index"]), np.asarray(g["x_value"]), g["x_absmax"], g["inertia"])
    except (OSError, KeyError, ValueError):
        pass
    out, x64 = {}, None
    for prec in precs:
        S = mds.solver_for(prob, precision=prec)
        sd, db = S.dev(st["sigma_d"]), S.dev(st["dsbase"])
        rd, rs, ry = S.dev(st["r_d"]), S.dev(st["r_s"]), S.dev(st["r_y"])
        steps = 3 if prec == "fp64" else 60

        def once():
            S.condense(sd, db)
            _, inn, _ = S.factor_inertia()
            sol, info = S.refine(rd, rs, ry, steps, 1e-14)
            return sol, info, inn

        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sol, info, inn = once()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        S.set_timing(True)
        once()
        tim = S.get_timings()
        S.set_timing(False)
        fac_ms = factor_ms_of(tim, 1)
        x = torch.cat(sol).cpu().numpy()
        if x64 is None:
            x64 = x
        rec = dict(ms_condense_factor_refine=dt * 1e3, ms_factor=fac_ms,
                   ms_trailing=tim["trailing"]["ms"] + tim["near"]["ms"],
                   ms_panel=tim["panel"]["ms"] + tim["panel_tail"]["ms"],
                   tflops_nominal=(N ** 3 / 3.0 + 2.0 * N ** 2) / dt / 1e12,
                   refine_iterations=info["steps"], eta=info["eta"],
                   inertia=[inn["npos"], inn["nzero"], inn["nneg"]],
                   rel_err_vs_fp64=float(np.abs(x - x64).max() / np.abs(x64).max()))
        if gold is not None:
            rec["rel_err_vs_oracle_sampled"] = float(
                np.abs(x[gold[0]] - gold[1]).max() / gold[2])
            rec["inertia_equals_oracle"] = rec["inertia"] == gold[3]
        out[prec] = rec
        del S
        torch.cuda.empty_cache()
    base = out[precs[0]]["ms_condense_factor_refine"]
    for prec, rec in out.items():
        if "fp64" in out:
            rec["speedup_vs_fp64"] = base / rec["ms_condense_factor_refine"]
        rec["converged_1e-14"] = rec["eta"] <= 1e-14
    return out


# ---------------------------------------------------------------- N = 4096
def opf_section(steps=10, warmup=2):
    """IPM Newton steps on the OPF-scale workload (n_d = 1024, n_s = 200000,
    m = 3072, N = 4096): per-step time and TFLOP/s, the per-class breakdown,
    and one whole IPM from the cold start to E_0 <= 1e-8."""
    import torch
    import paper_2605_13736_amd as mds
    import synth
    prob = synth.config_problem(synth.OPF_N4096)
    N = prob["n_d"] + prob["m"]
    S = mds.solver_for(prob)
    it = S.new_iterate()
    S.ipm_init(it)

    def step():
        st, info = S.ipm_step(it)
        if st != 0:
            S.ipm_init(it)
            st, info = S.ipm_step(it)
        return info

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    facs = solves = 0
    for _ in range(steps):
        info = step()
        facs += info["trials"]
        solves += info["solves"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.set_timing(True)
    efacs = 0
    for _ in range(steps):
        efacs += step()["trials"]
    tim = S.get_timings()
    S.set_timing(False)
    pstats = S.panel_stats()
    P = (N + 1023) // 1024
    xfloor = dict(P=P, first_exchange_us=S.probe_exchange(P, 2000, 69),
                  second_exchange_us=S.probe_exchange(P, 2000, 16),
                  words=dict(first=69, second=16), rounds=2000)
    fac_ms = factor_ms_of(tim, efacs)
    # whole IPM
    r = S.ipm_solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = S.ipm_solve()
    torch.cuda.synchronize()
    t_ipm = time.perf_counter() - t1
    last = r["trace"][r["iters"]] if len(r["trace"]) > r["iters"] else r["trace"][-1]
    out = dict(workload="FP64 IPM Newton steps, n_d=1024 n_s=200000 m=3072 (N=4096), J_s 6 nnz/row",
               ms_per_step=dt / steps * 1e3,
               tflops=(facs * N ** 3 / 3.0 + solves * 2.0 * N ** 2) / dt / 1e12,
               factor_ms=fac_ms, factor_tflops=(N ** 3 / 3.0) / (fac_ms / 1e3) / 1e12,
               kernel_ms_per_step={k: v["ms"] / steps for k, v in tim.items()},
               panel_latency=panel_latency_model(tim, efacs, N, S.info()["nb"], pstats, xfloor),
               whole_ipm=dict(status=r["status"], iters=r["iters"], seconds=t_ipm,
                              solves_per_s=1.0 / t_ipm, final_E0=last["E0"],
                              last_step_eta=r["trace"][r["iters"] - 1]["eta"]))
    del S
    torch.cuda.empty_cache()
    return out, prob


def opf_mixed_section(prob, reps=3):
    """One Newton system of the N = 4096 workload at a seeded interior point,
    solved to backward error 1e-14 by FP64 factor + classic refinement and by
    the mixed modes + FP64 GMRES refinement."""
    import numpy as np
    import torch
    import paper_2605_13736_amd as mds
    import synth
    it = synth.interior_iterate(prob, 0)
    nd = prob["n_d"]
    N = nd + prob["m"]
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
        t0 = time.perf_counter()
        for _ in range(reps):
            sol, info = once()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        x = torch.cat(sol).cpu().numpy()
        if ref is None:
            ref = x
        out[prec] = dict(ms_condense_factor_refine=dt * 1e3,
                         tflops_nominal=(N ** 3 / 3.0 + 2.0 * N ** 2) / dt / 1e12,
                         refine_iterations=info["steps"], eta=info["eta"],
                         rel_err_vs_fp64=float(abs(x - ref).max() / max(abs(ref).max(), 1e-300)))
        del S
        torch.cuda.empty_cache()
    return out


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


def batch_section(count, mu=0.05, singles=6):
    """The scenario batch: count problems with N = 4 U{64..512}, n_d = N/4,
    m = 3N/4, n_s = 50N, 4 nonzeros per row of J_s, each at a seeded barrier
    state; solved by the persistent kernel after autotuning, in FP64 and in
    the FP32-tile form with FP64 refinement.  Also times a loop of
    single-problem FP64 solves on the first `singles` problems."""
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


def batch_ipm_section(count, singles=4):
    """Whole FP64 IPMs of the scenario batch in one persistent kernel (each
    workgroup runs complete IPMs of the problems it takes, largest first):
    count problems with N = 4 U{64..512}, n_d = N/4, m = 3N/4, n_s = 50N,
    4 nonzeros per row of J_s.  Also times a loop of single-problem GPU IPMs
    on the first `singles` problems."""
    import numpy as np
    import torch
    import paper_2605_13736_amd as mds
    import synth
    probs = []
    for p in range(count):
        sz = synth.batch_sizes(p)
        probs.append(synth.make_problem(sz["n_d"], sz["n_s"], sz["m"], sz["r"], cfg=3, p=p))
    B = mds.BatchIPM(probs, max_iter=200)
    B.solve(trace=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = B.solve(trace=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = np.array([r["iters"] for r in res], dtype=np.float64)
    facs = np.array([r["factorizations"] for r in res], dtype=np.float64)
    lat = np.array([r["t_done"] for r in res], dtype=np.float64) / 1e5
    Ns = [q["n_d"] + q["m"] for q in probs]
    flops = sum(f * (N ** 3 / 3.0) for f, N in zip(facs, Ns))
    conv = sum(r["status"] == "converged" for r in res)
    B.close()
    del B
    torch.cuda.empty_cache()
    t_single = 0.0
    for p in range(singles):
        S = mds.solver_for(probs[p])
        S.ipm_solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S.ipm_solve()
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t1
        del S
    per_single = t_single / singles
    return dict(workload=f"{count} problems, N = 4*U{{64..512}} (mean {np.mean(Ns):.0f}), "
                         "n_d = N/4, m = 3N/4, n_s = 50N, 4 nnz/row of J_s; whole FP64 IPM "
                         "to E_0 <= 1e-8 per problem",
                ipm_solves_per_s=count / dt, seconds=dt, converged=int(conv),
                iters_mean=float(iters.mean()), iters_max=int(iters.max()),
                factorizations_total=int(facs.sum()),
                factor_tflops_nominal=flops / dt / 1e12,
                latency_s_p50=float(np.percentile(lat, 50)) / 1e3,
                latency_s_p99=float(np.percentile(lat, 99)) / 1e3,
                single_loop_s_per_problem=per_single,
                speedup_vs_single_loop=per_single * count / dt,
                single_loop_sample=f"first {singles} problems of the batch, one GPU IPM each")


def warmstart_section(n_train, n_held, hidden=1024, steps=2000, lr=1e-3, noise=0.5,
                      data_budget_s=None):
    """Learned warm start on the OPF-scale family (N = 4096; b = b0 (1 + 0.1
    N(0,1)) per entry): cold FP64 IPM solves generate the training set (at
    most n_train, or what data_budget_s seconds of solves produce); the
    perceptron b (3072) -> 1024 -> 1024 -> (x_d, y, log10 mu0) (4097) with
    GELU (plus a linear skip path) is trained with the library's kernels;
    held-out problems are solved warm (BF16 inference, cold fallback) and
    cold."""
    import numpy as np
    import torch
    import paper_2605_13736_amd as mds
    import synth
    from paper_2605_13736_amd import warmstart
    base = synth.config_problem(synth.OPF_N4096)
    t0 = time.perf_counter()
    train = [synth.family_member(base, p) for p in range(n_train)]
    X, T, cold_train_iters, _ = warmstart.solve_family(
        train, time_budget_s=data_budget_s,
        progress=lambda k, t: log(f"warm start: {k} training solves in {t:.0f} s"))
    t_data = time.perf_counter() - t0
    ws = warmstart.WarmStart(base["m"], base["n_d"], hidden=hidden, max_batch=256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = ws.fit(X, T, steps=steps, lr=lr, batch=min(128, len(X)), noise=noise)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    S = mds.solver_for(base)
    cold_it, warm_it, cold_t, warm_t, fb, err = [], [], [], [], 0, 0.0
    for p in range(n_held):
        if p and p % 10 == 0:
            log(f"warm start: {p} of {n_held} held-out problems")
        q = synth.family_member(base, 10 ** 6 + p)
        S.P["b"].copy_(S.dev(q["b"]))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c = S.ipm_solve()
        torch.cuda.synchronize()
        cold_t.append(time.perf_counter() - t1)
        xc = c["x"].cpu().numpy().copy()
        t1 = time.perf_counter()
        w = ws.solve(S, q["b"])
        torch.cuda.synchronize()
        warm_t.append(time.perf_counter() - t1)
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
    return dict(workload=f"family of the N=4096 problem (n_d=1024, n_s=200000, m=3072), "
                         f"b = b0 (1 + 0.1 N(0,1)); {len(X)} training solves, "
                         f"{n_held} held-out seeds",
                mlp=f"{ws.dims[0]}-{hidden}-{hidden}-{ws.dims[3]}, GELU, linear skip, "
                    f"FP32-MFMA training (Adam lr {lr}, {steps} steps, input noise {noise}), "
                    "BF16-MFMA inference with FP32 accumulation",
                params=int(ws.net.nparam), data_s=t_data, train_s=t_train,
                train_solves=len(X), loss_first=losses[0], loss_last=losses[-1],
                inference_ms=t_inf * 1e3,
                cold_iters_mean=float(np.mean(cold_it)), warm_iters_mean=float(np.mean(warm_it)),
                iters_saved_frac=1.0 - float(np.mean(warm_it)) / float(np.mean(cold_it)),
                cold_time_to_1e8_s_mean=float(np.mean(cold_t)),
                warm_time_to_1e8_s_mean=float(np.mean(warm_t)),
                speedup=float(np.mean(cold_t)) / float(np.mean(warm_t)),
                fallback_rate=fb / n_held, max_abs_x_diff_vs_cold=err)


# ---------------------------------------------------------------- CPU
def cpu_baseline(prob, st, kstop):
    """The oracle on a bounded sample of the headline workload: the first
    kstop pivot columns of its unblocked Bunch-Kaufman elimination of the
    N = 16384 condensed matrix (the condensation itself is timed and
    reported apart), on one host core pinned with sched_setaffinity and on
    every available core (the elimination's columns split over threads,
    bit-identical results)."""
    import numpy as np
    import oracle
    info, avail = host_info()
    P = oracle.Problem(prob)
    t = time.perf_counter()
    M, _ = oracle.condense(P, st["sigma_d"], st["dsbase"], 0.0, 0.0)
    t_cond = time.perf_counter() - t
    N = M.shape[0]
    flops = sum(float(N - k - 1) * float(N - k) for k in range(kstop))
    res = {}
    old_aff = set(avail)
    for label, cpus in (("one_core", [avail[0]]), ("all_cores", avail)):
        A = np.asfortranarray(M.copy())
        try:
            os.sched_setaffinity(0, set(cpus))
        except (AttributeError, OSError):
            pass
        oracle.set_threads(len(cpus))
        t = time.perf_counter()
        _, ipiv = oracle.bk_partial(A, kstop)
        res[label] = (time.perf_counter() - t, len(cpus), ipiv[:kstop].copy())
        oracle.set_threads(1)
        try:
            os.sched_setaffinity(0, old_aff)
        except (AttributeError, OSError):
            pass
    t1, c1, p1 = res["one_core"]
    tn, cn, pn = res["all_cores"]
    return dict(value=flops / t1 / 1e12, unit="TFLOP/s", cores=c1, kind="oracle",
                sample=f"the first {kstop} pivot columns of the oracle's unblocked Bunch-Kaufman "
                       f"elimination of the N={N} condensed matrix ({flops:.3g} flops, "
                       f"{t1:.1f} s on one core pinned to cpu {avail[0]}); the condensation "
                       f"took {t_cond:.1f} s",
                seconds=t1, host=info,
                all_cores=dict(value=flops / tn / 1e12, cores=cn, seconds=tn,
                               pivots_identical_to_one_core=bool(np.array_equal(p1, pn))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--sweep-precision", default="",
                    help="profiling: only time the headline Newton matrix factored and "
                         "refined in this precision (fp64, fp32, bf16x3, bf16) and print it")
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the headline steps and print them (profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-kstop", type=int, default=60)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-opf", action="store_true")
    ap.add_argument("--no-ipm-solves", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the scenario-batch section and print it (profiling)")
    ap.add_argument("--opf-only", action="store_true",
                    help="run only the N = 4096 section and print it (profiling)")
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--ws-train", type=int, default=400)
    ap.add_argument("--ws-budget", type=float, default=60.0,
                    help="seconds of cold solves that generate warm-start training data")
    ap.add_argument("--ws-held", type=int, default=16)
    ap.add_argument("--ipm-only", action="store_true",
                    help="run only the whole-IPM section (N = 192) and print it (profiling)")
    ap.add_argument("--warmstart-only", action="store_true",
                    help="run only the learned warm-start section and print it")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design only)", file=sys.stderr)
        sys.exit(2)
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
    if args.batch_only:
        print(json.dumps({"batch": batch_section(args.batch_count),
                          "batch_ipm": batch_ipm_section(args.batch_count)}))
        return
    if args.sweep_precision:
        import synth
        prob = synth.config_problem(synth.LARGE_N16384)
        st = synth.kkt_state(prob, 2)
        N = prob["n_d"] + prob["m"]
        print(json.dumps({"precision_sweep": precision_sweep(prob, st, N, reps=args.steps,
                                                             precs=(args.sweep_precision,))}))
        return
    if args.ipm_only:
        print(json.dumps({"ipm_solves": ipm_solves_section()}))
        return
    if args.warmstart_only:
        print(json.dumps({"warmstart": warmstart_section(args.ws_train, args.ws_held,
                                                         data_budget_s=args.ws_budget)}))
        return
    if args.opf_only:
        print(json.dumps({"opf_n4096": opf_section(args.steps, args.warmup)[0]}))
        return

    h, prob, st = kkt_step_section(args)
    N, nb = h["N"], h["info"]["nb"]
    tim, efacs = h["tim"], h["efacs"]
    fac_ms = factor_ms_of(tim, efacs)
    factor_tfs = (N ** 3 / 3.0) / (fac_ms / 1e3) / 1e12
    out = {
        "metric": METRIC, "value": h["value"], "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": h["dt"] / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"KKT factor+solve of one Newton system, n_d=4096 n_s=1000000 "
                               f"m=12288 (N={N}), J_s 8 nnz/row, Sigma_d and D_s log-uniform "
                               "1e-8..1e8, FP64 refinement to backward error 1e-14, "
                               "seeded synthetic", "N": N, "nb": nb,
                   "panel": h["info"]["panel"], "precision": "fp64",
                   "lookahead_cus": h["info"]["lookahead_cus"]},
        "roofline": roofline_of(tim, efacs, N, nb, h.get("pstats"), h.get("xfloor")),
        "factor": {"ms_per_factorization": fac_ms, "tflops": factor_tfs,
                   "bound": "mfma", "peak_tflops": FP64_MFMA_PEAK_TFS,
                   "frac_fp64_mfma_peak": factor_tfs / FP64_MFMA_PEAK_TFS,
                   "factorizations": h["facs"], "solves": h["solves"],
                   "eta": h["eta"],
                   "inertia": [h["inertia"]["npos"], h["inertia"]["nzero"], h["inertia"]["nneg"]]},
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in tim.items()},
        "panel_latency": panel_latency_model(tim, efacs, N, nb, h.get("pstats"), h.get("xfloor")),
        "event_region": {"steps": args.steps, "ms_per_step": h["dte"] / args.steps * 1e3,
                         "factorizations": efacs},
    }
    if args.headline_only:
        print(json.dumps(out), flush=True)
        return
    if not args.no_sweep:
        log("precision sweep")
        out["precision_sweep"] = precision_sweep(prob, st, N)
    if not args.no_opf:
        log("N = 4096 section")
        opf, prob1 = opf_section()
        opf["mixed"] = opf_mixed_section(prob1)
        out["opf_n4096"] = opf
    if not args.no_ipm_solves:
        out["ipm_solves"] = ipm_solves_section()
    if not args.no_batch:
        log("batch section")
        out["batch"] = batch_section(args.batch_count)
    if not args.no_batch:
        log("batch whole-IPM section")
        out["batch_ipm"] = batch_ipm_section(args.batch_count)
    if not args.no_warmstart:
        log("learned warm start section")
        out["warmstart"] = warmstart_section(args.ws_train, args.ws_held,
                                             data_budget_s=args.ws_budget)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(prob, st, args.cpu_kstop)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

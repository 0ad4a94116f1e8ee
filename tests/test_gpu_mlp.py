"""Warm-start perceptron kernels and the warm-started IPM against the oracle.

Bars:
* forward: FP32 MFMA within 1e-4 and BF16 MFMA within 3e-2 of the FP64
  reference (relative to max |Y|);
* gradient of the mean-squared error within 1e-3 (relative to max |g|) and
  the loss within 1e-5 of the reference; one Adam step equal to the
  reference update applied to the same gradient within 1e-6;
* warm-started IPM: same status, iteration count, per-iteration inertia,
  trials and backtracks as the oracle's warm start, final x within 1e-8;
* learned warm start end to end: every held-out problem converges (warm, or
  cold after a warm failure) to the cold solution within 1e-5 (two different
  paths end at two points with E_0 <= 1e-8, which on this problem lie up to
  ~1e-6 apart);
* trained on 1024 solves, the learned start saves at least half an IPM
  iteration on average over 16 held-out problems (measured: about 1.5 of 13).
"""
import numpy as np
import pytest

import oracle
import paper_2605_13736_amd as mds
import synth
from oracle import mlp as omlp
from paper_2605_13736_amd import warmstart

pytestmark = pytest.mark.gpu

DIMS = (128, 256, 256, 193)


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _setup(seed=0, batch=64):
    rng = np.random.default_rng(seed)
    p = omlp.init_params(DIMS, seed) + 0.02 * rng.standard_normal(omlp.n_params(DIMS))
    X = rng.standard_normal((batch, DIMS[0]))
    T = rng.standard_normal((batch, DIMS[3]))
    net = mds.MLP(DIMS, 128)
    net.set_params(p.astype(np.float32))
    p32 = p.astype(np.float32).astype(np.float64)  # the reference sees the FP32 parameters
    return net, p32, X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 3e-2)])
def test_mlp_forward_matches_reference(prec, tol):
    say(f"mlp forward {prec}")
    net, p, X, _ = _setup()
    Y = net.forward(X, precision=prec).cpu().numpy().astype(np.float64)
    Yr, _ = omlp.forward(p, DIMS, X)
    assert np.abs(Y - Yr).max() <= tol * np.abs(Yr).max()


def test_mlp_gradient_and_adam_match_reference():
    say("mlp gradient + adam")
    net, p, X, T = _setup(1)
    loss = net.train_step(X, T, 1e-3)
    g = net.get_grad().astype(np.float64)
    Lr, gr = omlp.loss_and_grad(p, DIMS, X, T)
    assert loss == pytest.approx(Lr, rel=1e-5)
    assert np.abs(g - gr).max() <= 1e-3 * np.abs(gr).max()
    p1 = net.get_params().astype(np.float64)
    pr, _, _ = omlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    assert np.abs(p1 - pr).max() <= 1e-6


def test_warm_started_ipm_matches_oracle():
    prob = synth.config_problem(synth.IPM_N192)
    say("warm-started ipm N=192")
    P = oracle.Problem(prob)
    cold = oracle.ipm(P)
    nd = prob["n_d"]
    rng = np.random.default_rng(7)
    warm = dict(x_d=cold["x"][:nd] + 0.05 * rng.standard_normal(nd),
                y=cold["y"] * (1 + 0.05 * rng.standard_normal(prob["m"])), mu0=1e-3)
    r_o = oracle.ipm(P, warm=warm)
    S = mds.solver_for(prob)
    r_g = S.ipm_solve_warm(warm["x_d"], warm["y"], warm["mu0"])
    assert r_g["status"] == r_o["status"] == "converged"
    assert r_g["iters"] == r_o["iters"]
    for k in range(r_o["iters"]):
        a, b = r_g["trace"][k], r_o["trace"][k]
        assert a["mu"] == pytest.approx(b["mu"], rel=1e-10), k
        assert a["inertia"] == b["inertia"] and a["trials"] == b["trials"], k
        assert a["backtracks"] == b["backtracks"], k
    x = r_g["x"].cpu().numpy()
    assert np.abs(x - r_o["x"]).max() <= 1e-8 * max(1.0, np.abs(r_o["x"]).max())


def test_learned_warm_start_end_to_end():
    base = synth.config_problem(synth.IPM_N192)
    say("learned warm start: 48 training problems, 6 held out")
    train = [synth.family_member(base, p) for p in range(48)]
    held = [synth.family_member(base, 10 ** 6 + p) for p in range(6)]
    X, T, cold_iters, _ = warmstart.solve_family(train)
    assert len(X) == 48
    ws = warmstart.WarmStart(base["m"], base["n_d"], hidden=256, max_batch=64)
    losses = ws.fit(X, T, steps=200, lr=1e-3, batch=32)
    assert losses[-1] < losses[0]
    S = mds.solver_for(base)
    for q in held:
        S.P["b"].copy_(S.dev(q["b"]))
        c = S.ipm_solve()
        xc = c["x"].cpu().numpy().copy()
        w = ws.solve(S, q["b"])
        say(f"  cold {c['iters']} warm {w['warm_iters']} fallback {w['fallback']}")
        assert w["status"] == "converged"
        assert np.abs(w["x"].cpu().numpy() - xc).max() <= 1e-5


def test_learned_warm_start_saves_iterations():
    # 1024 training solves of the N = 192 family, 16 held-out problems: the
    # learned start (two GELU layers plus the linear skip path, trained on
    # input-noised minibatches) needs fewer IPM iterations than the cold start
    base = synth.config_problem(synth.IPM_N192)
    say("learned warm start gain: 1024 training problems, 16 held out")
    train = [synth.family_member(base, p) for p in range(1024)]
    held = [synth.family_member(base, 10 ** 6 + p) for p in range(16)]
    X, T, _, _ = warmstart.solve_family(train)
    ws = warmstart.WarmStart(base["m"], base["n_d"], hidden=128, max_batch=256)
    ws.fit(X, T, steps=3000, lr=3e-3, batch=128, noise=0.5)
    S = mds.solver_for(base)
    cold, warm = [], []
    for q in held:
        S.P["b"].copy_(S.dev(q["b"]))
        c = S.ipm_solve()
        w = ws.solve(S, q["b"])
        assert c["status"] == w["status"] == "converged"
        cold.append(c["iters"])
        warm.append(w["warm_iters"] if not w["fallback"] else 2 * c["iters"])
    say(f"  cold {np.mean(cold):.2f} warm {np.mean(warm):.2f} iterations")
    assert np.mean(warm) <= np.mean(cold) - 0.5

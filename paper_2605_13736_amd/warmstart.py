"""Learned warm start of the IPM: a perceptron maps the constraint right-hand
side b of a problem family (same matrices, objective and bounds) to a
proposed start (x_d, y) and initial barrier parameter; the cold-start IPM is
the fallback.

Everything numerical runs in the library: the training data are solutions the
library's own IPM produces, the model's forward/backward/Adam steps are the
mds_mlp_* kernels, the warm start is mds_ipm_init_warm.  This module only
arranges arrays (normalisation, batching) and the host-side schedule.

Targets per training problem: x_d* and y* of the converged cold solve, and
log10 of the barrier parameter at the first cold iteration whose scaled
optimality error is <= 1e-2.  The warm start completes x_s from y and takes
bound multipliers that carry the dual residual of the proposal (see
mds_ipm_init_warm), so a proposal near the solution starts near-stationary
and a small mu0 pays off.
"""
from __future__ import annotations

import numpy as np

from . import MLP, solver_for


def mu_target(trace, level=1e-2):
    for row in trace:
        if row["E0"] <= level:
            return row["mu"]
    return trace[-1]["mu"]


def solve_family(problems, device="cuda:0", time_budget_s=None, progress=None):
    """Cold IPM solves of a list of family members on one Solver (the
    matrices are shared; only b is replaced), in order, stopping early once
    time_budget_s seconds have passed (None: no limit).  progress(count,
    seconds), when given, is called every 25 solves.  Returns X (b's),
    targets and per-problem iteration counts / solutions."""
    import time
    S = solver_for(problems[0], device=device)
    X, T, iters, xs = [], [], [], []
    t0 = time.perf_counter()
    for k, q in enumerate(problems):
        if time_budget_s is not None and X and time.perf_counter() - t0 > time_budget_s:
            break
        if progress is not None and k and k % 25 == 0:
            progress(k, time.perf_counter() - t0)
        S.P["b"].copy_(S.dev(q["b"]))
        r = S.ipm_solve()
        if r["status"] != "converged":
            continue
        nd = q["n_d"]
        x = r["x"].cpu().numpy()
        y = r["y"].cpu().numpy()
        X.append(np.asarray(q["b"]))
        T.append(np.concatenate([x[:nd], y, [np.log10(mu_target(r["trace"]))]]))
        iters.append(r["iters"])
        xs.append(x)
    return np.array(X), np.array(T), iters, xs


class WarmStart:
    """Perceptron b -> (x_d, y, log10 mu0) with per-feature normalisation; its
    linear skip path carries the affine part of the map (what a least-squares
    fit would find), the GELU layers the rest."""

    def __init__(self, m, n_d, hidden=1024, max_batch=256, device="cuda:0", seed=0):
        self.m, self.n_d = m, n_d
        self.dims = (m, hidden, hidden, n_d + m + 1)
        self.net = MLP(self.dims, max_batch, device=device)
        self.max_batch = max_batch
        self.rng = np.random.default_rng(seed)
        self.net.set_params(self._init(seed))

    def _init(self, seed):
        rng = np.random.default_rng(np.random.SeedSequence([55, seed]))
        d = self.dims
        parts = []
        for q, (a, b) in enumerate(((d[0], d[1]), (d[1], d[2]), (d[2], d[3]))):
            # the output layer of the GELU branch starts at zero, so training
            # first fits the skip path and the branch grows from there
            w = rng.standard_normal((a, b)) * np.sqrt(2.0 / a)
            parts.append(w if q < 2 else np.zeros((a, b)))
            parts.append(np.zeros(b))
        parts.append(np.zeros((d[0], d[3])))  # skip path starts at zero
        return np.concatenate([p.ravel() for p in parts]).astype(np.float32)

    def fit(self, X, T, steps=300, lr=1e-3, batch=64, noise=0.0):
        """Adam on minibatches of the normalised data; noise > 0 adds
        N(0, noise^2) to the normalised inputs of every minibatch (for the
        linear part the same as a ridge penalty, for the branch a smoothing)."""
        self.xm, self.xs = X.mean(0), X.std(0) + 1e-12
        self.tm, self.ts = T.mean(0), T.std(0) + 1e-12
        Xn = ((X - self.xm) / self.xs).astype(np.float32)
        Tn = ((T - self.tm) / self.ts).astype(np.float32)
        n = len(Xn)
        batch = min(batch, n, self.max_batch)
        losses = []
        for s in range(steps):
            idx = self.rng.choice(n, batch, replace=False)
            xb = Xn[idx]
            if noise > 0.0:
                xb = xb + (noise * self.rng.standard_normal(xb.shape)).astype(np.float32)
            losses.append(self.net.train_step(xb, Tn[idx], lr))
        return losses

    def predict(self, b, precision="bf16"):
        Xn = ((np.atleast_2d(b) - self.xm) / self.xs).astype(np.float32)
        Y = self.net.forward(Xn, precision=precision).cpu().numpy().astype(np.float64)
        Y = Y * self.ts + self.tm
        nd, m = self.n_d, self.m
        mu0 = float(np.clip(10.0 ** Y[0, nd + m], 1e-8, 0.1))
        return Y[0, :nd], Y[0, nd:nd + m], mu0

    def solve(self, S, b, precision="bf16"):
        """Warm-started IPM on Solver S for right-hand side b; falls back to
        the cold start when the warm run does not converge."""
        S.P["b"].copy_(S.dev(b))
        xd0, y0, mu0 = self.predict(b, precision)
        r = S.ipm_solve_warm(xd0, y0, mu0)
        r["fallback"] = False
        r["warm_iters"] = r["iters"]
        if r["status"] != "converged":
            c = S.ipm_solve()
            c["fallback"] = True
            c["warm_iters"] = r["iters"]
            return c
        return r

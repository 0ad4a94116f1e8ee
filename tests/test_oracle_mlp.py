"""Pins of the FP64 warm-start MLP reference and of the oracle's warm start."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp


def test_gelu_special_values():
    # GELU(0) = 0, GELU'(0) = Phi(0) = 1/2, GELU(x) - GELU(-x) = x (Phi(x) + Phi(-x) = 1)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, rtol=0, atol=1e-14)
    # tails: identity for large positive, zero for large negative
    assert abs(mlp.gelu(np.array([12.0]))[0] - 12.0) < 1e-15 * 12
    assert abs(mlp.gelu(np.array([-12.0]))[0]) < 1e-30
    # Phi(1) from the textbook value 0.8413447460685429
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_gelu_grad_matches_finite_differences():
    z = np.linspace(-4, 4, 33)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=0, atol=1e-9)


def test_loss_gradient_matches_finite_differences():
    dims = (3, 5, 4, 2)
    rng = np.random.default_rng(0)
    p = mlp.init_params(dims, 1) + 0.1 * rng.standard_normal(mlp.n_params(dims))
    X = rng.standard_normal((7, 3))
    T = rng.standard_normal((7, 2))
    L, g = mlp.loss_and_grad(p, dims, X, T)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (mlp.loss_and_grad(p + e, dims, X, T)[0] - mlp.loss_and_grad(p - e, dims, X, T)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    assert L == pytest.approx(np.mean((mlp.forward(p, dims, X)[0] - T) ** 2))


def test_identity_regime_reduces_to_linear_map():
    # with large positive pre-activations GELU is the identity, so the network
    # is the affine map X W0 W1 W2 + (b0 W1 + b1) W2 + b2, plus the skip X Ws
    dims = (2, 3, 3, 2)
    W0 = np.array([[1.0, 0.5, 0.2], [0.3, 1.0, 0.4]])
    W1 = np.eye(3)
    W2 = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    b0 = np.full(3, 40.0)
    b1 = np.zeros(3)
    b2 = np.array([0.5, -0.5])
    Ws = np.array([[2.0, -1.0], [0.0, 3.0]])
    p = np.concatenate([W0.ravel(), b0, W1.ravel(), b1, W2.ravel(), b2, Ws.ravel()])
    X = np.array([[0.1, 0.2], [-0.3, 0.4]])
    Y, _ = mlp.forward(p, dims, X)
    ref = (X @ W0 + b0) @ W1 @ W2 + b2 + X @ Ws
    assert np.allclose(Y, ref, rtol=1e-14, atol=1e-12)


def test_adam_first_step_is_signed_lr():
    # m_hat = g, v_hat = g^2 after one step: update = lr g / (|g| + eps)
    g = np.array([3.0, -0.25, 1e-3])
    p0 = np.zeros(3)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_oracle_warm_start_from_solution_converges_to_it():
    prob = synth.config_problem(synth.IPM_N192)
    P = oracle.Problem(prob)
    cold = oracle.ipm(P)
    nd = prob["n_d"]
    warm = oracle.ipm(P, warm=dict(x_d=cold["x"][:nd], y=cold["y"], mu0=1e-6))
    assert cold["status"] == warm["status"] == "converged"
    assert np.abs(warm["x"] - cold["x"]).max() <= 1e-5
    assert warm["iters"] <= cold["iters"]


def test_oracle_warm_start_point_definition():
    # one IPM iteration cap: the trace's first row reports mu0; theta of the
    # completed start point follows from x_s = -(g + J_s' y0) / w pushed into [-1, 1]
    prob = synth.make_problem(4, 12, 3, 2, cfg=900, p=0)
    P = oracle.Problem(prob)
    xd0 = np.array([0.2, -0.3, 0.0, 0.95])
    y0 = np.array([0.5, -1.0, 2.0])
    r = oracle.ipm(P, warm=dict(x_d=xd0, y=y0, mu0=0.01), max_iter=1)
    assert r["trace"][0]["mu"] <= 0.01
    jty = np.zeros(prob["n_s"])
    for i in range(prob["m"]):
        for a in range(prob["rp"][i], prob["rp"][i + 1]):
            jty[prob["ci"][a]] += prob["v"][a] * y0[i]
    xs = -(prob["g"] + jty) / prob["w"]
    x = np.clip(np.concatenate([xd0, xs]), -1 + 1e-2, 1 - 1e-2)
    Jx = prob["Jd"] @ x[:4]
    for i in range(prob["m"]):
        for a in range(prob["rp"][i], prob["rp"][i + 1]):
            Jx[i] += prob["v"][a] * x[4 + prob["ci"][a]]
    theta = np.abs(Jx - prob["b"]).sum()
    assert r["trace"][0]["theta"] == pytest.approx(theta, rel=1e-12)


def test_oracle_warm_start_multipliers_carry_dual_residual():
    # start point (no iteration): z_l = mu0/(x-l) + max(r, 0), z_u = mu0/(u-x)
    # + max(-r, 0) with r = grad f(x) + J'y0, so that z_l - z_u - mu0/(x-l)
    # + mu0/(u-x) is the stationarity residual of the start
    prob = synth.make_problem(4, 12, 3, 2, cfg=900, p=0)
    P = oracle.Problem(prob)
    xd0 = np.array([0.2, -0.3, 0.0, 0.95])
    y0 = np.array([0.5, -1.0, 2.0])
    mu0 = 0.01
    st = oracle.ipm(P, warm=dict(x_d=xd0, y=y0, mu0=mu0), max_iter=0)
    x = st["x"]
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    H = np.asarray(prob["H"], dtype=np.float64).reshape(nd, nd, order="F")
    Jd = np.asarray(prob["Jd"], dtype=np.float64).reshape(m, nd, order="F")
    Js = np.zeros((m, ns))
    for i in range(m):
        for a in range(prob["rp"][i], prob["rp"][i + 1]):
            Js[i, prob["ci"][a]] = prob["v"][a]
    grad = np.concatenate([H @ x[:nd] + prob["c"], prob["w"] * x[nd:] + prob["g"]])
    r = grad + np.concatenate([Jd.T @ y0, Js.T @ y0])
    sl, su = x - prob["xl"], prob["xu"] - x
    assert np.allclose(st["zl"], mu0 / sl + np.maximum(r, 0.0), rtol=1e-12, atol=1e-14)
    assert np.allclose(st["zu"], mu0 / su + np.maximum(-r, 0.0), rtol=1e-12, atol=1e-14)
    assert np.array_equal(st["y"], y0)


def test_oracle_warm_start_from_solution_saves_iterations():
    # from the converged primal-dual point with a small barrier parameter the
    # near-stationary start needs several iterations fewer than the cold start
    prob = synth.config_problem(synth.IPM_N192)
    P = oracle.Problem(prob)
    cold = oracle.ipm(P)
    nd = prob["n_d"]
    warm = oracle.ipm(P, warm=dict(x_d=cold["x"][:nd], y=cold["y"], mu0=1e-4))
    assert warm["status"] == "converged"
    assert warm["iters"] <= cold["iters"] - 3
    assert np.abs(warm["x"] - cold["x"]).max() <= 1e-5

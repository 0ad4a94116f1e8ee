"""Plain-definition helpers for the tests (numpy only).

These build the *uncondensed* objects the paper defines (the Newton/KKT
matrix of eq. (linsys4x4) restricted to equality constraints) so that the
oracle's condensed path can be checked against them.  Nothing here is used by
the oracle or by the GPU library.
"""
from __future__ import annotations

import numpy as np


def dense_js(prob):
    m, ns = prob["m"], prob["n_s"]
    J = np.zeros((m, ns))
    rp, ci, v = prob["rp"], prob["ci"], prob["v"]
    for i in range(m):
        for a in range(rp[i], rp[i + 1]):
            J[i, ci[a]] += v[a]
    return J


def full_kkt(prob, sigma_d, dsbase, dw=0.0, dc=0.0, dcv=None):
    """K = [[H+diag(sigma_d)+dw I, 0, Jd'], [0, diag(dsbase)+dw I, Js'],
    [Jd, Js, -dc I - diag(dcv)]] with unknown order [x_d, x_s, y]."""
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    n = nd + ns
    K = np.zeros((n + m, n + m))
    H = np.asarray(prob["H"]).reshape(nd, nd)
    K[:nd, :nd] = H + np.diag(np.asarray(sigma_d, dtype=float) + dw)
    K[nd:n, nd:n] = np.diag(np.asarray(dsbase, dtype=float) + dw)
    Jd = np.asarray(prob["Jd"]).reshape(m, nd)
    Js = dense_js(prob)
    K[n:, :nd] = Jd
    K[:nd, n:] = Jd.T
    K[n:, nd:n] = Js
    K[nd:n, n:] = Js.T
    K[n:, n:] = -dc * np.eye(m)
    if dcv is not None:
        K[n:, n:] -= np.diag(np.asarray(dcv, dtype=float))
    return K


def perm_from_ipiv(ipiv):
    """Position -> original index after applying the interchanges in order."""
    N = len(ipiv)
    p = np.arange(N)
    k = 0
    while k < N:
        if ipiv[k] > 0:
            kp = ipiv[k] - 1
            p[[k, kp]] = p[[kp, k]]
            k += 1
        else:
            kp = -ipiv[k] - 1
            p[[k + 1, kp]] = p[[kp, k + 1]]
            k += 2
    return p


def block_d(ipiv, dd, ds):
    N = len(ipiv)
    D = np.diag(np.asarray(dd, dtype=float))
    k = 0
    while k < N:
        if ipiv[k] < 0:
            D[k + 1, k] = D[k, k + 1] = ds[k]
            k += 2
        else:
            k += 1
    return D


def sign_counts(eigs, tol=0.0):
    return (int((eigs > tol).sum()), int((np.abs(eigs) <= tol).sum()), int((eigs < -tol).sum()))

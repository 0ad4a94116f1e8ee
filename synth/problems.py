"""Seeded synthetic mixed dense-sparse problems.

This module holds the input recipe only: random draws and the assembly of the
problem data (H, c, w, g, J_d, J_s, b, bounds).  It contains none of the
interior-point arithmetic; both the CPU oracle and the GPU library are fed
from it.

Recipe (the paper's workloads, the HiOp mini app and Kron-reduced ACOPF
grids, are not available; these draws stand in for them):

* objective 0.5 x_d'H x_d + c'x_d + sum_i (0.5 w_i x_s,i^2 + g_i x_s,i);
  H = Q Q'/n_d + S with Q, c ~ N(0,1); S = U diag(lam) U' with lam ~ U[-1,1]
  and U Haar-orthogonal (QR of a Gaussian with the sign of diag(R) fixed);
  w ~ U[0.1, 10]; g ~ N(0,1);
* equality constraints J_d x_d + J_s x_s = b: J_s has r distinct columns per
  row drawn uniformly without replacement (sorted), N(0,1) values; J_d is
  N(0,1)/sqrt(n_d); b = J_s x0_s + J_d x0_d with x0 ~ U[-0.5, 0.5];
* bounds [-1, 1] on every variable;
* optional inequality rows (eq. (ineq) of the paper): the last m_I rows of J
  become hl <= (J x) <= hu around the row value at x0, hl = (J x0) - a,
  hu = (J x0) + c with a, c ~ U[0.05, 0.5]; a quarter of the rows keep only
  the lower bound, a quarter only the upper one (so x0 is strictly feasible
  and some bounds bind at the solution).

* optional coupling blocks of the sparse Hessian (assumption A2 in its
  general form): the sparse variables split into consecutive blocks of
  1 .. sblk variables (sizes uniform), each block B B'/s + 0.01 I with
  B ~ N(0,1) (s x s), added to diag(w).

Draw order inside one ``SeedSequence([cfg, p])`` stream:
x0_d, x0_s, Q, lam, G (for U), c, w, g, J_s pattern, J_s values, J_d, and
then (only when m_I > 0) a, c and the side selector of the inequality rows.
The coupling blocks come from a stream of their own, ``SeedSequence([cfg,
p, 5])``: sizes, then the B of each block in order.
"""
from __future__ import annotations

import numpy as np

# named workloads: (n_d, n_s, m, nnz per row of J_s); the key also seeds the
# workload's random stream
IPM_N192, OPF_N4096, LARGE_N16384 = 0, 1, 2
CONFIGS = {
    IPM_N192: dict(n_d=64, n_s=2000, m=128, r=4),            # whole FP64 IPM, N = 192
    OPF_N4096: dict(n_d=1024, n_s=200000, m=3072, r=6),      # OPF-scale step, N = 4096
    LARGE_N16384: dict(n_d=4096, n_s=1000000, m=12288, r=8), # large condensed system
}


def _rng(cfg: int, p: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(p)]))


def _haar(rng, n):
    G = rng.standard_normal((n, n))
    Qm, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Qm * d[None, :]


def _pattern(rng, m, n_s, r):
    """r distinct sorted column indices per row (rejection of repeated rows)."""
    r = min(r, n_s)
    if m == 0 or r == 0:
        return np.zeros((m, 0), dtype=np.int64)
    cols = rng.integers(0, n_s, size=(m, r))
    cols.sort(axis=1)
    for i in range(m):
        row = cols[i]
        while r > 1 and np.any(row[1:] == row[:-1]):
            row = np.sort(rng.integers(0, n_s, size=r))
        cols[i] = row
    return cols


def make_problem(n_d: int, n_s: int, m: int, r: int, cfg: int = 0, p: int = 0,
                 h_scale: str = "n_d", s_scale: float = 1.0, m_I: int = 0,
                 sblk: int = 0) -> dict:
    """One seeded problem.  h_scale='n_d' divides Q Q' by n_d (and J_d by
    sqrt(n_d)); '64' uses the literal constant 64 for both.  s_scale widens the
    eigenvalue range of S to U[-s_scale, s_scale] (a more nonconvex variant
    used to exercise the inertia correction).  m_I: number of inequality rows
    (the last m_I of the m rows).  sblk > 0: coupling blocks of at most sblk
    sparse variables (keys bp, Wb)."""
    rng = _rng(cfg, p)
    x0_d = rng.uniform(-0.5, 0.5, n_d)
    x0_s = rng.uniform(-0.5, 0.5, n_s)
    Q = rng.standard_normal((n_d, n_d))
    lam = rng.uniform(-1.0, 1.0, n_d) * s_scale
    U = _haar(rng, n_d) if n_d > 0 else np.zeros((0, 0))
    c = rng.standard_normal(n_d)
    w = rng.uniform(0.1, 10.0, n_s)
    g = rng.standard_normal(n_s)
    cols = _pattern(rng, m, n_s, r)
    rr = cols.shape[1]
    vals = rng.standard_normal(m * rr)
    scale = float(max(n_d, 1)) if h_scale == "n_d" else 64.0
    Jd = rng.standard_normal((m, n_d)) / np.sqrt(scale)
    S = (U * lam[None, :]) @ U.T if n_d > 0 else np.zeros((0, 0))
    S = 0.5 * (S + S.T)
    H = Q @ Q.T / scale + S
    H = 0.5 * (H + H.T)
    rp = (np.arange(m + 1) * rr).astype(np.int32)
    ci = cols.reshape(-1).astype(np.int32)
    # b = J_s x0_s + J_d x0_d, evaluated once here and stored
    bs = np.zeros(m)
    if m and rr:
        bs = (vals.reshape(m, rr) * x0_s[cols]).sum(axis=1)
    b = np.asarray(bs + (Jd @ x0_d if n_d else 0.0), dtype=np.float64)
    n = n_d + n_s
    if not 0 <= m_I <= m:
        raise ValueError("m_I must lie in [0, m]")
    hl, hu = np.zeros(0), np.zeros(0)
    if m_I > 0:
        lo_w = rng.uniform(0.05, 0.5, m_I)
        up_w = rng.uniform(0.05, 0.5, m_I)
        side = rng.integers(0, 4, m_I)   # 0: lower only, 1: upper only, else both
        hx0 = b[m - m_I:]
        hl = np.where(side == 1, -np.inf, hx0 - lo_w)
        hu = np.where(side == 0, np.inf, hx0 + up_w)
    out = dict(n_d=n_d, n_s=n_s, m=m, r=rr, H=np.asfortranarray(H), c=c, w=w, g=g,
               Jd=np.asfortranarray(Jd), rp=rp, ci=ci, v=vals, b=b,
               xl=-np.ones(n), xu=np.ones(n), x0=np.concatenate([x0_d, x0_s]),
               m_I=m_I, hl=hl, hu=hu)
    if sblk > 0 and n_s > 0:
        out.update(sparse_blocks(n_s, sblk, cfg, p))
    return out


def sparse_blocks(n_s: int, sblk: int, cfg: int, p: int) -> dict:
    """Coupling blocks over n_s sparse variables: bp (block starts) and Wb
    (each block B B'/s + 0.01 I, column-major, exactly symmetric)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg), int(p), 5]))
    sizes = []
    left = n_s
    while left > 0:
        sz = min(int(rng.integers(1, sblk + 1)), left)
        sizes.append(sz)
        left -= sz
    bp = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    parts = []
    for sz in sizes:
        B = rng.standard_normal((sz, sz))
        Wb = B @ B.T / sz + 0.01 * np.eye(sz)
        Wb = 0.5 * (Wb + Wb.T)
        parts.append(Wb.reshape(-1, order="F"))
    return dict(bp=bp, Wb=np.concatenate(parts))


def config_problem(cfg: int, p: int = 0, **kw) -> dict:
    c = CONFIGS[cfg]
    return make_problem(c["n_d"], c["n_s"], c["m"], c["r"], cfg=cfg, p=p, **kw)


def batch_sizes(p: int, cfg: int = 3):
    """Sizes of batched scenario problem p: N = 4*U{64..512}, n_d = N/4,
    m = 3N/4, n_s = 50N, 4 nonzeros per row of J_s."""
    rng = np.random.default_rng(np.random.SeedSequence([cfg, p, 1]))
    N = 4 * int(rng.integers(64, 513))
    return dict(n_d=N // 4, n_s=50 * N, m=3 * N // 4, r=4, N=N)


def kkt_state(prob: dict, seed: int, log_range=(-8.0, 8.0)) -> dict:
    """A Newton system at a synthetic late-barrier state: Sigma_d and
    D_s = w + Sigma_s drawn log-uniform over 10^log_range, right-hand sides
    N(0,1)."""
    rng = np.random.default_rng(np.random.SeedSequence([99, seed]))
    lo, hi = log_range
    sigma_d = 10.0 ** rng.uniform(lo, hi, prob["n_d"])
    dsbase = 10.0 ** rng.uniform(lo, hi, prob["n_s"])
    return dict(sigma_d=sigma_d, dsbase=dsbase,
                r_d=rng.standard_normal(prob["n_d"]),
                r_s=rng.standard_normal(prob["n_s"]),
                r_y=rng.standard_normal(prob["m"]))


def interior_iterate(prob: dict, seed: int) -> dict:
    """A random strictly interior primal-dual point (x in (-0.9, 0.9),
    y ~ N(0,1), bound multipliers log-uniform in [1e-3, 10]) and mu."""
    rng = np.random.default_rng(np.random.SeedSequence([77, seed]))
    n = prob["n_d"] + prob["n_s"]
    return dict(x=rng.uniform(-0.9, 0.9, n), y=rng.standard_normal(prob["m"]),
                zl=10.0 ** rng.uniform(-3, 1, n), zu=10.0 ** rng.uniform(-3, 1, n),
                mu=float(10.0 ** rng.uniform(-6, -1)))


def family_member(prob: dict, p: int, cfg: int = 4) -> dict:
    """Problem p of the warm-start family around prob: the same matrices,
    objective and bounds, and the constraint right-hand side perturbed entry
    by entry, b = b0 * (1 + 0.1 xi) with xi ~ N(0, 1) drawn from the seed
    (cfg, p, 3) and b0 = prob's b."""
    rng = np.random.default_rng(np.random.SeedSequence([cfg, p, 3]))
    b0 = np.asarray(prob["b"], dtype=np.float64)
    q = dict(prob)
    q["b"] = b0 * (1.0 + 0.1 * rng.standard_normal(len(b0)))
    return q


def nlp_terms(prob: dict, cfg: int, p: int, q_scale: float = 0.3, e_scale: float = 1.0,
              q_per_row: int = 2) -> dict:
    """Nonlinear terms of the separable NLP test family on a problem dict:
    Q (m x n_d): each row gets q_per_row quadratic coefficients U[-q_scale,
    q_scale] on distinct random dense variables (rows r, sum_j Q_rj x_d,j^2);
    e (n_s) ~ U[0, e_scale]: objective terms e_k (exp(x_s,k) - x_s,k).  Drawn
    from SeedSequence([cfg, p, 7]); the problem's own draws are untouched.
    The equality rows' b is shifted by Q's terms at the generating point x0,
    so x0 stays feasible for them."""
    rng = np.random.default_rng(np.random.SeedSequence([int(cfg), int(p), 7]))
    nd, ns, m = prob["n_d"], prob["n_s"], prob["m"]
    Q = np.zeros((m, nd))
    if nd > 0:
        k = min(q_per_row, nd)
        for r in range(m):
            cols = rng.choice(nd, size=k, replace=False)
            Q[r, cols] = rng.uniform(-q_scale, q_scale, k)
    e = rng.uniform(0.0, e_scale, ns)
    x0d = prob["x0"][:nd]
    b = np.asarray(prob["b"], dtype=np.float64).copy()
    mE = m - int(prob.get("m_I", 0))
    b[:mE] = b[:mE] + (Q[:mE] @ (x0d * x0d) if nd else 0.0)
    q = dict(prob)
    q["b"] = b
    q["Q"] = np.asfortranarray(Q)
    q["e"] = e
    return q

"""Plain FP64 CPU oracle (ctypes wrapper around ``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; it is used by the test suite, by the smoke check and by the
CPU-baseline leg of the benchmark.  The C sources (``mds_oracle.c``) are plain
loops in double precision built with ``-ffp-contract=off``; see that file for
the passages of the paper each function follows.

All arrays are numpy float64 / int32, column-major for dense matrices.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "mds_oracle.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no BLAS, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class OrqProblem(C.Structure):
    _fields_ = [("n_d", C.c_int32), ("n_s", C.c_int32), ("m", C.c_int32),
                ("H", _dp), ("c", _dp), ("w", _dp), ("g", _dp), ("Jd", _dp),
                ("rp", _ip), ("ci", _ip), ("v", _dp), ("b", _dp),
                ("xl", _dp), ("xu", _dp), ("m_I", C.c_int32), ("hl", _dp), ("hu", _dp),
                ("nblk", C.c_int32), ("bp", _ip), ("Wb", _dp)]


class OrFactor(C.Structure):
    _fields_ = [("N", C.c_int32), ("dw", C.c_double), ("dc", C.c_double),
                ("L", _dp), ("dd", _dp), ("ds", _dp), ("ipiv", _ip), ("inv_d", _dp),
                ("lblk", _dp), ("inertia", C.c_int32 * 3), ("info", C.c_int32), ("trials", C.c_int32),
                ("dcv", _dp), ("sig_h", _dp)]


class OrIpmOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("mu0", C.c_double), ("max_iter", C.c_int32),
                ("refine_steps", C.c_int32), ("dw_max", C.c_double)]


class OrIpmTrace(C.Structure):
    _fields_ = [("mu", C.c_double), ("E0", C.c_double), ("theta", C.c_double),
                ("phi", C.c_double), ("alpha_pr", C.c_double), ("alpha_du", C.c_double),
                ("dw", C.c_double), ("dc", C.c_double), ("inertia", C.c_int32 * 3),
                ("trials", C.c_int32), ("backtracks", C.c_int32), ("soc", C.c_int32),
                ("resto", C.c_int32), ("pad", C.c_int32)]


class OrNlpStats(C.Structure):
    _fields_ = [("soc_trials", C.c_int32), ("soc_accepted", C.c_int32),
                ("resto_iters", C.c_int32), ("resto_calls", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER(OrqProblem)
        F = C.POINTER(OrFactor)
        L.or_condense.argtypes = [P, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_condense_dcv.argtypes = [P, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.or_rhs_condense.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.or_backsub.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.or_blk_words.argtypes = [P]
        L.or_blk_words.restype = C.c_int64
        L.or_bk.argtypes = [C.c_int32, _dp, _ip, _dp, _dp, _ip]
        L.or_bk.restype = C.c_int
        L.or_inertia.argtypes = [C.c_int32, _ip, _dp, _dp, _ip]
        L.or_bk_partial.argtypes = [C.c_int32, _dp, _ip, _dp, _dp, C.c_int32]
        L.or_bk_partial.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int32]
        L.or_ldl_solve.argtypes = [C.c_int32, _dp, _ip, _dp, _dp, _dp]
        L.or_ldl_solve.restype = C.c_int
        L.or_kkt_matvec.argtypes = [P, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp,
                                    _dp, _dp, _dp]
        L.or_kkt_norm_inf.argtypes = [P, _dp, _dp, C.c_double, C.c_double]
        L.or_kkt_norm_inf.restype = C.c_double
        L.or_kkt_matvec_dcv.argtypes = [P, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp,
                                        _dp, _dp, _dp, _dp]
        L.or_kkt_norm_inf_dcv.argtypes = [P, _dp, _dp, C.c_double, C.c_double, _dp]
        L.or_kkt_norm_inf_dcv.restype = C.c_double
        L.or_ineq_dcv.argtypes = [P, _dp, C.c_double, _dp]
        L.or_newton_direction.argtypes = [P, _dp, _dp, _dp, _dp, C.c_double, C.c_int32, _dp,
                                          _dp, _dp, _dp]
        L.or_newton_direction.restype = C.c_int
        L.or_factor_set_slack.argtypes = [F, _dp]
        L.or_factor_new.argtypes = [P]
        L.or_factor_new.restype = F
        L.or_factor_free.argtypes = [F]
        L.or_factor_once.argtypes = [P, _dp, _dp, C.c_double, C.c_double, F]
        L.or_factor_inertia.argtypes = [P, _dp, _dp, C.c_double, _dp, C.c_double, F]
        L.or_factor_inertia.restype = C.c_int
        L.or_newton_solve.argtypes = [P, F, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_newton_solve.restype = C.c_int
        L.or_newton_refine.argtypes = [P, F, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                       C.c_int32, C.c_double, _dp]
        L.or_newton_refine.restype = C.c_int
        L.or_sigma_rhs.argtypes = [P, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.or_ftb.argtypes = [C.c_int64, _dp, _dp, C.c_double]
        L.or_ftb.restype = C.c_double
        L.or_opt_error.argtypes = [P, _dp, _dp, _dp, _dp, C.c_double, _dp]
        L.or_opt_error.restype = C.c_double
        for nm in ("or_objective", "or_theta"):
            getattr(L, nm).argtypes = [P, _dp]
            getattr(L, nm).restype = C.c_double
        L.or_barrier.argtypes = [P, _dp, C.c_double]
        L.or_barrier.restype = C.c_double
        L.or_ipm.argtypes = [P, C.POINTER(OrIpmOpts), _dp, _dp, _dp, _dp, _ip,
                             C.POINTER(OrIpmTrace)]
        L.or_ipm.restype = C.c_int
        L.or_ipm_warm.argtypes = [P, C.POINTER(OrIpmOpts), _dp, _dp, C.c_double, _dp, _dp, _dp,
                                  _dp, _ip, C.POINTER(OrIpmTrace)]
        L.or_ipm_warm.restype = C.c_int
        L.or_nlp_test_ipm.argtypes = [P, _dp, _dp, C.POINTER(OrIpmOpts), C.c_int32, _dp, _dp,
                                      _dp, _dp, _ip, C.POINTER(OrIpmTrace),
                                      C.POINTER(OrNlpStats)]
        L.or_nlp_test_ipm.restype = C.c_int
        L.or_nlp_test_eval.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_nlp_test_eval.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """Holds contiguous copies of a problem dict and the C struct that views them."""

    def __init__(self, p: dict):
        self.n_d, self.n_s, self.m = int(p["n_d"]), int(p["n_s"]), int(p["m"])
        self.H = _f64(np.asarray(p["H"]).reshape(-1, order="F"))
        self.c = _f64(p["c"])
        self.w = _f64(p["w"])
        self.g = _f64(p["g"])
        self.Jd = _f64(np.asarray(p["Jd"]).reshape(-1, order="F"))
        self.rp = np.ascontiguousarray(p["rp"], dtype=np.int32)
        self.ci = np.ascontiguousarray(p["ci"], dtype=np.int32)
        self.v = _f64(p["v"])
        self.b = _f64(p["b"])
        self.xl = _f64(p["xl"])
        self.xu = _f64(p["xu"])
        # inequality rows (eq. (ineq)): the last m_I rows, bounds hl <= J x <= hu
        self.m_I = int(p.get("m_I", 0))
        self.hl = _f64(p.get("hl", np.zeros(0)))
        self.hu = _f64(p.get("hu", np.zeros(0)))
        assert len(self.hl) == len(self.hu) == self.m_I <= self.m
        # coupling blocks of the sparse Hessian (assumption A2, general form):
        # bp splits 0..n_s into consecutive blocks, Wb holds them column-major
        self.bp = np.ascontiguousarray(p.get("bp", np.zeros(0)), dtype=np.int32)
        self.Wb = _f64(p.get("Wb", np.zeros(0)))
        self.nblk = max(len(self.bp) - 1, 0)
        if self.nblk:
            sz = np.diff(self.bp)
            assert self.bp[0] == 0 and self.bp[-1] == self.n_s and np.all(sz > 0)
            assert len(self.Wb) == int(np.sum(sz.astype(np.int64) ** 2))
        self._keep = [np.zeros(1)]
        self.s = OrqProblem(self.n_d, self.n_s, self.m, *[_d(self._nz(a)) for a in (
            self.H, self.c, self.w, self.g, self.Jd)], _i(self._nzi(self.rp)),
            _i(self._nzi(self.ci)), _d(self._nz(self.v)), _d(self._nz(self.b)),
            _d(self._nz(self.xl)), _d(self._nz(self.xu)), self.m_I, _d(self._nz(self.hl)),
            _d(self._nz(self.hu)), self.nblk, _i(self._nzi(self.bp)), _d(self._nz(self.Wb)))

    def _nz(self, a):
        if a.size == 0:
            a = np.zeros(1)
            self._keep.append(a)
        return a

    def _nzi(self, a):
        if a.size == 0:
            a = np.zeros(1, dtype=np.int32)
            self._keep.append(a)
        return a

    @property
    def N(self):
        return self.n_d + self.m

    @property
    def nx(self):
        """Length of the IPM's primal vector: variables, then inequality slacks."""
        return self.n_d + self.n_s + self.m_I

    @property
    def ptr(self):
        return C.byref(self.s)


def _buf(n, dtype=np.float64):
    return np.zeros(max(int(n), 1), dtype=dtype)


def blk_words(P: Problem):
    return int(lib().or_blk_words(P.ptr))


def condense(P: Problem, sigma_d, dsbase, dw=0.0, dc=0.0, dcv=None, with_blocks=False):
    """Condensed matrix M (N x N, full symmetric) and inv_d: 1/(dsbase+dw)
    without coupling blocks, 1/Delta of the blocks' L Delta L' with them.
    dcv (m, optional): per-row diagonal subtracted from M22 after dc.
    with_blocks: also return the blocks' unit lower factors (Wb's layout)."""
    N = P.N
    M = _buf(N * N)
    inv_d = _buf(P.n_s)
    lb = _buf(blk_words(P))
    sd = _d(_f64(sigma_d) if P.n_d else _buf(1))
    db = _d(_f64(dsbase) if P.n_s else _buf(1))
    if dcv is None:
        lib().or_condense(P.ptr, sd, db, dw, dc, _d(M), _d(inv_d), _d(lb))
    else:
        dv = _f64(dcv) if P.m else _buf(1)
        lib().or_condense_dcv(P.ptr, sd, db, dw, dc, _d(dv), _d(M), _d(inv_d), _d(lb))
    out = (M[:N * N].reshape((N, N), order="F"), inv_d[:P.n_s])
    return out + (lb[:blk_words(P)],) if with_blocks else out


def rhs_condense(P: Problem, inv_d, r_s, r_y, lblk=None):
    out = _buf(P.m)
    lb = _f64(lblk) if lblk is not None and len(lblk) else _buf(1)
    lib().or_rhs_condense(P.ptr, _d(_f64(inv_d) if P.n_s else _buf(1)), _d(lb),
                          _d(_f64(r_s) if P.n_s else _buf(1)),
                          _d(_f64(r_y) if P.m else _buf(1)), _d(out))
    return out[:P.m]


def backsub(P: Problem, inv_d, r_s, dy, lblk=None):
    out = _buf(P.n_s)
    lb = _f64(lblk) if lblk is not None and len(lblk) else _buf(1)
    lib().or_backsub(P.ptr, _d(_f64(inv_d) if P.n_s else _buf(1)), _d(lb),
                     _d(_f64(r_s) if P.n_s else _buf(1)), _d(_f64(dy) if P.m else _buf(1)),
                     _d(out))
    return out[:P.n_s]


def bk(A):
    """Bunch-Kaufman LDL' of symmetric A (lower triangle read).

    Returns (L, dd, ds, ipiv, info, kind): L unit lower in standard form
    (P'AP = L D L'), D's diagonal and sub-diagonal, LAPACK 1-based ipiv.
    """
    A = np.asarray(A, dtype=np.float64)
    N = A.shape[0]
    W = _buf(N * N)
    W[:N * N] = A.reshape(-1, order="F")
    ipiv = _buf(N, np.int32)
    dd, ds = _buf(N), _buf(N)
    kind = _buf(N, np.int32)
    info = lib().or_bk(N, _d(W), _i(ipiv), _d(dd), _d(ds), _i(kind))
    L = np.tril(W[:N * N].reshape((N, N), order="F"), -1) + np.eye(N)
    return L, dd[:N], ds[:N], ipiv[:N], info, kind[:N]


def set_threads(n: int):
    """Threads of the oracle's elimination (bit-identical results for any n)."""
    lib().or_set_threads(int(n))


def bk_partial(A, kstop):
    """The first kstop pivot columns of the Bunch-Kaufman elimination of A
    (a timing sample); A is overwritten (column-major float64, N x N)."""
    N = A.shape[0]
    ipiv = _buf(N, np.int32)
    dd, ds = _buf(N), _buf(N)
    return lib().or_bk_partial(N, _d(A.reshape(-1, order="F")), _i(ipiv), _d(dd), _d(ds),
                               int(kstop)), ipiv


def inertia(ipiv, dd, ds):
    N = len(ipiv)
    out = np.zeros(3, dtype=np.int32)
    lib().or_inertia(N, _i(np.ascontiguousarray(ipiv, dtype=np.int32) if N else _buf(1, np.int32)),
                     _d(_f64(dd) if N else _buf(1)), _d(_f64(ds) if N else _buf(1)), _i(out))
    return tuple(int(v) for v in out)


def ldl_solve(L, ipiv, dd, ds, b):
    N = len(ipiv)
    x = _f64(np.array(b, dtype=np.float64, copy=True))
    Lf = _f64(np.asarray(L).reshape(-1, order="F"))
    st = lib().or_ldl_solve(N, _d(Lf), _i(np.ascontiguousarray(ipiv, dtype=np.int32)),
                            _d(_f64(dd)), _d(_f64(ds)), _d(x))
    return x, st


def kkt_matvec(P: Problem, sigma_d, dsbase, dw, dc, dx_d, dx_s, dy, dcv=None):
    o_d, o_s, o_y = _buf(P.n_d), _buf(P.n_s), _buf(P.m)
    a = [_f64(v) if len(v) else _buf(1) for v in (sigma_d, dsbase, dx_d, dx_s, dy)]
    if dcv is None:
        lib().or_kkt_matvec(P.ptr, _d(a[0]), _d(a[1]), dw, dc, _d(a[2]), _d(a[3]), _d(a[4]),
                            _d(o_d), _d(o_s), _d(o_y))
    else:
        dv = _f64(dcv) if P.m else _buf(1)
        lib().or_kkt_matvec_dcv(P.ptr, _d(a[0]), _d(a[1]), dw, dc, _d(dv), _d(a[2]), _d(a[3]),
                                _d(a[4]), _d(o_d), _d(o_s), _d(o_y))
    return o_d[:P.n_d], o_s[:P.n_s], o_y[:P.m]


def kkt_norm_inf(P: Problem, sigma_d, dsbase, dw, dc, dcv=None):
    a = [_f64(v) if len(v) else _buf(1) for v in (sigma_d, dsbase)]
    if dcv is None:
        return lib().or_kkt_norm_inf(P.ptr, _d(a[0]), _d(a[1]), dw, dc)
    dv = _f64(dcv) if P.m else _buf(1)
    return lib().or_kkt_norm_inf_dcv(P.ptr, _d(a[0]), _d(a[1]), dw, dc, _d(dv))


def ineq_dcv(P: Problem, sig_h, dw):
    """(4,4) diagonal of the inequality rows: 0 on equality rows, 1/(sig_h + dw)."""
    out = _buf(P.m)
    sh = _f64(sig_h) if len(sig_h) else _buf(1)
    lib().or_ineq_dcv(P.ptr, _d(sh), dw, _d(out))
    return out[:P.m]


class Factor:
    """A factored, regularised Newton system owned by the oracle."""

    def __init__(self, P: Problem, sig_h=None):
        """sig_h (m_I, optional): slack barrier diagonal; every condensation
        then forms the inequality rows' (4,4) block 1 / (sig_h + dw)."""
        self.P = P
        self.p = lib().or_factor_new(P.ptr)
        if sig_h is not None:
            self._sh = _f64(sig_h) if len(sig_h) else _buf(1)
            lib().or_factor_set_slack(self.p, _d(self._sh))

    @property
    def dcv(self):
        m = self.P.m
        return np.ctypeslib.as_array(self.s.dcv, shape=(max(m, 1),))[:m].copy()

    def __del__(self):
        try:
            lib().or_factor_free(self.p)
        except Exception:
            pass

    @property
    def s(self):
        return self.p.contents

    def once(self, sigma_d, dsbase, dw=0.0, dc=0.0):
        self._sd, self._db = _f64(sigma_d) if len(sigma_d) else _buf(1), \
            _f64(dsbase) if len(dsbase) else _buf(1)
        lib().or_factor_once(self.P.ptr, _d(self._sd), _d(self._db), dw, dc, self.p)
        return self

    def correct(self, sigma_d, dsbase, mu, dw_last=0.0, dw_max=1e20):
        """Inertia-correction loop.  Returns (status, dw_last_new)."""
        self._sd, self._db = _f64(sigma_d) if len(sigma_d) else _buf(1), \
            _f64(dsbase) if len(dsbase) else _buf(1)
        dl = np.array([dw_last], dtype=np.float64)
        st = lib().or_factor_inertia(self.P.ptr, _d(self._sd), _d(self._db), mu, _d(dl),
                                     dw_max, self.p)
        return st, float(dl[0])

    @property
    def inertia(self):
        return tuple(int(v) for v in self.s.inertia)

    @property
    def ipiv(self):
        N = self.s.N
        return np.ctypeslib.as_array(self.s.ipiv, shape=(max(N, 1),))[:N].copy()

    @property
    def dd(self):
        N = self.s.N
        return np.ctypeslib.as_array(self.s.dd, shape=(max(N, 1),))[:N].copy()

    @property
    def ds(self):
        N = self.s.N
        return np.ctypeslib.as_array(self.s.ds, shape=(max(N, 1),))[:N].copy()

    @property
    def L(self):
        N = self.s.N
        a = np.ctypeslib.as_array(self.s.L, shape=(max(N * N, 1),))[:N * N].copy()
        return np.tril(a.reshape((N, N), order="F"), -1) + np.eye(N)

    def solve(self, r_d, r_s, r_y):
        P = self.P
        o = [_buf(P.n_d), _buf(P.n_s), _buf(P.m)]
        a = [_f64(v) if len(v) else _buf(1) for v in (r_d, r_s, r_y)]
        st = lib().or_newton_solve(P.ptr, self.p, _d(a[0]), _d(a[1]), _d(a[2]),
                                   _d(o[0]), _d(o[1]), _d(o[2]))
        return o[0][:P.n_d], o[1][:P.n_s], o[2][:P.m], st

    def refine(self, r_d, r_s, r_y, max_steps=5, eta_tol=1e-14):
        P = self.P
        o = [_buf(P.n_d), _buf(P.n_s), _buf(P.m)]
        a = [_f64(v) if len(v) else _buf(1) for v in (r_d, r_s, r_y)]
        eta = np.zeros(1)
        steps = lib().or_newton_refine(P.ptr, self.p, _d(self._sd), _d(self._db), _d(a[0]),
                                       _d(a[1]), _d(a[2]), _d(o[0]), _d(o[1]), _d(o[2]),
                                       max_steps, eta_tol, _d(eta))
        return o[0][:P.n_d], o[1][:P.n_s], o[2][:P.m], steps, float(eta[0])


def sigma_rhs(P: Problem, x, y, zl, zu, mu):
    n = P.nx
    sig, rx, ry = _buf(n), _buf(n), _buf(P.m)
    a = [_f64(v) if len(v) else _buf(1) for v in (x, y, zl, zu)]
    lib().or_sigma_rhs(P.ptr, _d(a[0]), _d(a[1]), _d(a[2]), _d(a[3]), mu, _d(sig), _d(rx),
                       _d(ry))
    return sig[:n], rx[:n], ry[:P.m]


def newton_direction(P: Problem, x, y, zl, zu, mu, refine_steps=2):
    """One IPM iteration's Newton direction at (x, y, zl, zu) (correction loop
    from delta_w^last = 0).  Returns (status, dx (nx), dy (m), dzl, dzu)."""
    n = P.nx
    dx, dzl, dzu, dy = _buf(n), _buf(n), _buf(n), _buf(P.m)
    a = [_f64(v) if len(v) else _buf(1) for v in (x, y, zl, zu)]
    st = lib().or_newton_direction(P.ptr, _d(a[0]), _d(a[1]), _d(a[2]), _d(a[3]), mu,
                                   int(refine_steps), _d(dx), _d(dy), _d(dzl), _d(dzu))
    return st, dx[:n], dy[:P.m], dzl[:n], dzu[:n]


def ftb(v, dv, tau):
    v, dv = _f64(v), _f64(dv)
    return lib().or_ftb(len(v), _d(v if len(v) else _buf(1)), _d(dv if len(dv) else _buf(1)),
                        tau)


def opt_error(P: Problem, x, y, zl, zu, mu):
    parts = np.zeros(6)
    a = [_f64(v) if len(v) else _buf(1) for v in (x, y, zl, zu)]
    e = lib().or_opt_error(P.ptr, _d(a[0]), _d(a[1]), _d(a[2]), _d(a[3]), mu, _d(parts))
    return e, parts


def objective(P: Problem, x):
    return lib().or_objective(P.ptr, _d(_f64(x)))


def barrier(P: Problem, x, mu):
    return lib().or_barrier(P.ptr, _d(_f64(x)), mu)


def theta(P: Problem, x):
    return lib().or_theta(P.ptr, _d(_f64(x)))


IPM_STATUS = {4: "converged", 5: "ls_fail", 6: "maxiter", 2: "inertia_fail", 7: "nonfinite"}


def ipm(P: Problem, tol=1e-8, mu0=0.1, max_iter=200, refine_steps=2, dw_max=1e20,
        warm=None):
    """Whole filter line-search IPM.  warm: None (cold start) or a dict with
    x_d, y and mu0 (warm start).  Returns dict with x, y, zl, zu, status,
    iters, trace."""
    n = P.nx
    x, zl, zu, y = _buf(n), _buf(n), _buf(n), _buf(P.m)
    it = np.zeros(1, dtype=np.int32)
    opts = OrIpmOpts(tol, mu0, max_iter, refine_steps, dw_max)
    tr = (OrIpmTrace * (max_iter + 1))()
    if warm is None:
        st = lib().or_ipm(P.ptr, C.byref(opts), _d(x), _d(y), _d(zl), _d(zu), _i(it), tr)
    else:
        xd0 = _f64(warm["x_d"]) if P.n_d else _buf(1)
        y0 = _f64(warm["y"]) if P.m else _buf(1)
        st = lib().or_ipm_warm(P.ptr, C.byref(opts), _d(xd0), _d(y0), float(warm["mu0"]),
                               _d(x), _d(y), _d(zl), _d(zu), _i(it), tr)
    if st == 8:
        raise ValueError("the warm start is defined for a diagonal sparse Hessian block only")
    iters = int(it[0])
    rows = []
    for k in range(min(iters + 1, max_iter)):
        t = tr[k]
        rows.append(dict(mu=t.mu, E0=t.E0, theta=t.theta, phi=t.phi, alpha_pr=t.alpha_pr,
                         alpha_du=t.alpha_du, dw=t.dw, dc=t.dc, inertia=tuple(t.inertia),
                         trials=t.trials, backtracks=t.backtracks))
    return dict(x=x[:n], y=y[:P.m], zl=zl[:n], zu=zu[:n], status=IPM_STATUS.get(st, st),
                code=st, iters=iters, trace=rows)


# ---- general NLP (external model): the separable nonlinear test family ----
NLP_STATUS = dict(IPM_STATUS)
NLP_STATUS[9] = "hessian_negative"


def _trace_rows(tr, iters, max_iter):
    rows = []
    for k in range(min(iters + 1, max_iter)):
        t = tr[k]
        rows.append(dict(mu=t.mu, E0=t.E0, theta=t.theta, phi=t.phi, alpha_pr=t.alpha_pr,
                         alpha_du=t.alpha_du, dw=t.dw, dc=t.dc, inertia=tuple(t.inertia),
                         trials=t.trials, backtracks=t.backtracks, soc=t.soc, resto=t.resto))
    return rows


def nlp_test_ipm(P: Problem, Q, e, tol=1e-8, mu0=0.1, max_iter=200, refine_steps=2,
                 dw_max=1e20, force_resto=-1):
    """The general-NLP IPM (second-order correction, restoration) on the
    separable nonlinear test family built on P's data: Q (m x n_d quadratic
    coefficients of the rows), e (n_s exponential weights of the objective)."""
    n = P.nx
    Qf = _f64(np.asarray(Q, dtype=np.float64).reshape(-1, order="F"))
    ef = _f64(e)
    x, zl, zu, y = _buf(n), _buf(n), _buf(n), _buf(P.m)
    it = np.zeros(1, dtype=np.int32)
    opts = OrIpmOpts(tol, mu0, max_iter, refine_steps, dw_max)
    tr = (OrIpmTrace * (max_iter + 1))()
    stats = OrNlpStats()
    st = lib().or_nlp_test_ipm(P.ptr, _d(Qf if Qf.size else _buf(1)), _d(ef if ef.size else _buf(1)),
                               C.byref(opts), int(force_resto), _d(x), _d(y), _d(zl), _d(zu),
                               _i(it), tr, C.byref(stats))
    iters = int(it[0])
    return dict(x=x[:n], y=y[:P.m], zl=zl[:n], zu=zu[:n], status=NLP_STATUS.get(st, st),
                code=st, iters=iters, trace=_trace_rows(tr, iters, max_iter),
                soc_trials=stats.soc_trials, soc_accepted=stats.soc_accepted,
                resto_iters=stats.resto_iters, resto_calls=stats.resto_calls)


def nlp_test_eval(P: Problem, Q, e, x, y):
    """The test family's model at (x, y): f, gradient, constraints, Jacobian
    values (J_d, J_s) and the Lagrangian Hessian (H, w)."""
    nd, ns, m = P.n_d, P.n_s, P.m
    Qf = _f64(np.asarray(Q, dtype=np.float64).reshape(-1, order="F"))
    g, c = _buf(nd + ns), _buf(m)
    Jd, v = _buf(m * nd), _buf(len(P.v))
    H, w = _buf(nd * nd), _buf(ns)
    f = lib().or_nlp_test_eval(P.ptr, _d(Qf if Qf.size else _buf(1)),
                               _d(_f64(e) if len(e) else _buf(1)), _d(_f64(x)),
                               _d(_f64(y) if m else _buf(1)), _d(g), _d(c), _d(Jd), _d(v),
                               _d(H), _d(w))
    return dict(f=f, g=g[:nd + ns], c=c[:m], Jd=Jd[:m * nd].reshape((m, nd), order="F"),
                v=v[:len(P.v)], H=H[:nd * nd].reshape((nd, nd), order="F"), w=w[:ns])

"""Python binding of libmdsipm (the gfx950 HIP library declared in include/mdsipm.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  Importing this
package does not need a GPU; creating a :class:`Solver` does, and it raises
if the built library or a ROCm device is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdsipm.so")

# status codes (include/mdsipm.h)
MDS_OK = 0
MDS_ZERO_PIVOT = 1
MDS_INERTIA_FAIL = 2
MDS_REFINE_NOCONV = 3
MDS_IPM_CONVERGED = 4
MDS_IPM_LS_FAIL = 5
MDS_IPM_MAXITER = 6
MDS_IPM_NONFINITE = 7
MDS_DEBUG_COOP_ABORT = 1
MDS_DEBUG_FORCE_RESTO = 2
STATUS_NAMES = {4: "converged", 5: "ls_fail", 6: "maxiter", 2: "inertia_fail", 7: "nonfinite"}

_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Dims(C.Structure):
    _fields_ = [("n_d", C.c_int32), ("n_s", C.c_int32), ("m", C.c_int32), ("m_I", C.c_int32),
                ("nnz_s", C.c_int64)]


class Options(C.Structure):
    _fields_ = [("nb", C.c_int32), ("panel", C.c_int32), ("precision", C.c_int32),
                ("panel_threads", C.c_int32), ("nlp", C.c_int32), ("sblk_max", C.c_int32),
                ("lookahead", C.c_int32), ("reserved", C.c_int32 * 1)]


# panel kernels: automatic choice, panel in device memory, register-resident
# (one workgroup), register-resident over several cooperating workgroups,
# whole matrix in one workgroup's LDS (unblocked, N <= 199)
PANELS = {"auto": 0, "mem": 1, "reg": 2, "coop": 3, "lds": 4}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
# look-ahead of the cooperative factorization (next panel beside the
# trailing update): automatic (N >= 8192), on, off
LOOKAHEAD = {"auto": 0, "on": 1, "off": 2}


class Problem(C.Structure):
    _fields_ = [("H", _vp), ("c", _vp), ("w", _vp), ("g", _vp), ("J_d", _vp),
                ("Js_rowptr", _vp), ("Js_col", _vp), ("Js_val", _vp), ("b", _vp),
                ("xl", _vp), ("xu", _vp), ("hl", _vp), ("hu", _vp)]


class Inertia(C.Structure):
    _fields_ = [("npos", C.c_int32), ("nzero", C.c_int32), ("nneg", C.c_int32),
                ("n2x2", C.c_int32), ("info", C.c_int32)]


class Reg(C.Structure):
    _fields_ = [("delta_w_last", C.c_double), ("delta_w", C.c_double), ("delta_c", C.c_double),
                ("delta_w_max", C.c_double), ("trials", C.c_int32), ("pad", C.c_int32)]


class RefineInfo(C.Structure):
    _fields_ = [("eta", C.c_double), ("rel_residual", C.c_double), ("steps", C.c_int32),
                ("pad", C.c_int32)]


class Iterate(C.Structure):
    _fields_ = [("x", _vp), ("y", _vp), ("zl", _vp), ("zu", _vp), ("mu", C.c_double),
                ("tau", C.c_double), ("iter", C.c_int32), ("pad", C.c_int32)]


class IpmOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("mu0", C.c_double), ("max_iter", C.c_int32),
                ("refine_steps", C.c_int32), ("dw_max", C.c_double), ("gmres_max", C.c_int32),
                ("pad", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("mu", C.c_double), ("E0", C.c_double), ("theta", C.c_double),
                ("phi", C.c_double), ("alpha_pr", C.c_double), ("alpha_du", C.c_double),
                ("delta_w", C.c_double), ("delta_c", C.c_double), ("eta", C.c_double),
                ("inertia", C.c_int32 * 3), ("trials", C.c_int32), ("solves", C.c_int32),
                ("backtracks", C.c_int32), ("status", C.c_int32), ("fallback", C.c_int32),
                ("nlp_event", C.c_int32)]


# general-NLP model objects (mds_nlp_model): device pointers throughout
NLP_OBJECTIVE = C.CFUNCTYPE(C.c_int, _vp, _vp, _dp)
NLP_VEC = C.CFUNCTYPE(C.c_int, _vp, _vp, _vp)
NLP_JAC = C.CFUNCTYPE(C.c_int, _vp, _vp, _vp, _vp)
NLP_HESS = C.CFUNCTYPE(C.c_int, _vp, _vp, _vp, _vp, _vp)


class NlpModel(C.Structure):
    _fields_ = [("ctx", _vp), ("objective", NLP_OBJECTIVE), ("gradient", NLP_VEC),
                ("constraints", NLP_VEC), ("jacobian", NLP_JAC), ("hessian", NLP_HESS)]


class PanelStats(C.Structure):
    _fields_ = [("panels", C.c_int32), ("coop_steps", C.c_int32), ("coop_second", C.c_int32),
                ("n2x2", C.c_int32)]


class NlpStats(C.Structure):
    _fields_ = [("soc_trials", C.c_int32), ("soc_accepted", C.c_int32),
                ("resto_calls", C.c_int32), ("resto_iters", C.c_int32)]


class Fallbacks(C.Structure):
    _fields_ = [("coop_aborts", C.c_int64), ("fp64_refactors", C.c_int64)]


T_CLASSES = ("condense", "panel", "trailing", "solve", "permute", "panel_tail", "factor", "near")


class Info(C.Structure):
    _fields_ = [("nb", C.c_int32), ("min_width", C.c_int32), ("panel", C.c_int32),
                ("precision", C.c_int32), ("panel_threads", C.c_int32),
                ("lookahead_cus", C.c_int32), ("workspace_bytes", C.c_int64)]


class BatchProblem(C.Structure):
    _fields_ = [("n_d", C.c_int32), ("n_s", C.c_int32), ("m", C.c_int32), ("pad", C.c_int32),
                ("nnz_s", C.c_int64), ("H", _vp), ("J_d", _vp), ("Js_rowptr", _vp),
                ("Js_col", _vp), ("Js_val", _vp), ("sigma_d", _vp), ("dsbase", _vp),
                ("r_d", _vp), ("r_s", _vp), ("r_y", _vp), ("dx_d", _vp), ("dx_s", _vp),
                ("dy", _vp)]


class BatchResult(C.Structure):
    _fields_ = [("npos", C.c_int32), ("nzero", C.c_int32), ("nneg", C.c_int32),
                ("trials", C.c_int32), ("delta_w", C.c_double), ("delta_c", C.c_double),
                ("t_start", C.c_int64), ("t_done", C.c_int64), ("status", C.c_int32),
                ("slot", C.c_int32), ("refine_steps", C.c_int32), ("pad", C.c_int32),
                ("residual", C.c_double)]


class BatchOpts(C.Structure):
    _fields_ = [("nb", C.c_int32), ("grid", C.c_int32), ("use_graph", C.c_int32),
                ("precision", C.c_int32), ("refine_steps", C.c_int32),
                ("ipm_max_iter", C.c_int32), ("reserved", C.c_int32 * 2)]


class BatchIpmProblem(C.Structure):
    _fields_ = [("c", _vp), ("w", _vp), ("g", _vp), ("b", _vp), ("xl", _vp), ("xu", _vp),
                ("x", _vp), ("y", _vp), ("zl", _vp), ("zu", _vp)]


class BatchIpmResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("mu", C.c_double),
                ("E0", C.c_double), ("t_start", C.c_int64), ("t_done", C.c_int64),
                ("slot", C.c_int32), ("factorizations", C.c_int32)]


class BatchIpmIter(C.Structure):
    _fields_ = [("mu", C.c_double), ("alpha_pr", C.c_double), ("delta_w", C.c_double),
                ("inertia", C.c_int32 * 3), ("trials", C.c_int32), ("backtracks", C.c_int32),
                ("pad", C.c_int32)]


class Timings(C.Structure):
    _fields_ = [("ms", C.c_double * len(T_CLASSES)), ("launches", C.c_int64 * len(T_CLASSES))]


# exported functions: name -> (restype, argtypes)
SIGNATURES = {
    "mds_workspace_bytes": (C.c_size_t, [C.POINTER(Dims), C.POINTER(Options)]),
    "mds_create": (C.c_int, [C.POINTER(_vp), C.POINTER(Dims), C.POINTER(Options), _vp, _vp,
                             C.c_size_t]),
    "mds_destroy": (None, [_vp]),
    "mds_set_problem": (C.c_int, [_vp, C.POINTER(Problem)]),
    "mds_condense": (C.c_int, [_vp, _vp, _vp, C.c_double, C.c_double]),
    "mds_factor_inertia": (C.c_int, [_vp, C.POINTER(Reg), C.c_double, C.POINTER(Inertia)]),
    "mds_solve": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mds_refine": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, C.c_double,
                             C.POINTER(RefineInfo)]),
    "mds_sigma_rhs": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double, _vp, _vp, _vp]),
    "mds_ftb": (C.c_int, [_vp, C.c_int64, _vp, _vp, C.c_double, _dp]),
    "mds_ftb_noalloc": (C.c_int, [C.c_int64, _vp, _vp, C.c_double, _vp, _vp]),
    "mds_ftb_noalloc_scratch_bytes": (C.c_size_t, []),
    "mds_opt_error": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double, _dp, _dp]),
    "mds_merit": (C.c_int, [_vp, _vp, C.c_double, _dp, _dp, _dp]),
    "mds_ipm_init": (C.c_int, [_vp, C.POINTER(Iterate), C.POINTER(IpmOpts)]),
    "mds_ipm_step": (C.c_int, [_vp, C.POINTER(Iterate), C.POINTER(StepInfo)]),
    "mds_ipm_init_warm": (C.c_int, [_vp, C.POINTER(Iterate), C.POINTER(IpmOpts), _vp, _vp,
                                    C.c_double]),
    "mds_ipm_solve": (C.c_int, [_vp, C.POINTER(Iterate), C.POINTER(IpmOpts),
                                C.POINTER(StepInfo), C.c_int32, _ip]),
    "mds_get_matrix": (C.c_int, [_vp, _dp]),
    "mds_get_factor": (C.c_int, [_vp, _dp, _dp, _dp, _ip]),
    "mds_set_m22_diag": (C.c_int, [_vp, _vp]),
    "mds_set_sparse_blocks": (C.c_int, [_vp, C.c_int32, _ip, _vp]),
    "mds_set_nlp": (C.c_int, [_vp, C.POINTER(NlpModel)]),
    "mds_get_panel_stats": (C.c_int, [_vp, C.POINTER(PanelStats)]),
    "mds_probe_exchange": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _dp]),
    "mds_get_nlp_stats": (C.c_int, [_vp, C.POINTER(NlpStats)]),
    "mds_sep_model_workspace_bytes": (C.c_size_t, []),
    "mds_sep_model_create": (C.c_int, [C.POINTER(_vp), C.POINTER(Dims), C.POINTER(Problem), _vp,
                                       _vp, _vp, _vp, C.c_size_t, C.POINTER(NlpModel)]),
    "mds_sep_model_destroy": (None, [_vp]),
    "mds_get_pivots": (C.c_int, [_vp, _ip]),
    "mds_get_inv_ds": (C.c_int, [_vp, _dp]),
    "mds_get_info": (C.c_int, [_vp, C.POINTER(Info)]),
    "mds_set_timing": (C.c_int, [_vp, C.c_int]),
    "mds_get_fallbacks": (C.c_int, [_vp, C.POINTER(Fallbacks)]),
    "mds_set_debug": (C.c_int, [_vp, C.c_int32]),
    "mds_get_timings": (C.c_int, [_vp, C.POINTER(Timings)]),
    "mds_batch_workspace_bytes": (C.c_size_t, [C.POINTER(BatchProblem), C.c_int32,
                                               C.POINTER(BatchOpts)]),
    "mds_batch_create": (C.c_int, [C.POINTER(_vp), C.POINTER(BatchProblem), C.c_int32,
                                   C.POINTER(BatchOpts), _vp, _vp, C.c_size_t]),
    "mds_batch_run": (C.c_int, [_vp, C.c_double, C.POINTER(BatchResult)]),
    "mds_batch_autotune": (C.c_int, [_vp, C.c_double, C.POINTER(BatchOpts)]),
    "mds_batch_ipm": (C.c_int, [_vp, C.POINTER(BatchIpmProblem), C.POINTER(IpmOpts),
                                C.POINTER(BatchIpmResult), C.POINTER(BatchIpmIter)]),
    "mds_batch_get_config": (C.c_int, [_vp, C.POINTER(BatchOpts)]),
    "mds_batch_destroy": (None, [_vp]),
    "mds_batch_last_error": (C.c_char_p, [_vp]),
    "mds_mlp_workspace_bytes": (C.c_size_t, [_ip, C.c_int32]),
    "mds_mlp_create": (C.c_int, [C.POINTER(_vp), _ip, C.c_int32, _vp, _vp, C.c_size_t]),
    "mds_mlp_destroy": (None, [_vp]),
    "mds_mlp_param_count": (C.c_int32, [_vp]),
    "mds_mlp_set_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "mds_mlp_get_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "mds_mlp_get_grad": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "mds_mlp_forward": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, _vp]),
    "mds_mlp_train_step": (C.c_int, [_vp, _vp, _vp, C.c_int32, C.c_float, _dp]),
    "mds_status_string": (C.c_char_p, [C.c_int]),
    "mds_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def lib():
    """Load libmdsipm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2605_13736_amd/build.py`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class MdsError(RuntimeError):
    pass


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(
        t.data_ptr() if t is not None else 0)


class Solver:
    """One library handle bound to a device, a stream and a workspace tensor."""

    def __init__(self, n_d: int, n_s: int, m: int, nnz_s: int, nb: int = 0,
                 device: str = "cuda:0", stream=None, panel: str = "auto",
                 precision: str = "fp64", panel_threads: int = 0, m_I: int = 0,
                 sblk_max: int = 0, nlp: bool = False, lookahead: str = "auto"):
        torch = _torch()
        if not torch.cuda.is_available():
            raise MdsError("no ROCm GPU visible: the mdsipm library has no CPU path")
        self.torch = torch
        self.device = torch.device(device)
        self.dims = Dims(n_d, n_s, m, m_I, nnz_s)
        if precision not in PRECISIONS:
            raise MdsError(f"precision must be one of {sorted(PRECISIONS)}")
        self.precision = precision
        if panel not in PANELS:
            raise MdsError("panel must be one of " + ", ".join(PANELS))
        if lookahead not in LOOKAHEAD:
            raise MdsError("lookahead must be one of " + ", ".join(LOOKAHEAD))
        self.opts = Options(nb, PANELS[panel], PRECISIONS[precision],
                            int(panel_threads), int(bool(nlp)), int(sblk_max),
                            LOOKAHEAD[lookahead])
        self.n_d, self.n_s, self.m, self.m_I = n_d, n_s, m, m_I
        self.N, self.n = n_d + m, n_d + n_s
        self.nx = self.n + m_I  # IPM primal vector: variables, then inequality slacks
        L = lib()
        nbytes = L.mds_workspace_bytes(C.byref(self.dims), C.byref(self.opts))
        if nbytes == 0:
            raise MdsError("invalid dimensions")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            aligned = (base + 255) & ~255
            h = C.c_void_p()
            st = L.mds_create(C.byref(h), C.byref(self.dims), C.byref(self.opts),
                              C.c_void_p(self.stream.cuda_stream), C.c_void_p(aligned), nbytes)
        if st != 0:
            raise MdsError(f"mds_create: {L.mds_status_string(st).decode()}")
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            lib().mds_destroy(self.h)
            self.h = None
        if getattr(self, "_sep", None):
            lib().mds_sep_model_destroy(self._sep)
            self._sep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers --------------------------------------------------------
    def _check(self, st, what, ok=(0,)):
        if st < 0:
            msg = lib().mds_last_error(self.h).decode()
            raise MdsError(f"{what}: {lib().mds_status_string(st).decode()} ({msg})")
        return st

    def dev(self, a, dtype=None):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            return a.to(self.device).contiguous()
        arr = np.asarray(a)
        if dtype is None:
            dtype = torch.int32 if arr.dtype.kind in "iu" else torch.float64
        return torch.as_tensor(np.ascontiguousarray(arr)).to(device=self.device,
                                                            dtype=dtype).contiguous()

    def empty(self, n):
        return self.torch.empty(max(int(n), 0), dtype=self.torch.float64, device=self.device)

    # ---- problem --------------------------------------------------------
    def set_problem(self, prob: dict):
        torch = self.torch
        nd, m = self.n_d, self.m
        T = dict(
            H=self.dev(np.asarray(prob["H"], dtype=np.float64).reshape(-1, order="F")),
            c=self.dev(np.asarray(prob["c"], dtype=np.float64)),
            w=self.dev(np.asarray(prob["w"], dtype=np.float64)),
            g=self.dev(np.asarray(prob["g"], dtype=np.float64)),
            J_d=self.dev(np.asarray(prob["Jd"], dtype=np.float64).reshape(-1, order="F")),
            Js_rowptr=self.dev(np.asarray(prob["rp"], dtype=np.int32), torch.int32),
            Js_col=self.dev(np.asarray(prob["ci"], dtype=np.int32), torch.int32),
            Js_val=self.dev(np.asarray(prob["v"], dtype=np.float64)),
            b=self.dev(np.asarray(prob["b"], dtype=np.float64)),
            xl=self.dev(np.asarray(prob["xl"], dtype=np.float64)),
            xu=self.dev(np.asarray(prob["xu"], dtype=np.float64)),
            hl=self.dev(np.asarray(prob.get("hl", np.zeros(0)), dtype=np.float64)),
            hu=self.dev(np.asarray(prob.get("hu", np.zeros(0)), dtype=np.float64)),
        )
        assert T["hl"].numel() == self.m_I and T["hu"].numel() == self.m_I
        assert T["H"].numel() == nd * nd and T["J_d"].numel() == m * nd
        self.P = T
        self.cp = Problem(*[_ptr(T[k]) for k, _ in Problem._fields_])
        st = lib().mds_set_problem(self.h, C.byref(self.cp))
        self._check(st, "mds_set_problem")
        return st

    # ---- Newton-step hot path -------------------------------------------
    def condense(self, sigma_d, dsbase, delta_w=0.0, delta_c=0.0):
        sd, db = self.dev(sigma_d), self.dev(dsbase)
        self._keep["sigma_d"], self._keep["dsbase"] = sd, db
        st = lib().mds_condense(self.h, _ptr(sd), _ptr(db), float(delta_w), float(delta_c))
        return self._check(st, "mds_condense")

    def set_m22_diag(self, dcv=None):
        """Per-row diagonal subtracted from M22 (None clears); kept alive here."""
        if dcv is None:
            self._keep.pop("dcv", None)
            st = lib().mds_set_m22_diag(self.h, None)
        else:
            t = self.dev(dcv)
            st = lib().mds_set_m22_diag(self.h, _ptr(t))
            if st == 0:
                self._keep["dcv"] = t
        return self._check(st, "mds_set_m22_diag")

    def set_sparse_blocks(self, bp=None, Wb=None):
        """Coupling blocks of the sparse Hessian (bp: block starts, n_blocks + 1
        entries; Wb: the blocks column-major, one after another); None clears."""
        if bp is None:
            self._keep.pop("Wb", None)
            return self._check(lib().mds_set_sparse_blocks(self.h, 0, None, None),
                               "mds_set_sparse_blocks")
        bp = np.ascontiguousarray(bp, dtype=np.int32)
        t = self.dev(np.asarray(Wb, dtype=np.float64))
        st = lib().mds_set_sparse_blocks(self.h, len(bp) - 1, bp.ctypes.data_as(_ip), _ptr(t))
        if st == 0:
            self._keep["Wb"] = t
        return self._check(st, "mds_set_sparse_blocks")

    # ---- general NLP ------------------------------------------------------
    def set_nlp(self, model=None, keep=None):
        """NLP mode with the model objects `model` (an NlpModel whose
        callbacks and context outlive the mode; `keep` is held with it), or
        back to the quadratic problem (None)."""
        if model is None:
            st = lib().mds_set_nlp(self.h, None)
            self._check(st, "mds_set_nlp")
            self._keep.pop("nlp", None)
            return st
        st = lib().mds_set_nlp(self.h, C.byref(model))
        self._check(st, "mds_set_nlp")
        self._keep["nlp"] = (model, keep)
        return st

    def set_sep_model(self, Q, e):
        """NLP mode with the library's separable nonlinear model on the
        attached problem's data: rows gain sum_j Q_rj x_d,j^2 (Q: m x n_d) and
        the objective sum_k e_k (exp(x_s,k) - x_s,k)."""
        torch = self.torch
        Qd = self.dev(np.asarray(Q, dtype=np.float64).reshape(-1, order="F"))
        ed = self.dev(np.asarray(e, dtype=np.float64))
        assert Qd.numel() == self.m * self.n_d and ed.numel() == self.n_s
        L = lib()
        nbytes = L.mds_sep_model_workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (ws.data_ptr() + 255) & ~255
        model = NlpModel()
        sep = C.c_void_p()
        st = L.mds_sep_model_create(C.byref(sep), C.byref(self.dims), C.byref(self.cp), _ptr(Qd),
                                    _ptr(ed), C.c_void_p(self.stream.cuda_stream),
                                    C.c_void_p(aligned), nbytes, C.byref(model))
        if st != 0:
            raise MdsError(f"mds_sep_model_create: {L.mds_status_string(st).decode()}")
        if getattr(self, "_sep", None):
            self.set_nlp(None)
            L.mds_sep_model_destroy(self._sep)
        self._sep = sep
        return self.set_nlp(model, keep=(Qd, ed, ws))

    def nlp_stats(self):
        s = NlpStats()
        self._check(lib().mds_get_nlp_stats(self.h, C.byref(s)), "mds_get_nlp_stats")
        return dict(soc_trials=s.soc_trials, soc_accepted=s.soc_accepted,
                    resto_calls=s.resto_calls, resto_iters=s.resto_iters)

    def factor_inertia(self, mu=0.0, reg=None):
        """reg None: factor as condensed.  reg dict (delta_w_last, delta_w_max):
        run the inertia-correction loop.  Returns (status, inertia, reg)."""
        inn = Inertia()
        if reg is None:
            st = lib().mds_factor_inertia(self.h, None, float(mu), C.byref(inn))
            self._check(st, "mds_factor_inertia")
            return st, _inertia_dict(inn), None
        r = Reg(reg.get("delta_w_last", 0.0), 0.0, 0.0, reg.get("delta_w_max", 0.0), 0, 0)
        st = lib().mds_factor_inertia(self.h, C.byref(r), float(mu), C.byref(inn))
        self._check(st, "mds_factor_inertia")
        return st, _inertia_dict(inn), dict(delta_w_last=r.delta_w_last, delta_w=r.delta_w,
                                            delta_c=r.delta_c, trials=r.trials)

    def solve(self, r_d, r_s, r_y):
        a = [self.dev(v) for v in (r_d, r_s, r_y)]
        o = [self.empty(self.n_d), self.empty(self.n_s), self.empty(self.m)]
        st = lib().mds_solve(self.h, *[_ptr(t) for t in a], *[_ptr(t) for t in o])
        self._check(st, "mds_solve")
        return o

    def refine(self, r_d, r_s, r_y, max_steps=5, eta_tol=1e-14):
        a = [self.dev(v) for v in (r_d, r_s, r_y)]
        o = [self.empty(self.n_d), self.empty(self.n_s), self.empty(self.m)]
        info = RefineInfo()
        st = lib().mds_refine(self.h, *[_ptr(t) for t in a], *[_ptr(t) for t in o],
                              int(max_steps), float(eta_tol), C.byref(info))
        self._check(st, "mds_refine")
        return o, dict(status=st, eta=info.eta, rel_residual=info.rel_residual,
                       steps=info.steps)

    # ---- vector kernels -------------------------------------------------
    def sigma_rhs(self, x, y, zl, zu, mu):
        a = [self.dev(v) for v in (x, y, zl, zu)]
        sig, rx, ry = self.empty(self.nx), self.empty(self.nx), self.empty(self.m)
        st = lib().mds_sigma_rhs(self.h, *[_ptr(t) for t in a], float(mu), _ptr(sig), _ptr(rx),
                                 _ptr(ry))
        self._check(st, "mds_sigma_rhs")
        return sig, rx, ry

    def ftb(self, v, dv, tau):
        v, dv = self.dev(v), self.dev(dv)
        out = C.c_double()
        st = lib().mds_ftb(self.h, v.numel(), _ptr(v), _ptr(dv), float(tau), C.byref(out))
        self._check(st, "mds_ftb")
        return out.value

    def opt_error(self, x, y, zl, zu, mu):
        a = [self.dev(v) for v in (x, y, zl, zu)]
        E = C.c_double()
        parts = (C.c_double * 6)()
        st = lib().mds_opt_error(self.h, *[_ptr(t) for t in a], float(mu), C.byref(E), parts)
        self._check(st, "mds_opt_error")
        return E.value, list(parts)

    def merit(self, x, mu):
        x = self.dev(x)
        f, phi, th = C.c_double(), C.c_double(), C.c_double()
        st = lib().mds_merit(self.h, _ptr(x), float(mu), C.byref(f), C.byref(phi), C.byref(th))
        self._check(st, "mds_merit")
        return f.value, phi.value, th.value

    # ---- IPM ------------------------------------------------------------
    def new_iterate(self):
        it = dict(x=self.empty(self.nx), y=self.empty(self.m), zl=self.empty(self.nx),
                  zu=self.empty(self.nx))
        it["c"] = Iterate(_ptr(it["x"]), _ptr(it["y"]), _ptr(it["zl"]), _ptr(it["zu"]),
                          0.0, 0.0, 0, 0)
        return it

    def ipm_init(self, it, tol=1e-8, mu0=0.1, max_iter=200, refine_steps=2, dw_max=1e20,
                 gmres_max=0):
        self._opts = IpmOpts(tol, mu0, max_iter, refine_steps, dw_max, gmres_max, 0)
        st = lib().mds_ipm_init(self.h, C.byref(it["c"]), C.byref(self._opts))
        return self._check(st, "mds_ipm_init")

    def ipm_step(self, it):
        info = StepInfo()
        st = lib().mds_ipm_step(self.h, C.byref(it["c"]), C.byref(info))
        self._check(st, "mds_ipm_step")
        return st, _step_dict(info)

    def ipm_solve_warm(self, x_d0, y0, mu0, tol=1e-8, max_iter=200, refine_steps=2,
                       dw_max=1e20, gmres_max=0):
        """IPM from a proposed start (mds_ipm_init_warm), stepped to the end."""
        it = self.new_iterate()
        xd, yy = self.dev(x_d0), self.dev(y0)
        self._opts = IpmOpts(tol, float(mu0), max_iter, refine_steps, dw_max, gmres_max, 0)
        st = lib().mds_ipm_init_warm(self.h, C.byref(it["c"]), C.byref(self._opts), _ptr(xd),
                                     _ptr(yy), float(mu0))
        self._check(st, "mds_ipm_init_warm")
        trace = []
        while True:
            code, info = self.ipm_step(it)
            trace.append(info)
            if code != 0:
                break
        return dict(status=STATUS_NAMES.get(code, code), code=code, iters=it["c"].iter,
                    trace=trace, x=it["x"], y=it["y"], zl=it["zl"], zu=it["zu"],
                    mu=it["c"].mu)

    def ipm_solve(self, it=None, tol=1e-8, mu0=0.1, max_iter=200, refine_steps=2, dw_max=1e20,
                  gmres_max=0):
        it = it if it is not None else self.new_iterate()
        opts = IpmOpts(tol, mu0, max_iter, refine_steps, dw_max, gmres_max, 0)
        cap = max_iter + 2
        tr = (StepInfo * cap)()
        iters = C.c_int32()
        st = lib().mds_ipm_solve(self.h, C.byref(it["c"]), C.byref(opts), tr, cap,
                                 C.byref(iters))
        self._check(st, "mds_ipm_solve")
        n = min(iters.value + 1, cap)
        return dict(status=STATUS_NAMES.get(st, st), code=st, iters=iters.value,
                    trace=[_step_dict(tr[k]) for k in range(n)], x=it["x"], y=it["y"],
                    zl=it["zl"], zu=it["zu"], mu=it["c"].mu)

    def info(self):
        i = Info()
        self._check(lib().mds_get_info(self.h, C.byref(i)), "mds_get_info")
        prec = {v: k for k, v in PRECISIONS.items()}[i.precision]
        return dict(nb=i.nb, min_width=i.min_width, panel=("reg", "mem", "coop", "lds")[i.panel],
                    precision=prec, panel_threads=i.panel_threads,
                    lookahead_cus=i.lookahead_cus, workspace_bytes=i.workspace_bytes)

    def panel_stats(self):
        """Pivot statistics of the last factorization (mds_get_panel_stats)."""
        p = PanelStats()
        self._check(lib().mds_get_panel_stats(self.h, C.byref(p)), "mds_get_panel_stats")
        return dict(panels=p.panels, coop_steps=p.coop_steps, coop_second=p.coop_second,
                    n2x2=p.n2x2)

    def probe_exchange(self, P, rounds=2000, words=3):
        """Microseconds per exchange round trip of P cooperating workgroups
        (mds_probe_exchange)."""
        us = C.c_double()
        self._check(lib().mds_probe_exchange(self.h, int(P), int(rounds), int(words),
                                             C.byref(us)), "mds_probe_exchange")
        return us.value

    def fallbacks(self):
        f = Fallbacks()
        self._check(lib().mds_get_fallbacks(self.h, C.byref(f)), "mds_get_fallbacks")
        return dict(coop_aborts=int(f.coop_aborts), fp64_refactors=int(f.fp64_refactors))

    def set_debug(self, flags: int):
        self._check(lib().mds_set_debug(self.h, int(flags)), "mds_set_debug")

    # ---- timing ---------------------------------------------------------
    def set_timing(self, enable: bool):
        self._check(lib().mds_set_timing(self.h, int(bool(enable))), "mds_set_timing")

    def get_timings(self):
        t = Timings()
        self._check(lib().mds_get_timings(self.h, C.byref(t)), "mds_get_timings")
        return {name: dict(ms=t.ms[i], launches=int(t.launches[i]))
                for i, name in enumerate(T_CLASSES)}

    # ---- diagnostics ----------------------------------------------------
    def get_matrix(self):
        N = self.N
        out = np.empty(max(N * N, 1))
        st = lib().mds_get_matrix(self.h, out.ctypes.data_as(_dp))
        self._check(st, "mds_get_matrix")
        return out[:N * N].reshape((N, N), order="F")

    def get_factor(self):
        N = self.N
        L = np.empty(max(N * N, 1))
        dd, ds = np.empty(max(N, 1)), np.empty(max(N, 1))
        ipiv = np.empty(max(N, 1), dtype=np.int32)
        st = lib().mds_get_factor(self.h, L.ctypes.data_as(_dp), dd.ctypes.data_as(_dp),
                                  ds.ctypes.data_as(_dp), ipiv.ctypes.data_as(_ip))
        self._check(st, "mds_get_factor")
        Lm = L[:N * N].reshape((N, N), order="F") + np.eye(N)
        return Lm, dd[:N], ds[:N], ipiv[:N]

    def get_pivots(self):
        ipiv = np.empty(max(self.N, 1), dtype=np.int32)
        self._check(lib().mds_get_pivots(self.h, ipiv.ctypes.data_as(_ip)), "mds_get_pivots")
        return ipiv[:self.N]

    def get_inv_ds(self):
        out = np.empty(max(self.n_s, 1))
        st = lib().mds_get_inv_ds(self.h, out.ctypes.data_as(_dp))
        self._check(st, "mds_get_inv_ds")
        return out[:self.n_s]


def ftb_noalloc(v, dv, tau, alpha, stream=None):
    """Allocation-free fraction to the boundary (mds_ftb_noalloc): writes the
    step into the one-element FP64 device tensor `alpha` on `stream` (default:
    the current stream of alpha's device).  Asynchronous."""
    torch = _torch()
    for t in (v, dv, alpha):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise MdsError("ftb_noalloc takes contiguous FP64 device tensors")
    if v.numel() != dv.numel() or alpha.numel() < 1:
        raise MdsError("ftb_noalloc: v and dv differ in length, or alpha is empty")
    if stream is None:
        stream = torch.cuda.current_stream(alpha.device)
    st = lib().mds_ftb_noalloc(v.numel(), _ptr(v), _ptr(dv), float(tau), _ptr(alpha),
                               C.c_void_p(stream.cuda_stream))
    if st != 0:
        raise MdsError(f"mds_ftb_noalloc: {lib().mds_status_string(st).decode()}")


def _inertia_dict(i):
    return dict(npos=i.npos, nzero=i.nzero, nneg=i.nneg, n2x2=i.n2x2, info=i.info)


def _step_dict(s):
    return dict(mu=s.mu, E0=s.E0, theta=s.theta, phi=s.phi, alpha_pr=s.alpha_pr,
                alpha_du=s.alpha_du, dw=s.delta_w, dc=s.delta_c, eta=s.eta,
                inertia=tuple(s.inertia), trials=s.trials, solves=s.solves,
                backtracks=s.backtracks, status=s.status, fallback=s.fallback,
                nlp_event=s.nlp_event)


def solver_for(prob: dict, nb: int = 0, device: str = "cuda:0", panel: str = "auto",
               precision: str = "fp64", panel_threads: int = 0, nlp: bool = False,
               lookahead: str = "auto") -> Solver:
    """Create a Solver sized for a problem dict and attach the problem (and
    its coupling blocks of the sparse Hessian when it has them)."""
    bp = prob.get("bp")
    smax = int(np.max(np.diff(bp))) if bp is not None and len(bp) > 1 else 0
    s = Solver(prob["n_d"], prob["n_s"], prob["m"], len(prob["v"]), nb=nb, device=device,
               panel=panel, precision=precision, panel_threads=panel_threads,
               m_I=int(prob.get("m_I", 0)), sblk_max=smax, nlp=nlp, lookahead=lookahead)
    s.set_problem(prob)
    if smax:
        s.set_sparse_blocks(bp, prob["Wb"])
    return s


class Batch:
    """Many independent Newton systems solved by one persistent kernel.

    items: list of dicts with the problem arrays of a synthetic problem dict
    (H, Jd, rp, ci, v, n_d, n_s, m) plus sigma_d, dsbase, r_d, r_s, r_y."""

    def __init__(self, items, nb=0, grid=0, use_graph=True, device="cuda:0", precision="fp64",
                 refine_steps=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise MdsError("no ROCm GPU visible: the mdsipm library has no CPU path")
        self.torch, self.device = torch, torch.device(device)
        self.count = len(items)
        self._keep = []
        self.out = []
        descs = (BatchProblem * self.count)()

        def dev(a, dt=None):
            arr = np.asarray(a)
            if dt is None:
                dt = torch.int32 if arr.dtype.kind in "iu" else torch.float64
            t = torch.as_tensor(np.ascontiguousarray(arr)).to(device=self.device, dtype=dt)
            self._keep.append(t)
            return t

        for p, it in enumerate(items):
            nd, ns, m = int(it["n_d"]), int(it["n_s"]), int(it["m"])
            H = dev(np.asarray(it["H"], dtype=np.float64).reshape(-1, order="F"))
            Jd = dev(np.asarray(it["Jd"], dtype=np.float64).reshape(-1, order="F"))
            rp = dev(np.asarray(it["rp"], dtype=np.int32), torch.int32)
            ci = dev(np.asarray(it["ci"], dtype=np.int32), torch.int32)
            v = dev(np.asarray(it["v"], dtype=np.float64))
            ins = [dev(np.asarray(it[k], dtype=np.float64))
                   for k in ("sigma_d", "dsbase", "r_d", "r_s", "r_y")]
            o = [torch.empty(max(n, 0), dtype=torch.float64, device=self.device)
                 for n in (nd, ns, m)]
            self.out.append(o)
            descs[p] = BatchProblem(nd, ns, m, 0, int(len(it["v"])), _ptr(H), _ptr(Jd), _ptr(rp),
                                    _ptr(ci), _ptr(v), *[_ptr(t) for t in ins],
                                    *[_ptr(t) for t in o])
        self.descs = descs
        if precision not in ("fp64", "fp32"):
            raise MdsError("batch precision must be 'fp64' or 'fp32'")
        self.opts = BatchOpts(int(nb), int(grid), 1 if use_graph else 0, PRECISIONS[precision],
                              int(refine_steps))
        L = lib()
        nbytes = L.mds_batch_workspace_bytes(descs, self.count, C.byref(self.opts))
        if nbytes == 0:
            raise MdsError("invalid batch sizes (each problem needs 1 <= n_d + m <= 2048)")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.ws.data_ptr() + 255) & ~255
            h = C.c_void_p()
            st = L.mds_batch_create(C.byref(h), descs, self.count, C.byref(self.opts),
                                    C.c_void_p(self.stream.cuda_stream), C.c_void_p(aligned),
                                    nbytes)
        if st != 0:
            raise MdsError(f"mds_batch_create: {L.mds_status_string(st).decode()}")
        self.h = h
        self.workspace_bytes = nbytes

    def close(self):
        if getattr(self, "h", None):
            lib().mds_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, mu=0.0):
        res = (BatchResult * self.count)()
        st = lib().mds_batch_run(self.h, float(mu), res)
        if st != 0:
            raise MdsError(f"mds_batch_run: {lib().mds_status_string(st).decode()} "
                           f"({lib().mds_batch_last_error(self.h).decode()})")
        return [dict(inertia=(r.npos, r.nzero, r.nneg), trials=r.trials, delta_w=r.delta_w,
                     delta_c=r.delta_c, t_start=r.t_start, t_done=r.t_done, status=r.status,
                     slot=r.slot, refine_steps=r.refine_steps, residual=r.residual)
                for r in res]

    def autotune(self, mu=0.0):
        o = BatchOpts()
        st = lib().mds_batch_autotune(self.h, float(mu), C.byref(o))
        if st != 0:
            raise MdsError(f"mds_batch_autotune: {lib().mds_status_string(st).decode()} "
                           f"({lib().mds_batch_last_error(self.h).decode()})")
        return dict(nb=o.nb, grid=o.grid, use_graph=bool(o.use_graph),
                    precision="fp32" if o.precision == PRECISIONS["fp32"] else "fp64",
                    refine_steps=o.refine_steps)

    def config(self):
        o = BatchOpts()
        lib().mds_batch_get_config(self.h, C.byref(o))
        return dict(nb=o.nb, grid=o.grid, use_graph=bool(o.use_graph),
                    precision="fp32" if o.precision == PRECISIONS["fp32"] else "fp64",
                    refine_steps=o.refine_steps)

    def solution(self, p):
        return [t.detach().cpu().numpy() for t in self.out[p]]


class BatchIPM:
    """Whole FP64 IPMs of many independent problems in one persistent kernel
    (mds_batch_ipm).  problems: synthetic problem dicts (equality rows only)."""

    def __init__(self, problems, nb=0, grid=0, max_iter=200, device="cuda:0"):
        torch = _torch()
        if not torch.cuda.is_available():
            raise MdsError("no ROCm GPU visible: the mdsipm library has no CPU path")
        self.torch, self.device = torch, torch.device(device)
        self.count = len(problems)
        self.max_iter = int(max_iter)
        self._keep = []
        self.out = []
        descs = (BatchProblem * self.count)()
        ipm = (BatchIpmProblem * self.count)()

        def dev(a, dt=None):
            arr = np.asarray(a)
            if dt is None:
                dt = torch.int32 if arr.dtype.kind in "iu" else torch.float64
            t = torch.as_tensor(np.ascontiguousarray(arr)).to(device=self.device, dtype=dt)
            self._keep.append(t)
            return t

        for p, q in enumerate(problems):
            if int(q.get("m_I", 0)) or q.get("bp") is not None:
                raise MdsError("the batched IPM takes equality rows and a diagonal sparse Hessian")
            nd, ns, m = int(q["n_d"]), int(q["n_s"]), int(q["m"])
            H = dev(np.asarray(q["H"], dtype=np.float64).reshape(-1, order="F"))
            Jd = dev(np.asarray(q["Jd"], dtype=np.float64).reshape(-1, order="F"))
            rp = dev(np.asarray(q["rp"], dtype=np.int32), torch.int32)
            ci = dev(np.asarray(q["ci"], dtype=np.int32), torch.int32)
            v = dev(np.asarray(q["v"], dtype=np.float64))
            descs[p] = BatchProblem(nd, ns, m, 0, int(len(q["v"])), _ptr(H), _ptr(Jd), _ptr(rp),
                                    _ptr(ci), _ptr(v), *([C.c_void_p(0)] * 8))
            data = [dev(np.asarray(q[k], dtype=np.float64)) for k in ("c", "w", "g", "b", "xl", "xu")]
            o = [torch.empty(max(k, 1), dtype=torch.float64, device=self.device)
                 for k in (nd + ns, m, nd + ns, nd + ns)]
            self.out.append((o, nd + ns, m))
            ipm[p] = BatchIpmProblem(*[_ptr(t) for t in data], *[_ptr(t) for t in o])
        self.descs, self.ipm = descs, ipm
        self.opts = BatchOpts(int(nb), int(grid), 0, 0, 0, self.max_iter)
        L = lib()
        nbytes = L.mds_batch_workspace_bytes(descs, self.count, C.byref(self.opts))
        if nbytes == 0:
            raise MdsError("invalid batch sizes (each problem needs 1 <= n_d + m <= 2048)")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.ws.data_ptr() + 255) & ~255
            h = C.c_void_p()
            st = L.mds_batch_create(C.byref(h), descs, self.count, C.byref(self.opts),
                                    C.c_void_p(self.stream.cuda_stream), C.c_void_p(aligned),
                                    nbytes)
        if st != 0:
            raise MdsError(f"mds_batch_create: {L.mds_status_string(st).decode()}")
        self.h = h
        self.workspace_bytes = nbytes

    def close(self):
        if getattr(self, "h", None):
            lib().mds_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, tol=1e-8, mu0=0.1, max_iter=None, refine_steps=2, dw_max=1e20, trace=True):
        mi = self.max_iter if max_iter is None else int(max_iter)
        opts = IpmOpts(tol, mu0, mi, refine_steps, dw_max, 0, 0)
        res = (BatchIpmResult * self.count)()
        rows = self.max_iter + 1
        tr = (BatchIpmIter * (self.count * rows))() if trace else None
        st = lib().mds_batch_ipm(self.h, self.ipm, C.byref(opts), res, tr)
        if st != 0:
            raise MdsError(f"mds_batch_ipm: {lib().mds_status_string(st).decode()} "
                           f"({lib().mds_batch_last_error(self.h).decode()})")
        out = []
        for p in range(self.count):
            r = res[p]
            d = dict(status=STATUS_NAMES.get(r.status, r.status), code=r.status, iters=r.iters,
                     mu=r.mu, E0=r.E0, t_start=r.t_start, t_done=r.t_done, slot=r.slot,
                     factorizations=r.factorizations)
            if trace:
                d["trace"] = [dict(mu=tr[p * rows + k].mu, alpha_pr=tr[p * rows + k].alpha_pr,
                                   delta_w=tr[p * rows + k].delta_w,
                                   inertia=tuple(tr[p * rows + k].inertia),
                                   trials=tr[p * rows + k].trials,
                                   backtracks=tr[p * rows + k].backtracks)
                              for k in range(min(r.iters, rows))]
            out.append(d)
        return out

    def solution(self, p):
        (x, y, zl, zu), n, m = self.out[p]
        return (x[:n].cpu().numpy(), y[:m].cpu().numpy(), zl[:n].cpu().numpy(),
                zu[:n].cpu().numpy())


class MLP:
    """The warm-start perceptron (mds_mlp_*): dims = (in, h, h, out)."""

    def __init__(self, dims, max_batch, device="cuda:0"):
        torch = _torch()
        if not torch.cuda.is_available():
            raise MdsError("no ROCm GPU visible: the mdsipm library has no CPU path")
        self.torch, self.device = torch, torch.device(device)
        self.dims = (C.c_int32 * 4)(*[int(d) for d in dims])
        self.max_batch = int(max_batch)
        L = lib()
        nbytes = L.mds_mlp_workspace_bytes(self.dims, self.max_batch)
        if nbytes == 0:
            raise MdsError("invalid MLP dimensions")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.ws.data_ptr() + 255) & ~255
            h = C.c_void_p()
            st = L.mds_mlp_create(C.byref(h), self.dims, self.max_batch,
                                  C.c_void_p(self.stream.cuda_stream), C.c_void_p(aligned), nbytes)
        if st != 0:
            raise MdsError(f"mds_mlp_create: {L.mds_status_string(st).decode()}")
        self.h = h
        self.nparam = L.mds_mlp_param_count(h)

    def close(self):
        if getattr(self, "h", None):
            lib().mds_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, a):
        t = self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32))
        return t.to(self.device).contiguous()

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparam
        st = lib().mds_mlp_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)))
        if st != 0:
            raise MdsError("mds_mlp_set_params failed")

    def get_params(self):
        p = np.empty(self.nparam, dtype=np.float32)
        lib().mds_mlp_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)))
        return p

    def get_grad(self):
        p = np.empty(self.nparam, dtype=np.float32)
        lib().mds_mlp_get_grad(self.h, p.ctypes.data_as(C.POINTER(C.c_float)))
        return p

    def forward(self, X, precision="fp32"):
        Xd = X if isinstance(X, self.torch.Tensor) else self._f32(X)
        B = Xd.shape[0]
        Y = self.torch.empty((B, self.dims[3]), dtype=self.torch.float32, device=self.device)
        st = lib().mds_mlp_forward(self.h, _ptr(Xd), B, PRECISIONS[precision], _ptr(Y))
        if st != 0:
            raise MdsError(f"mds_mlp_forward: {lib().mds_status_string(st).decode()}")
        return Y

    def train_step(self, X, T, lr):
        Xd = X if isinstance(X, self.torch.Tensor) else self._f32(X)
        Td = T if isinstance(T, self.torch.Tensor) else self._f32(T)
        loss = C.c_double()
        st = lib().mds_mlp_train_step(self.h, _ptr(Xd), _ptr(Td), Xd.shape[0], float(lr),
                                      C.byref(loss))
        if st != 0:
            raise MdsError(f"mds_mlp_train_step: {lib().mds_status_string(st).decode()}")
        return loss.value

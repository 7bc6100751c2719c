"""ctypes binding of libqpg.so (declared in include/qpg.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels. The
library must have been built (``python -m paper_1912_04263_amd.build``); loading fails loudly
otherwise — there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
# QPG_LIBRARY names another build of the same library (same ABI), e.g. to compare two builds
LIB_PATH = os.environ.get("QPG_LIBRARY") or os.path.join(HERE, "libqpg.so")

QPG_OK = 0
QPG_ERR_ARG, QPG_ERR_DATA, QPG_ERR_SIZE, QPG_ERR_DEVICE, QPG_ERR_OOM, QPG_ERR_STATE = -1, -2, -3, -4, -5, -6
QPG_ERR_HOST = -7
QPG_UNSOLVED, QPG_SOLVED, QPG_MAX_ITER_REACHED, QPG_NUMERICAL_ERROR = 0, 1, 2, 3
QPG_PRIMAL_INFEASIBLE, QPG_DUAL_INFEASIBLE = 4, 5
QPG_FP64, QPG_MIXED = 0, 1
QPG_PRECOND_JACOBI, QPG_PRECOND_LEARNED = 0, 1
QPG_NET_NPARAMS = 16705
QPG_NOALLOC_SCRATCH_BYTES, QPG_NOALLOC_MAX_N = 16777216, 1864128
QPG_OP_A, QPG_OP_AT, QPG_OP_P, QPG_OP_K = 0, 1, 2, 3
QPG_KERNEL_SPMV_A, QPG_KERNEL_SPMV_B, QPG_KERNEL_PCG_UPDATE, QPG_KERNEL_PCG_DIR = 0, 1, 2, 3
QPG_KERNEL_SPMV_A_STREAM, QPG_KERNEL_SPMV_B_STREAM = 4, 5
STATUS = {0: "unsolved", 1: "solved", 2: "max_iter_reached", 3: "numerical_error", 4: "primal_infeasible",
          5: "dual_infeasible"}


class Csc(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int32),
                ("colptr", C.POINTER(C.c_int32)), ("rowidx", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class Settings(C.Structure):
    _fields_ = [("rho", C.c_double), ("sigma", C.c_double), ("alpha", C.c_double),
                ("eps_abs", C.c_double), ("eps_rel", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("rho_update_every", C.c_int32),
                ("rho_update_gate", C.c_double), ("pcg_lambda", C.c_double),
                ("pcg_eps_min", C.c_double), ("pcg_eps_fixed", C.c_double),
                ("pcg_max_iter", C.c_int32), ("pcg_rel_test", C.c_int32),
                ("scaling_iters", C.c_int32), ("precision", C.c_int32), ("precond", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("verbose", C.c_int32),
                ("precond_weights", C.POINTER(C.c_float)), ("precond_trial", C.c_int32),
                ("spmv_tile_nnz", C.c_int32), ("spmv_plain_nnz", C.c_int32),
                ("eps_prim_inf", C.c_double), ("eps_dual_inf", C.c_double), ("rho_vector", C.c_int32),
                ("pcg_eps_schedule", C.c_int32), ("speculate", C.c_int32),
                ("spmv_window_cols", C.c_int32), ("spmv_min_seg", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iter", C.c_int32), ("pcg_iter_total", C.c_int64),
                ("pcg_iter_max", C.c_int32), ("rho_updates", C.c_int32), ("obj_val", C.c_double),
                ("prim_res", C.c_double), ("dual_res", C.c_double), ("rho_final", C.c_double),
                ("setup_time", C.c_double), ("solve_time", C.c_double),
                ("precision_used", C.c_int32), ("precond_used", C.c_int32),
                ("fallback_events", C.c_int32), ("scaling_passes", C.c_int32),
                ("precond_trials", C.c_int32), ("precond_learned_chosen", C.c_int32),
                ("precond_switches", C.c_int32), ("infeas_checks", C.c_int32),
                ("spec_resumes", C.c_int32)]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)
_PF = C.POINTER(C.c_float)
_PB = C.POINTER(C.c_int8)
_lib = None

# name -> (restype, argtypes); the full exported surface of include/qpg.h
SIGNATURES = {
    "qpg_default_settings": (C.c_int, [C.POINTER(Settings)]),
    "qpg_setup": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Csc), _PD, C.POINTER(Csc), _PD, _PD,
                            C.POINTER(Settings)]),
    "qpg_solve": (C.c_int, [C.c_void_p]),
    "qpg_get_x": (C.c_int, [C.c_void_p, _PD]),
    "qpg_get_y": (C.c_int, [C.c_void_p, _PD]),
    "qpg_get_z": (C.c_int, [C.c_void_p, _PD]),
    "qpg_get_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "qpg_get_scaling": (C.c_int, [C.c_void_p, _PD, _PD, _PD]),
    "qpg_get_certificate": (C.c_int, [C.c_void_p, _PD, _PD]),
    "qpg_apply": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _PD, _PD]),
    "qpg_pcg": (C.c_int, [C.c_void_p, C.c_int32, _PD, _PD, C.c_double, C.c_int32, C.c_int32, _PD,
                          _PI, _PD]),
    "qpg_set_rho": (C.c_int, [C.c_void_p, C.c_double]),
    "qpg_time_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _PD]),
    "qpg_spmv_layout": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    "qpg_cleanup": (C.c_int, [C.c_void_p]),
    "qpg_get_kdiag": (C.c_int, [C.c_void_p, C.c_double, _PD]),
    "qpg_hutchinson": (C.c_int, [C.c_void_p, _PB, C.c_int32, C.c_double, C.c_double, C.c_int32, _PD]),
    "qpg_hutchinson_noalloc": (C.c_int, [C.c_void_p, _PB, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                         _PD]),
    "qpg_net_create": (C.c_int, [C.POINTER(C.c_void_p), _PF, C.c_uint64, C.c_int32, C.c_int32]),
    "qpg_net_get_params": (C.c_int, [C.c_void_p, _PF]),
    "qpg_net_set_params": (C.c_int, [C.c_void_p, _PF]),
    "qpg_net_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, _PF]),
    "qpg_net_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, _PF, _PD, _PF]),
    "qpg_net_adam_step": (C.c_int, [C.c_void_p, C.c_float]),
    "qpg_net_destroy": (C.c_int, [C.c_void_p]),
    "qpg_error_string": (C.c_char_p, [C.c_int]),
    "qpg_last_error": (C.c_char_p, [C.c_void_p]),
}


def lib():
    """Load libqpg.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1912_04263_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class QpgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{lib().qpg_error_string(code).decode()} ({code}): {msg}")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(_PD)


def _iptr(a):
    return a.ctypes.data_as(_PI)


def default_settings(**kw) -> Settings:
    s = Settings()
    lib().qpg_default_settings(C.byref(s))
    keep = []
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": QPG_FP64, "mixed": QPG_MIXED}[v]
        if k == "precond" and isinstance(v, str):
            v = {"jacobi": QPG_PRECOND_JACOBI, "learned": QPG_PRECOND_LEARNED}[v]
        if k == "precond_weights":
            w = np.ascontiguousarray(v, dtype=np.float32)
            if w.size != QPG_NET_NPARAMS:
                raise ValueError(f"precond_weights needs {QPG_NET_NPARAMS} floats")
            keep.append(w)
            v = w.ctypes.data_as(_PF)
        if not hasattr(s, k):
            raise TypeError(f"unknown setting {k}")
        setattr(s, k, v)
    s._keep = keep  # arrays referenced by pointer fields (read during setup)
    return s


@dataclasses.dataclass
class SolveInfo:
    status: str
    iter: int
    pcg_iter_total: int
    pcg_iter_max: int
    rho_updates: int
    obj_val: float
    prim_res: float
    dual_res: float
    rho_final: float
    setup_time: float
    solve_time: float
    precision_used: str
    fallback_events: int
    scaling_passes: int
    precond_used: str = "jacobi"
    precond_trials: int = 0
    precond_learned_chosen: int = 0
    precond_switches: int = 0
    infeas_checks: int = 0
    spec_resumes: int = 0


class _CscArrays:
    """Keeps the numpy arrays of one CSC matrix alive while the library reads them."""

    def __init__(self, M: sp.spmatrix):
        M = sp.csc_matrix(M)
        M.sort_indices()
        self.colptr = np.ascontiguousarray(M.indptr, dtype=np.int32)
        self.rowidx = np.ascontiguousarray(M.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(M.data, dtype=np.float64)
        self.c = Csc(M.shape[0], M.shape[1], int(M.nnz), _iptr(self.colptr), _iptr(self.rowidx),
                     _dptr(self.val))


class Solver:
    """One problem resident on the GPU (qpg_setup) and its solves."""

    def __init__(self, P_triu, q, A, l, u, settings: Settings | None = None, **kw):
        self.settings = settings if settings is not None else default_settings(**kw)
        P_triu = sp.csc_matrix(P_triu)
        A = sp.csc_matrix(A)
        self.n, self.m = A.shape[1], A.shape[0]
        Pc, Ac = _CscArrays(P_triu), _CscArrays(A)
        q = np.ascontiguousarray(q, dtype=np.float64)
        l = np.ascontiguousarray(l, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        h = C.c_void_p()
        rc = lib().qpg_setup(C.byref(h), C.byref(Pc.c), _dptr(q), C.byref(Ac.c), _dptr(l), _dptr(u),
                             C.byref(self.settings))
        if rc != QPG_OK:
            raise QpgError(rc, lib().qpg_last_error(None).decode())
        self._h = h

    @classmethod
    def from_qp(cls, qp, **kw):
        return cls(qp.P_triu, qp.q, qp.A, qp.l, qp.u, **kw)

    def _check(self, rc):
        if rc != QPG_OK:
            raise QpgError(rc, lib().qpg_last_error(self._h).decode())

    def solve(self) -> SolveInfo:
        self._check(lib().qpg_solve(self._h))
        return self.info()

    def info(self) -> SolveInfo:
        i = Info()
        self._check(lib().qpg_get_info(self._h, C.byref(i)))
        return SolveInfo(STATUS.get(i.status, str(i.status)), i.iter, i.pcg_iter_total, i.pcg_iter_max,
                         i.rho_updates, i.obj_val, i.prim_res, i.dual_res, i.rho_final, i.setup_time,
                         i.solve_time, "mixed" if i.precision_used == QPG_MIXED else "fp64",
                         i.fallback_events, i.scaling_passes,
                         "learned" if i.precond_used == QPG_PRECOND_LEARNED else "jacobi",
                         i.precond_trials, i.precond_learned_chosen, i.precond_switches, i.infeas_checks,
                         i.spec_resumes)

    def x(self):
        out = np.empty(self.n)
        self._check(lib().qpg_get_x(self._h, _dptr(out)))
        return out

    def y(self):
        out = np.empty(self.m)
        self._check(lib().qpg_get_y(self._h, _dptr(out)))
        return out

    def z(self):
        out = np.empty(self.m)
        self._check(lib().qpg_get_z(self._h, _dptr(out)))
        return out

    def certificate(self):
        """(δx, δy) of an infeasible last solve, each scaled to ‖·‖∞ = 1 (δy certifies primal,
        δx dual infeasibility)."""
        dx, dy = np.empty(self.n), np.empty(self.m)
        self._check(lib().qpg_get_certificate(self._h, _dptr(dx), _dptr(dy)))
        return dx, dy

    def scaling(self):
        D, E, c = np.empty(self.n), np.empty(self.m), C.c_double()
        self._check(lib().qpg_get_scaling(self._h, _dptr(D), _dptr(E), C.byref(c)))
        return D, E, c.value

    def apply(self, op: int, v, precision: int = QPG_FP64):
        v = np.ascontiguousarray(v, dtype=np.float64)
        nin = self.m if op == QPG_OP_AT else self.n
        nout = self.m if op == QPG_OP_A else self.n
        if v.shape != (nin,):
            raise ValueError(f"operator {op} takes a vector of length {nin}")
        out = np.empty(nout)
        self._check(lib().qpg_apply(self._h, op, precision, _dptr(v), _dptr(out)))
        return out

    def pcg(self, b, x0=None, eps=1e-10, rel=True, max_iter=1000, precision=QPG_FP64):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x0 = np.zeros(self.n) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        x = np.empty(self.n)
        it = C.c_int32()
        rn = C.c_double()
        rc = lib().qpg_pcg(self._h, precision, _dptr(b), _dptr(x0), float(eps), int(rel), int(max_iter),
                           _dptr(x), C.byref(it), C.byref(rn))
        if rc not in (QPG_OK, QPG_ERR_STATE):
            self._check(rc)
        return x, it.value, rn.value, rc == QPG_ERR_STATE

    def time_kernel(self, kernel: int, reps: int = 100, precision: int = QPG_FP64) -> float:
        """Average device microseconds of one PCG kernel (HIP events on the solver's stream)."""
        us = C.c_double()
        self._check(lib().qpg_time_kernel(self._h, kernel, precision, reps, C.byref(us)))
        return us.value

    def spmv_layout(self, matrix: int) -> dict:
        """Work-list layout of Ā (0) or B (1): entries, stored positions with/without an LDS
        window, tiles, windowed tiles, staged window columns, slots, chunks."""
        out = (C.c_int64 * 8)()
        self._check(lib().qpg_spmv_layout(self._h, matrix, out))
        keys = ("entries", "windowed_positions", "plain_positions", "tiles", "windowed_tiles",
                "staged_columns", "slots", "chunks")
        return dict(zip(keys, (int(v) for v in out)))

    def kdiag(self, rho: float):
        out = np.empty(self.n)
        self._check(lib().qpg_get_kdiag(self._h, float(rho), _dptr(out)))
        return out

    def hutchinson(self, signs, rho: float, eps: float = 1e-10, max_iter: int = 5000):
        """Hutchinson estimate of diag(K⁻¹) from the given ±1 probes (s×n)."""
        z = np.ascontiguousarray(signs, dtype=np.int8)
        if z.ndim != 2 or z.shape[1] != self.n:
            raise ValueError("signs must be s×n")
        out = np.empty(self.n)
        self._check(lib().qpg_hutchinson(self._h, z.ctypes.data_as(_PB), z.shape[0], float(rho), float(eps),
                                         int(max_iter), _dptr(out)))
        return out

    def hutchinson_noalloc(self, signs, rho: float, eps: float = 1e-10, max_iter: int = 5000):
        """qpg_hutchinson_noalloc: the same estimate with the library's static device scratch."""
        z = np.ascontiguousarray(signs, dtype=np.int8)
        if z.ndim != 2 or z.shape[1] != self.n:
            raise ValueError("signs must be s×n")
        out = np.empty(self.n)
        self._check(lib().qpg_hutchinson_noalloc(self._h, z.ctypes.data_as(_PB), z.shape[0], float(rho),
                                                 float(eps), int(max_iter), _dptr(out)))
        return out

    def set_rho(self, rho: float):
        self._check(lib().qpg_set_rho(self._h, float(rho)))

    def close(self):
        if getattr(self, "_h", None):
            lib().qpg_cleanup(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


WEIGHTS_DIR = os.path.join(HERE, "weights")


def load_weights(name: str = "portfolio_h32") -> np.ndarray:
    """Trained parameters of the learned preconditioner (raw little-endian float32)."""
    w = np.fromfile(os.path.join(WEIGHTS_DIR, name + ".f32"), dtype="<f4")
    if w.size != QPG_NET_NPARAMS:
        raise ValueError(f"{name}: {w.size} floats, expected {QPG_NET_NPARAMS}")
    return w


def solve(P_triu, q, A, l, u, **kw):
    """One-shot solve; returns (x, y, SolveInfo)."""
    with Solver(P_triu, q, A, l, u, **kw) as s:
        info = s.solve()
        return s.x(), s.y(), info


class Net:
    """Network of the learned preconditioner (device-resident parameters and Adam state)."""

    def __init__(self, params=None, seed: int = 0, bf16: bool = True, device: int = 0):
        h = C.c_void_p()
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if p is not None and p.size != QPG_NET_NPARAMS:
            raise ValueError(f"params needs {QPG_NET_NPARAMS} floats")
        rc = lib().qpg_net_create(C.byref(h), None if p is None else p.ctypes.data_as(_PF), int(seed),
                                  int(bool(bf16)), int(device))
        if rc != QPG_OK:
            raise QpgError(rc, "qpg_net_create")
        self._h = h

    def _check(self, rc, what):
        if rc != QPG_OK:
            raise QpgError(rc, what)

    def params(self):
        out = np.empty(QPG_NET_NPARAMS, dtype=np.float32)
        self._check(lib().qpg_net_get_params(self._h, out.ctypes.data_as(_PF)), "get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(lib().qpg_net_set_params(self._h, p.ctypes.data_as(_PF)), "set_params")

    def forward(self, solver: Solver, rho: float):
        g = np.empty(solver.n, dtype=np.float32)
        self._check(lib().qpg_net_forward(self._h, solver._h, float(rho), g.ctypes.data_as(_PF)), "forward")
        return g

    def loss_grad(self, solver: Solver, rho: float, target, want_grad: bool = True):
        t = np.ascontiguousarray(target, dtype=np.float32)
        loss = C.c_double()
        grad = np.empty(QPG_NET_NPARAMS, dtype=np.float32) if want_grad else None
        self._check(lib().qpg_net_loss_grad(self._h, solver._h, float(rho), t.ctypes.data_as(_PF), C.byref(loss),
                                            None if grad is None else grad.ctypes.data_as(_PF)), "loss_grad")
        return loss.value, grad

    def adam_step(self, lr: float):
        self._check(lib().qpg_net_adam_step(self._h, float(lr)), "adam_step")

    def close(self):
        if getattr(self, "_h", None):
            lib().qpg_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

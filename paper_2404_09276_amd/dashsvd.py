"""ctypes binding of libdashsvd.so (the C ABI declared in include/dashsvd.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  Device buffers are torch tensors on the GPU (torch is
used for device memory and streams); host inputs may be numpy arrays.  If the
library is not built, loading fails loudly -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdashsvd.so")

OK, NOT_CONVERGED, RANK_DEFICIENT = 0, 1, 2
ERR_INVALID_ARG, ERR_BAD_CSR, ERR_NONFINITE, ERR_OOM, ERR_HIP, ERR_STATE = -1, -2, -3, -4, -5, -6
F32, F64, BF16 = 0, 1, 2
PREC = {"fp32": 0, "fp64": 1, "bf16": 2}
SHIFT = {"paper": 0, "none": 1, "fixed": 2, "schedule": 3, "learned": 4}
PVE = {"r2": 0, "r1": 1, "nosurr": 2}
EIG = {"auto": 0, "jacobi": 1, "onesided": 2, "tridiag": 3, "cholqr": 4}
# timing: False / True (every kernel group) / "spmm" (the two SpMM groups only)
TIMING = {False: 0, True: 1, "spmm": 2}
# reorder: "auto" (from 2^22 nonzeros), True, False
REORDER = {"auto": 0, True: 1, False: -1}
HEAD = {"auto": 0, "off": -1}
MAX_L = 160
MAX_TRACE = 256


class DashSVDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dashsvd status {status}: {msg}")
        self.status = status


class _Csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p), ("value_dtype", C.c_int32),
                ("on_device", C.c_int32)]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("shift_policy", C.c_int32), ("pve_mode", C.c_int32),
                ("p_max", C.c_int32), ("seed", C.c_uint64), ("hip_stream", C.c_void_p),
                ("long_row", C.c_int32), ("check_interval", C.c_int32), ("schedule", C.c_void_p),
                ("omega", C.c_void_p), ("omega_dtype", C.c_int32), ("omega_on_device", C.c_int32),
                ("timing", C.c_int32), ("tuning_db", C.c_char_p), ("eig_method", C.c_int32),
                ("reorder", C.c_int32), ("slab_kib", C.c_int32), ("batch_nnz_max", C.c_int64),
                ("lane_vectors", C.c_int32), ("dense_head", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("passes", C.c_int32), ("converged", C.c_int32), ("rank_deficient", C.c_int32),
                ("status", C.c_int32), ("l", C.c_int32), ("learned_fallback", C.c_int32),
                ("final_alpha", C.c_double), ("alpha_used", C.c_double * MAX_TRACE),
                ("ratio", C.c_double * MAX_TRACE), ("time_total_ms", C.c_double),
                ("time_setup_ms", C.c_double), ("time_loop_ms", C.c_double),
                ("time_final_ms", C.c_double), ("long_chunks_A", C.c_int64),
                ("long_chunks_AT", C.c_int64), ("kt_ms", C.c_double * 10), ("kt_count", C.c_int32 * 10),
                ("eig_calls", C.c_int32), ("eig_sweeps", C.c_int32),
                ("sweeps_per_call", C.c_int32 * (MAX_TRACE + 2)), ("long_row_used", C.c_int32),
                ("learned_n", C.c_int32),
                ("promoted", C.c_int32), ("cholqr_calls", C.c_int32), ("sub_batches", C.c_int32),
                ("graph_launches", C.c_int32), ("lane_vectors_used", C.c_int32), ("slab_kib_used", C.c_int32),
                ("reordered", C.c_int32), ("head_rows", C.c_int32), ("head_rows_t", C.c_int32)]

class _Metrics(C.Structure):
    _fields_ = [("eps_pve", C.c_double), ("eps_sigma", C.c_double), ("eps_res", C.c_double),
                ("eps_spec", C.c_double), ("spec_norm", C.c_double), ("lanczos_steps", C.c_int32),
                ("pad", C.c_int32)]


KT_NAMES = ["spmm", "spmm_t", "gram", "eig", "rescale", "transpose", "sketch", "final", "cholqr", "check"]


_lib = None

EXPORTS = [
    "dashsvd_create", "dashsvd_destroy", "dashsvd_set_options", "dashsvd_run", "dashsvd_get_USV",
    "dashsvd_get_info", "dashsvd_get_trace", "dashsvd_evaluate", "dashsvd_evaluate_all", "dashsvd_run_batched",
    "dashsvd_get_USV_batched", "dashsvd_get_info_batched", "dashsvd_autotune", "dashsvd_mlp_init",
    "dashsvd_mlp_num_params", "dashsvd_mlp_set_params", "dashsvd_mlp_get_params", "dashsvd_mlp_forward",
    "dashsvd_mlp_grad", "dashsvd_mlp_train_step", "dashsvd_learned_features", "dashsvd_workspace_size",
    "dashsvd_workspace_size_batched", "dashsvd_handle_workspace_size", "dashsvd_set_workspace",
    "dashsvd_status_string",
    "dashsvd_last_error", "dashsvd_k_gaussian", "dashsvd_k_philox_raw", "dashsvd_k_sort_index",
    "dashsvd_k_transpose",
    "dashsvd_k_spmm", "dashsvd_k_spmm_static", "dashsvd_k_gram", "dashsvd_k_eig", "dashsvd_k_eig_prof", "dashsvd_k_eig_onesided",
    "dashsvd_k_eig_tridiag", "dashsvd_k_cholqr", "dashsvd_k_rescale",
]


def lib():
    """Load libdashsvd.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.dashsvd_create.argtypes = [C.POINTER(P), C.POINTER(_Options)]
        L.dashsvd_destroy.argtypes = [P]
        L.dashsvd_destroy.restype = None
        L.dashsvd_set_options.argtypes = [P, C.POINTER(_Options)]
        L.dashsvd_run.argtypes = [P, C.POINTER(_Csr), i32, i32, f64]
        L.dashsvd_get_USV.argtypes = [P, P, i64, P, P, i64, i32, i32]
        L.dashsvd_get_info.argtypes = [P, C.POINTER(_Info)]
        L.dashsvd_get_trace.argtypes = [P, P, i32]
        L.dashsvd_evaluate.argtypes = [P, C.POINTER(_Csr), P, i32, P, P]
        L.dashsvd_evaluate_all.argtypes = [P, C.POINTER(_Csr), P, i32, i32, u64, C.POINTER(_Metrics)]
        L.dashsvd_run_batched.argtypes = [P, C.POINTER(_Csr), i32, i32, i32, f64]
        L.dashsvd_get_USV_batched.argtypes = [P, i32, P, i64, P, P, i64, i32, i32]
        L.dashsvd_get_info_batched.argtypes = [P, i32, C.POINTER(_Info)]
        L.dashsvd_autotune.argtypes = [P, C.POINTER(_Csr), i32, i32, i32, C.c_char_p, C.POINTER(C.c_int32)]
        L.dashsvd_mlp_init.argtypes = [P, i32, u64, f64]
        L.dashsvd_mlp_num_params.argtypes = [P, C.POINTER(C.c_int64)]
        L.dashsvd_mlp_set_params.argtypes = [P, P, i64]
        L.dashsvd_mlp_get_params.argtypes = [P, P, i64]
        L.dashsvd_mlp_forward.argtypes = [P, P, i32, P]
        L.dashsvd_mlp_grad.argtypes = [P, P, P, i32, P, P]
        L.dashsvd_mlp_train_step.argtypes = [P, P, P, i32, C.c_float, P]
        L.dashsvd_learned_features.argtypes = [P, P, i32]
        L.dashsvd_workspace_size.argtypes = [C.POINTER(_Csr), i32, i32, i32, C.POINTER(C.c_size_t)]
        L.dashsvd_workspace_size_batched.argtypes = [C.POINTER(_Csr), i32, i32, i32, i32,
                                                     C.POINTER(C.c_size_t)]
        L.dashsvd_handle_workspace_size.argtypes = [P, C.POINTER(_Csr), i32, i32, i32, i32,
                                                    C.POINTER(C.c_size_t)]
        L.dashsvd_set_workspace.argtypes = [P, P, C.c_size_t]
        L.dashsvd_status_string.argtypes = [i32]
        L.dashsvd_status_string.restype = C.c_char_p
        L.dashsvd_last_error.argtypes = [P]
        L.dashsvd_last_error.restype = C.c_char_p
        L.dashsvd_k_gaussian.argtypes = [u64, i64, i64, P, i64, i32, P]
        L.dashsvd_k_philox_raw.argtypes = [u64, i64, P, P]
        L.dashsvd_k_sort_index.argtypes = [i64, P, P, P, i32, i32, P]
        L.dashsvd_k_transpose.argtypes = [i64, i64, i64, P, P, P, i32, P, P, P, P]
        L.dashsvd_k_spmm.argtypes = [i64, i64, i64, P, P, P, P, i64, i32, P, i64, i32, i32, P, i64, P,
                                     i32, P]
        L.dashsvd_k_spmm_static.argtypes = L.dashsvd_k_spmm.argtypes
        L.dashsvd_k_gram.argtypes = [i64, i32, P, i64, i32, P, P]
        L.dashsvd_k_eig.argtypes = [i32, P, P, P, P, P, P]
        L.dashsvd_k_eig_prof.argtypes = [i32, P, P, P, P, P, P, P]
        L.dashsvd_k_eig_onesided.argtypes = [i32, P, P, P, P, f64, P, P, P, P]
        L.dashsvd_k_eig_tridiag.argtypes = [i32, P, P, P, P, P, P, P]
        L.dashsvd_k_rescale.argtypes = [i64, i32, P, i64, i32, P, i64, i32, P, i64, i32, P]
        for name in EXPORTS:
            if name not in ("dashsvd_destroy", "dashsvd_status_string", "dashsvd_last_error"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(st: int, h=None, ok=(OK,)):
    if st in ok or st > 0:
        return st
    msg = lib().dashsvd_last_error(h).decode(errors="replace")
    raise DashSVDError(st, f"{lib().dashsvd_status_string(st).decode()}: {msg}")


# ---------------------------------------------------------------- marshalling

def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        return C.c_void_p(x.data_ptr())
    return x.ctypes.data_as(C.c_void_p)


def _dtype_code(x) -> int:
    name = str(x.dtype)
    if "float64" in name:
        return F64
    if "bfloat16" in name:
        return BF16
    if "float32" in name:
        return F32
    raise TypeError(f"unsupported dtype {x.dtype}")


def _on_device(x) -> bool:
    return _is_torch(x) and x.is_cuda


def make_csr(m: int, n: int, row_ptr, col, val) -> tuple:
    """Build the C struct; returns (struct, keepalive)."""
    dev = _on_device(row_ptr)
    if dev:
        if not (_on_device(col) and _on_device(val)):
            raise ValueError("row_ptr, col and val must all be device tensors or all host arrays")
        import torch
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32
        keep = (row_ptr, col, val)
    else:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        if val.dtype not in (np.float32, np.float64):
            val = val.astype(np.float64)
        val = np.ascontiguousarray(val)
        keep = (row_ptr, col, val)
    nnz = int(row_ptr[-1]) if not dev else int(col.shape[0])
    s = _Csr(m, n, nnz, _ptr(row_ptr).value, _ptr(col).value if nnz else None,
             _ptr(val).value if nnz else None, _dtype_code(val), 1 if dev else 0)
    return s, keep


@dataclass
class Info:
    passes: int
    converged: bool
    rank_deficient: bool
    status: int
    l: int
    learned_fallback: bool
    final_alpha: float
    alpha_used: np.ndarray
    ratio: np.ndarray
    time_total_ms: float
    time_setup_ms: float
    time_loop_ms: float
    time_final_ms: float
    long_chunks_A: int
    long_chunks_AT: int
    kt_ms: dict
    kt_count: dict
    eig_calls: int
    eig_sweeps: int
    sweeps_per_call: np.ndarray
    promoted: bool
    long_row_used: int
    learned_n: int
    cholqr_calls: int
    sub_batches: int = 1
    graph_launches: int = 0
    lane_vectors_used: int = 1
    slab_kib_used: int = 0
    reordered: bool = False
    head_rows: int = 0
    head_rows_t: int = 0


class DashSVD:
    """Handle of the library (dashsvd_create / dashsvd_run / dashsvd_get_USV)."""

    def __init__(self, precision: str = "fp32", shift_policy: str = "paper", pve_mode: str = "r2",
                 p_max: int = -1, seed: int = 0, stream=None, long_row: int = 0,
                 check_interval: int = 1, schedule=None, omega=None, timing=False,
                 tuning_db=None, eig_method: str = "auto", reorder="auto", slab_kib: int = 0,
                 batch_nnz_max: int = 0, lane_vectors: int = 0, dense_head="auto"):
        self._h = C.c_void_p()
        self._keep = []
        opt = self._options(precision, shift_policy, pve_mode, p_max, seed, stream, long_row,
                            check_interval, schedule, omega, timing, tuning_db, eig_method, reorder,
                            slab_kib, batch_nnz_max, lane_vectors, dense_head)
        st = lib().dashsvd_create(C.byref(self._h), C.byref(opt))
        _check(st, None)

    def _options(self, precision="fp32", shift_policy="paper", pve_mode="r2", p_max=-1, seed=0,
                 stream=None, long_row=0, check_interval=1, schedule=None, omega=None,
                 timing=False, tuning_db=None, eig_method="auto", reorder="auto", slab_kib=0,
                 batch_nnz_max=0, lane_vectors=0, dense_head="auto"):
        sched_arr = None
        if schedule is not None:
            sched_arr = np.ascontiguousarray(schedule, dtype=np.float64)
        om_ptr, om_dt, om_dev = None, F64, 0
        if omega is not None:
            if not _on_device(omega):
                omega = np.ascontiguousarray(omega)
            om_ptr, om_dt, om_dev = _ptr(omega).value, _dtype_code(omega), int(_on_device(omega))
        self._keep = [sched_arr, omega]
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        return _Options(PREC[precision], SHIFT[shift_policy], PVE[pve_mode], p_max, seed,
                        stream or None, long_row, check_interval,
                        _ptr(sched_arr).value if sched_arr is not None else None,
                        om_ptr, om_dt, om_dev, TIMING[timing],
                        tuning_db.encode() if tuning_db else None, EIG[eig_method], REORDER[reorder],
                        int(slab_kib), int(batch_nnz_max), int(lane_vectors), HEAD[dense_head])

    def set_workspace(self, buf):
        """dashsvd_set_workspace: run inside the caller's device buffer (a
        torch tensor on the GPU, e.g. torch.empty(n, dtype=torch.uint8,
        device="cuda")), or back in the handle's own arena with None.  The
        tensor is kept referenced while the handle uses it."""
        if buf is None:
            _check(lib().dashsvd_set_workspace(self._h, None, 0), self._h)
            self._ws = None
            return
        if not _on_device(buf):
            raise ValueError("the workspace must be a device tensor")
        nbytes = buf.numel() * buf.element_size()
        _check(lib().dashsvd_set_workspace(self._h, C.c_void_p(buf.data_ptr()), nbytes), self._h)
        self._ws = buf

    def workspace_bytes(self, A, k: int, p: int) -> int:
        """dashsvd_handle_workspace_size under this handle's options: A is one
        matrix (dashsvd_run) or a list of matrices (dashsvd_run_batched)."""
        batched = isinstance(A, (list, tuple))
        mats = A if batched else [A]
        structs, keeps = [], []
        for M in mats:
            sct, keep = make_csr(M.m, M.n, M.row_ptr, M.col, M.val)
            structs.append(sct)
            keeps.append(keep)
        arr = (_Csr * len(structs))(*structs)
        out = C.c_size_t()
        st = lib().dashsvd_handle_workspace_size(self._h, arr, len(structs), int(batched), k, p,
                                                 C.byref(out))
        del keeps
        _check(st, self._h)
        return int(out.value)

    def set_options(self, **kw):
        opt = self._options(**kw)
        _check(lib().dashsvd_set_options(self._h, C.byref(opt)), self._h)

    def close(self):
        if self._h:
            lib().dashsvd_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, A, k: int, p: int, tol: float, row_ptr=None, col=None, val=None) -> int:
        """dashsvd_run.  A: any object with m, n, row_ptr, col, val (numpy or
        device torch tensors).  Returns the (non-negative) status."""
        s, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
        self._m, self._n, self._k = A.m, A.n, k
        st = lib().dashsvd_run(self._h, C.byref(s), k, p, float(tol))
        del keep
        return _check(st, self._h)

    def get_usv(self, dtype: str = "float64", device: bool = False):
        """dashsvd_get_USV: U (m x k), S (k), V (n x k)."""
        m, n, k = self._dims()
        code = F64 if dtype == "float64" else F32
        if device:
            import torch
            td = torch.float64 if code == F64 else torch.float32
            U = torch.empty((m, k), dtype=td, device="cuda")
            V = torch.empty((n, k), dtype=td, device="cuda")
            S = torch.empty(k, dtype=torch.float64, device="cuda")
        else:
            nd = np.float64 if code == F64 else np.float32
            U = np.empty((m, k), dtype=nd)
            V = np.empty((n, k), dtype=nd)
            S = np.empty(k, dtype=np.float64)
        st = lib().dashsvd_get_USV(self._h, _ptr(U), k, _ptr(S), _ptr(V), k, code, int(device))
        _check(st, self._h)
        return U, S, V

    def _dims(self):
        return self._m, self._n, self._k

    def evaluate(self, A, sigma_ref):
        """dashsvd_evaluate: (eps_PVE, eps_sigma) of the last run on A (the
        same matrix) against reference singular values sigma_ref (>= k+1)."""
        s, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
        sr = np.ascontiguousarray(sigma_ref, dtype=np.float64)
        pve, es = C.c_double(), C.c_double()
        st = lib().dashsvd_evaluate(self._h, C.byref(s), _ptr(sr), int(sr.shape[0]), C.byref(pve),
                                    C.byref(es))
        del keep
        _check(st, self._h)
        return pve.value, es.value

    def evaluate_all(self, A, sigma_ref, max_steps: int = 200, seed: int = 7) -> dict:
        """dashsvd_evaluate_all: the four Sec. 4 metrics of the last run (and
        the Lanczos estimate of ||A - U S V^T||_2 with its step count)."""
        s, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
        sr = np.ascontiguousarray(sigma_ref, dtype=np.float64)
        out = _Metrics()
        st = lib().dashsvd_evaluate_all(self._h, C.byref(s), _ptr(sr), int(sr.shape[0]), int(max_steps),
                                        int(seed), C.byref(out))
        del keep
        _check(st, self._h)
        return {f[0]: getattr(out, f[0]) for f in _Metrics._fields_ if f[0] != "pad"}

    def info(self) -> Info:
        raw = _Info()
        _check(lib().dashsvd_get_info(self._h, C.byref(raw)), self._h)
        return _info_from(raw)

    # ------------------------------------------------------------ batched form
    def run_batched(self, mats, k: int, p: int, tol: float) -> int:
        """dashsvd_run_batched over a list of matrices (objects with m, n,
        row_ptr, col, val; all numpy or all device tensors)."""
        structs, keeps = [], []
        for A in mats:
            s, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
            structs.append(s)
            keeps.append(keep)
        arr = (_Csr * len(structs))(*structs)
        self._bdims = [(A.m, A.n) for A in mats]
        self._bk = k
        st = lib().dashsvd_run_batched(self._h, arr, len(structs), k, p, float(tol))
        del keeps
        return _check(st, self._h)

    def get_usv_batched(self, idx: int, dtype: str = "float64"):
        """dashsvd_get_USV_batched (host arrays): U, S, V of matrix idx."""
        m, n = self._bdims[idx]
        k = self._bk
        code = F64 if dtype == "float64" else F32
        nd = np.float64 if code == F64 else np.float32
        U, V, S = np.empty((m, k), dtype=nd), np.empty((n, k), dtype=nd), np.empty(k, dtype=np.float64)
        _check(lib().dashsvd_get_USV_batched(self._h, idx, _ptr(U), k, _ptr(S), _ptr(V), k, code, 0), self._h)
        return U, S, V

    def autotune(self, mats, k: int, p: int, db_path=None) -> int:
        """dashsvd_autotune on one matrix (a single object) or a batch (a
        list); returns the chosen SpMM chunk length."""
        if not isinstance(mats, (list, tuple)):
            mats = [mats]
        structs, keeps = [], []
        for A in mats:
            s, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
            structs.append(s)
            keeps.append(keep)
        arr = (_Csr * len(structs))(*structs)
        best = C.c_int32()
        st = lib().dashsvd_autotune(self._h, arr, len(structs), k, p,
                                    db_path.encode() if db_path else None, C.byref(best))
        del keeps
        _check(st, self._h)
        return best.value

    # ------------------------------------------------------------ learned shift
    def mlp_init(self, l: int, seed: int = 0, c_max: float = 0.9):
        _check(lib().dashsvd_mlp_init(self._h, l, seed, c_max), self._h)
        self._mlp_l = l
        self._mlp_cmax = c_max

    def mlp_num_params(self) -> int:
        n = C.c_int64()
        _check(lib().dashsvd_mlp_num_params(self._h, C.byref(n)), self._h)
        return n.value

    def mlp_params(self) -> np.ndarray:
        out = np.empty(self.mlp_num_params(), dtype=np.float32)
        _check(lib().dashsvd_mlp_get_params(self._h, _ptr(out), out.shape[0]), self._h)
        return out

    def mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().dashsvd_mlp_set_params(self._h, _ptr(p), p.shape[0]), self._h)

    def mlp_forward(self, X) -> np.ndarray:
        """(batch x 2): the multiplier c in [0.5, c_max] and log N."""
        X = np.ascontiguousarray(X, dtype=np.float32)
        out = np.empty((X.shape[0], 2), dtype=np.float32)
        _check(lib().dashsvd_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(out)), self._h)
        return out

    def mlp_grad(self, X, Y):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        g = np.empty(self.mlp_num_params(), dtype=np.float32)
        loss = C.c_float()
        _check(lib().dashsvd_mlp_grad(self._h, _ptr(X), _ptr(Y), X.shape[0], _ptr(g), C.byref(loss)), self._h)
        return g, loss.value

    def mlp_train_step(self, X, Y, lr: float) -> float:
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        loss = C.c_float()
        _check(lib().dashsvd_mlp_train_step(self._h, _ptr(X), _ptr(Y), X.shape[0], lr, C.byref(loss)),
               self._h)
        return loss.value

    def learned_features(self) -> np.ndarray:
        """Features of the last run (passes 1 and 2), as the LEARNED policy
        computes them on the device."""
        l = self.info().l
        f = np.empty(3 * l + 3, dtype=np.float32)
        _check(lib().dashsvd_learned_features(self._h, _ptr(f), f.shape[0]), self._h)
        return f

    def info_batched(self, idx: int) -> Info:
        """dashsvd_get_info_batched: matrix idx, or the batch summary for idx < 0."""
        raw = _Info()
        _check(lib().dashsvd_get_info_batched(self._h, idx, C.byref(raw)), self._h)
        return _info_from(raw)


    def trace(self) -> np.ndarray:
        """Per-pass S (passes x l) of the last run (dashsvd_get_trace)."""
        inf = self.info()
        out = np.zeros((max(inf.passes, 1), inf.l))
        _check(lib().dashsvd_get_trace(self._h, _ptr(out), inf.passes), self._h)
        return out[:inf.passes]

    def solve(self, A, k: int, p: int, tol: float, dtype: str = "float64", device: bool = False):
        """run + get_usv + info."""
        st = self.run(A, k, p, tol)
        U, S, V = self.get_usv(dtype=dtype, device=device)
        return U, S, V, st, self.info()


def workspace_size(A, k: int, p: int, precision: str = "fp32") -> int:
    s, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
    out = C.c_size_t()
    _check(lib().dashsvd_workspace_size(C.byref(s), k, p, PREC[precision], C.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- kernel-level entries

def _stream_ptr(stream):
    if stream is None:
        return None
    return stream if isinstance(stream, int) else stream.cuda_stream


def k_gaussian(seed: int, out, stream=None):
    """Fill the device tensor out (rows x cols, row-major, contiguous)."""
    rows, cols = out.shape
    _check(lib().dashsvd_k_gaussian(seed, rows, cols, _ptr(out), out.stride(0), _dtype_code(out),
                                    _stream_ptr(stream)))


def k_philox_raw(seed: int, out, stream=None):
    """out: device int64 tensor (bit pattern of uint64 words)."""
    _check(lib().dashsvd_k_philox_raw(seed, out.numel(), _ptr(out), _stream_ptr(stream)))


def k_sort_index(keys, keys_out, idx_out, bits: int, descending: bool = False, stream=None):
    """Stable radix sort of the device int32/uint32 tensor keys on its low bits."""
    _check(lib().dashsvd_k_sort_index(keys.numel(), _ptr(keys), _ptr(keys_out), _ptr(idx_out), int(bits),
                                      int(bool(descending)), _stream_ptr(stream)))


def k_transpose(m, n, row_ptr, col, val, rowT, colT, valT, stream=None):
    _check(lib().dashsvd_k_transpose(m, n, col.numel(), _ptr(row_ptr), _ptr(col), _ptr(val),
                                     _dtype_code(val), _ptr(rowT), _ptr(colT), _ptr(valT),
                                     _stream_ptr(stream)))


def k_spmm(rows, cols, row_ptr, col, val, X, Y, l, Q=None, alpha=None, long_row=0, stream=None):
    _check(lib().dashsvd_k_spmm(rows, cols, col.numel(), _ptr(row_ptr), _ptr(col), _ptr(val),
                                _ptr(X), X.stride(0), _dtype_code(X), _ptr(Y), Y.stride(0),
                                _dtype_code(Y), l, _ptr(Q), Q.stride(0) if Q is not None else 0,
                                _ptr(alpha), long_row, _stream_ptr(stream)))


def k_spmm_static(rows, cols, row_ptr, col, val, X, Y, l, Q=None, alpha=None, long_row=0, stream=None):
    """As k_spmm, through the entry point that allocates nothing (its plan
    lives in the library's static device scratch)."""
    _check(lib().dashsvd_k_spmm_static(rows, cols, col.numel(), _ptr(row_ptr), _ptr(col), _ptr(val),
                                       _ptr(X), X.stride(0), _dtype_code(X), _ptr(Y), Y.stride(0),
                                       _dtype_code(Y), l, _ptr(Q), Q.stride(0) if Q is not None else 0,
                                       _ptr(alpha), long_row, _stream_ptr(stream)))


def k_gram(Cm, l, G, stream=None):
    _check(lib().dashsvd_k_gram(Cm.shape[0], l, _ptr(Cm), Cm.stride(0), _dtype_code(Cm), _ptr(G),
                                _stream_ptr(stream)))


def k_eig(G, S, Vs, W, sweeps=None, stream=None):
    l = G.shape[0]
    _check(lib().dashsvd_k_eig(l, _ptr(G), _ptr(S), _ptr(Vs), _ptr(W), _ptr(sweeps),
                               _stream_ptr(stream)))


def k_eig_onesided(G, S, Vs, W, skip=2.0**-53, sweeps=None, prof=None, stream=None) -> bool:
    """The one-sided Jacobi eigensolver (l <= 128); True if G was accepted
    (positive definite to working precision), else nothing is written.
    prof: optional device int64 tensor of 6 step-profile counters."""
    l = G.shape[0]
    acc = C.c_int32(0)
    _check(lib().dashsvd_k_eig_onesided(l, _ptr(G), _ptr(S), _ptr(Vs), _ptr(W), C.c_double(skip), _ptr(sweeps),
                                        C.byref(acc), _ptr(prof), _stream_ptr(stream)))
    return bool(acc.value)


def k_eig_tridiag(G, S, Vs, W, prof=None, stream=None) -> bool:
    """The tridiagonal eigensolver (l <= 160); True if G was accepted (no
    eigenvalue cluster, nonzero finite entries), else S, Vs and W hold no
    result.  prof: optional device int64 tensor of 8 phase cycle counts."""
    l = G.shape[0]
    acc = C.c_int32(0)
    _check(lib().dashsvd_k_eig_tridiag(l, _ptr(G), _ptr(S), _ptr(Vs), _ptr(W), C.byref(acc),
                                       _ptr(prof) if prof is not None else None, _stream_ptr(stream)))
    return bool(acc.value)


def k_cholqr(G, S, W, stream=None) -> bool:
    """Cholesky-QR weights W = R^-1 and S from the eigenvalues of G; True if
    the kernel accepted G (else W and S are unspecified)."""
    l = G.shape[0]
    acc = C.c_int32(0)
    _check(lib().dashsvd_k_cholqr(l, _ptr(G), _ptr(S), _ptr(W), C.byref(acc), _stream_ptr(stream)))
    return bool(acc.value)


def k_eig_prof(G, S, Vs, W, sweeps, prof, stream=None):
    """k_eig with the step profile (prof: device int64 tensor of 4)."""
    l = G.shape[0]
    _check(lib().dashsvd_k_eig_prof(l, _ptr(G), _ptr(S), _ptr(Vs), _ptr(W), _ptr(sweeps),
                                    _ptr(prof), _stream_ptr(stream)))


def k_rescale(Cm, l, W, c, Out, stream=None):
    _check(lib().dashsvd_k_rescale(Cm.shape[0], l, _ptr(Cm), Cm.stride(0), _dtype_code(Cm), _ptr(W),
                                   W.stride(0), c, _ptr(Out), Out.stride(0), _dtype_code(Out),
                                   _stream_ptr(stream)))


def _info_from(raw) -> Info:
    npass = raw.passes
    return Info(raw.passes, bool(raw.converged), bool(raw.rank_deficient), raw.status, raw.l,
                bool(raw.learned_fallback), raw.final_alpha,
                np.array(raw.alpha_used[:min(npass, MAX_TRACE)]),
                np.array(raw.ratio[:min(npass, MAX_TRACE)]), raw.time_total_ms,
                raw.time_setup_ms, raw.time_loop_ms, raw.time_final_ms, raw.long_chunks_A,
                raw.long_chunks_AT, dict(zip(KT_NAMES, list(raw.kt_ms))),
                dict(zip(KT_NAMES, list(raw.kt_count))), raw.eig_calls, raw.eig_sweeps,
                np.array(raw.sweeps_per_call[:min(raw.eig_calls, MAX_TRACE + 2)]),
                bool(raw.promoted), raw.long_row_used, raw.learned_n, raw.cholqr_calls, raw.sub_batches,
                raw.graph_launches, raw.lane_vectors_used, raw.slab_kib_used, bool(raw.reordered),
                raw.head_rows, raw.head_rows_t)


def workspace_size_batched(mats, k: int, p: int, precision: str = "fp32") -> int:
    structs, keeps = [], []
    for A in mats:
        sct, keep = make_csr(A.m, A.n, A.row_ptr, A.col, A.val)
        structs.append(sct)
        keeps.append(keep)
    arr = (_Csr * len(structs))(*structs)
    out = C.c_size_t()
    st = lib().dashsvd_workspace_size_batched(arr, len(structs), k, p, PREC[precision], C.byref(out))
    del keeps
    _check(st)
    return int(out.value)

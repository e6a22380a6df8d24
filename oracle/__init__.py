"""FP64 CPU oracle for the dashSVD hot path.

TEST INFRASTRUCTURE ONLY.  This package may be imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``; the
product library (``paper_2404_09276_amd``) never imports, links or runs it.
It shares no code with the HIP sources: the arithmetic lives in
``dashsvd_oracle.c`` (plain loops, FP64, OpenMP over independent iterations),
built here with gcc into ``liboracle.so`` and called through ctypes.

Every function cites the passage of the paper it follows (Alg. 3 eigSVD,
Alg. 4/5 dashSVD, eq. (19) PVE check, Sec. 4 error metrics).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dashsvd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SHIFT_PAPER, SHIFT_NONE, SHIFT_FIXED, SHIFT_SCHEDULE = 0, 1, 2, 3
PVE_R2, PVE_R1, PVE_NOSURR = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, u64, i32, f64 = C.c_int64, C.c_uint64, C.c_int32, C.c_double
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_philox_raw.argtypes = [u64, i64, P]
        L.orc_gaussian.argtypes = [u64, i64, i64, P]
        L.orc_csr_spmm.argtypes = [i64, P, P, P, P, i64, P]
        L.orc_csr_transpose.argtypes = [i64, i64, P, P, P, P, P, P]
        L.orc_gram.argtypes = [i64, i64, P, P]
        L.orc_jacobi_eig.argtypes = [i64, P, P, P]
        L.orc_jacobi_eig.restype = C.c_int
        L.orc_eigsvd.argtypes = [i64, i64, P, P, P, P]
        L.orc_eigsvd.restype = C.c_int
        L.orc_pve_ratio.argtypes = [i64, P, P, f64, f64]
        L.orc_pve_ratio.restype = f64
        L.orc_shift_update.argtypes = [i64, P, f64]
        L.orc_shift_update.restype = f64
        L.orc_schedule_shift.argtypes = [i64, f64, f64, f64, f64, f64, f64, f64, P]
        L.orc_schedule_shift.restype = f64
        L.orc_dashsvd.argtypes = [i64, i64, P, P, P, i64, i64, i64, f64, u64, P, i32, i32, P,
                                  P, P, P, P, P]
        L.orc_dashsvd.restype = C.c_int
        L.orc_metrics.argtypes = [i64, i64, P, P, P, i64, P, P, P, P, P]
        L.orc_residual_metrics.argtypes = [i64, i64, P, P, P, i64, P, P, P, P, i64, u64, P, P, P, P]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr64(row_ptr, col, val):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64))


# ---------------------------------------------------------------- primitives

def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def philox_raw(seed: int, nwords: int) -> np.ndarray:
    out = np.zeros(nwords, dtype=np.uint64)
    lib().orc_philox_raw(seed, nwords, _p(out))
    return out


def gaussian(seed: int, rows: int, cols: int) -> np.ndarray:
    """Omega = randn(rows, cols) by Philox4x64-10 + Box-Muller (Alg. 5 step 1)."""
    out = np.zeros((rows, cols), dtype=np.float64)
    lib().orc_gaussian(seed, rows, cols, _p(out))
    return out


def csr_spmm(row_ptr, col, val, X) -> np.ndarray:
    rp, c, v = _csr64(row_ptr, col, val)
    X = np.ascontiguousarray(X, dtype=np.float64)
    m = rp.shape[0] - 1
    Y = np.zeros((m, X.shape[1]), dtype=np.float64)
    lib().orc_csr_spmm(m, _p(rp), _p(c), _p(v), _p(X), X.shape[1], _p(Y))
    return Y


def csr_transpose(m: int, n: int, row_ptr, col, val):
    rp, c, v = _csr64(row_ptr, col, val)
    nnz = int(rp[-1])
    rT = np.zeros(n + 1, dtype=np.int64)
    cT = np.zeros(max(nnz, 1), dtype=np.int32)
    vT = np.zeros(max(nnz, 1), dtype=np.float64)
    lib().orc_csr_transpose(m, n, _p(rp), _p(c), _p(v), _p(rT), _p(cT), _p(vT))
    return rT, cT[:nnz], vT[:nnz]


def gram(Cm) -> np.ndarray:
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    l = Cm.shape[1]
    G = np.zeros((l, l), dtype=np.float64)
    lib().orc_gram(Cm.shape[0], l, _p(Cm), _p(G))
    return G


def jacobi_eig(G):
    """Cyclic Jacobi (Golub & Van Loan Sec. 8.5); ascending eigenvalues."""
    G = np.array(G, dtype=np.float64, order="C", copy=True)
    l = G.shape[0]
    ev = np.zeros(l)
    V = np.zeros((l, l))
    sweeps = lib().orc_jacobi_eig(l, _p(G), _p(ev), _p(V))
    return ev, V, sweeps


def eigsvd(Cm, want_u: bool = True):
    """Alg. 3 (eigSVD): returns U (r x l), S (l, descending), V (l x l), deficient flag."""
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    r, l = Cm.shape
    U = np.zeros((r, l)) if want_u else None
    S = np.zeros(l)
    V = np.zeros((l, l))
    d = lib().orc_eigsvd(r, l, _p(Cm), _p(U) if want_u else None, _p(S), _p(V))
    return U, S, V, bool(d)


def pve_ratio(k: int, S, Sprev, a: float, aprev: float) -> float:
    """Alg. 5 step 5 / eq. (19) surrogate ratio."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    Sp = np.ascontiguousarray(Sprev, dtype=np.float64)
    return float(lib().orc_pve_ratio(k, _p(S), _p(Sp), a, aprev))


def shift_update(S, alpha: float) -> float:
    """Alg. 5 step 6: if S_l > alpha then alpha = (S_l + alpha)/2."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    return float(lib().orc_shift_update(S.shape[0], _p(S), alpha))


def schedule_shift(j: int, ratio: float, prev_ratio: float, ek1: float, prev_ek1: float,
                   el: float, alpha: float, c: float, off: bool):
    """Proposed-multiplier shift (our extension of Alg. 5 step 6) with its
    guard; returns (next shift, guard state)."""
    o = C.c_int32(1 if off else 0)
    a = lib().orc_schedule_shift(j, ratio, prev_ratio, ek1, prev_ek1, el, alpha, c, C.byref(o))
    return float(a), bool(o.value)


# ---------------------------------------------------------------- dashSVD

@dataclass
class OracleResult:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    passes: int
    converged: bool
    deficient: bool
    alpha: np.ndarray       # shift used in each executed pass
    ratio: np.ndarray       # PVE ratio of each executed pass
    s_hat: np.ndarray       # (passes, l) S of each executed pass
    final_alpha: float
    status: int
    Q: np.ndarray           # final basis, min(m,n) x l, algorithm orientation


class _Info(C.Structure):
    _fields_ = [("passes", C.c_int32), ("converged", C.c_int32), ("deficient", C.c_int32),
                ("trace_cap", C.c_int32), ("alpha_used", C.c_void_p), ("ratio", C.c_void_p),
                ("s_hat", C.c_void_p), ("final_alpha", C.c_double)]


def dashsvd(m: int, n: int, row_ptr, col, val, k: int, s: int, p_max: int, tol: float,
            seed: int = 0, omega=None, shift_policy: int = SHIFT_PAPER,
            pve_mode: int = PVE_R2, sched=None) -> OracleResult:
    """dashSVD with PVE accuracy control (Alg. 5; Alg. 4 when tol == 0)."""
    rp, c, v = _csr64(row_ptr, col, val)
    l = k + s
    U = np.zeros((m, k))
    S = np.zeros(k)
    V = np.zeros((n, k))
    Q = np.zeros((min(m, n), l))
    cap = max(p_max, 1)
    a_tr = np.zeros(cap)
    r_tr = np.zeros(cap)
    s_tr = np.zeros((cap, l))
    info = _Info(0, 0, 0, cap, a_tr.ctypes.data, r_tr.ctypes.data, s_tr.ctypes.data, 0.0)
    om = None
    if omega is not None:
        om = np.ascontiguousarray(omega, dtype=np.float64)
    sc = None
    if sched is not None:
        sc = np.ascontiguousarray(sched, dtype=np.float64)
        assert sc.shape[0] >= p_max + 1
    st = lib().orc_dashsvd(m, n, _p(rp), _p(c), _p(v), k, s, p_max, float(tol), seed,
                           _p(om) if om is not None else None, shift_policy, pve_mode,
                           _p(sc) if sc is not None else None, _p(U), _p(S), _p(V),
                           _p(Q), C.byref(info))
    if st < 0:
        raise ValueError(f"oracle rejected arguments (status {st})")
    np_ = info.passes
    return OracleResult(U, S, V, np_, bool(info.converged), bool(info.deficient),
                        a_tr[:np_].copy(), r_tr[:np_].copy(), s_tr[:np_].copy(),
                        info.final_alpha, st, Q)


def metrics(m: int, n: int, row_ptr, col, val, U, S, sigma_ref):
    """eps_PVE and eps_sigma of Sec. 4 against exact sigma_1..sigma_{k+1}."""
    rp, c, v = _csr64(row_ptr, col, val)
    U = np.ascontiguousarray(U, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    sr = np.ascontiguousarray(sigma_ref, dtype=np.float64)
    k = U.shape[1]
    assert sr.shape[0] >= k + 1
    pve = C.c_double()
    es = C.c_double()
    lib().orc_metrics(m, n, _p(rp), _p(c), _p(v), k, _p(U), _p(S), _p(sr), C.byref(pve),
                      C.byref(es))
    return pve.value, es.value


def residual_metrics(m: int, n: int, row_ptr, col, val, U, S, V, sigma_ref, steps: int = 200,
                     seed: int = 7):
    """eps_res and eps_spec of Sec. 4 (and ||A - U S V^T||_2 with the Lanczos
    steps taken) against exact sigma_1..sigma_{k+1}."""
    rp, c, v = _csr64(row_ptr, col, val)
    U = np.ascontiguousarray(U, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    sr = np.ascontiguousarray(sigma_ref, dtype=np.float64)
    k = U.shape[1]
    assert sr.shape[0] >= k + 1 and V.shape == (n, k) and U.shape == (m, k)
    er, es, en = C.c_double(), C.c_double(), C.c_double()
    st = C.c_int64()
    lib().orc_residual_metrics(m, n, _p(rp), _p(c), _p(v), k, _p(U), _p(S), _p(V), _p(sr), steps, seed,
                               C.byref(er), C.byref(es), C.byref(en), C.byref(st))
    return er.value, es.value, en.value, st.value


def num_threads() -> int:
    return int(lib().orc_num_threads())

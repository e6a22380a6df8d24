"""Seeded synthetic inputs for the dashSVD hot path.

This module holds the input generators only: sparse matrices with the shapes,
densities and degree distributions of the workloads, and nothing of the
method's arithmetic.  Both sides of every parity test (the HIP library and
the CPU oracle) consume the matrices it produces.  The Gaussian test block
Omega is NOT generated here: each side implements the counter-based
generator (Philox4x64-10 + Box-Muller) from its published definition.

The paper's real matrices (web graphs, social networks, rating matrices with
3.9 to 237 nonzeros per row on average) are not available; the power-law
generator below stands in for them.

Recipes
-------
uniform_csr(m, n, nnz, seed, row_scale_power):
    nnz distinct cells drawn uniformly without replacement from the m*n grid;
    values N(0, 1) times (i + 1)^(-row_scale_power) for 0-based row i (the
    1-based row index to the power -1/2 for the 2000 x 1500 case).
zipf_csr(m, n, nnz, seed, s=1.1):
    row weights (pi_r(i) + 1)^(-s) and column weights (pi_c(j) + 1)^(-s) with
    seeded random permutations pi, so hubs are scattered; row degrees are the
    weight-proportional share of nnz, capped at n with the excess spread over
    the uncapped rows (water filling), rounded down and topped up by largest
    remainder; each row then draws its degree's worth of distinct columns with
    probability proportional to the column weights (weighted sampling without
    replacement), sorted; values 1 - U[0, 1) in (0, 1], rounded to FP32.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    m: int
    n: int
    row_ptr: np.ndarray  # int64, m + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float32 or float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        A[rows, self.col] = self.val
        return A

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val.astype(np.float64), self.col, self.row_ptr),
                             shape=(self.m, self.n))


def _from_coo_sorted(m: int, n: int, rows: np.ndarray, cols: np.ndarray,
                     vals: np.ndarray) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=row_ptr[1:])
    return CSR(m, n, row_ptr, cols.astype(np.int32), vals)


def uniform_csr(m: int, n: int, nnz: int, seed: int, row_scale_power: float = 0.5,
                dtype=np.float32) -> CSR:
    """Uniform random positions, N(0,1) values scaled per row by i^-power (1-based i)."""
    rng = np.random.default_rng(seed)
    pos = np.sort(rng.choice(m * n, size=nnz, replace=False))
    rows = (pos // n).astype(np.int64)
    cols = (pos % n).astype(np.int64)
    vals = rng.standard_normal(nnz) * (rows + 1.0) ** (-row_scale_power)
    return _from_coo_sorted(m, n, rows, cols, vals.astype(dtype))


def _water_fill(weights: np.ndarray, total: int, cap: int) -> np.ndarray:
    """Integer degrees proportional to weights, each <= cap, summing to total."""
    k = weights.shape[0]
    total = min(total, k * cap)
    capped = np.zeros(k, dtype=bool)
    target = np.zeros(k, dtype=np.float64)
    for _ in range(64):
        free = ~capped
        rem = total - cap * int(capped.sum())
        target[free] = rem * weights[free] / weights[free].sum()
        target[capped] = cap
        new_cap = free & (target > cap)
        if not new_cap.any():
            break
        capped |= new_cap
    d = np.floor(target).astype(np.int64)
    d = np.minimum(d, cap)
    short = total - int(d.sum())
    if short > 0:
        frac = np.where(d < cap, target - np.floor(target), -1.0)
        # largest remainder first; stable in the index on ties
        order = np.argsort(-frac, kind="stable")
        d[order[:short]] += 1
    return d


_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "zipf_gen.c")
_GEN_LIB = os.path.join(_HERE, "libzipfgen.so")
_gen = None


def build(force: bool = True) -> str:
    """Compile the power-law row sampler with gcc (OpenMP)."""
    if force or not os.path.exists(_GEN_LIB) or \
            os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
        tmp = _GEN_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _GEN_SRC, "-lm"])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _genlib():
    global _gen
    if _gen is None:
        if not os.path.exists(_GEN_LIB) or \
                os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
            build()
        L = ctypes.CDLL(_GEN_LIB)
        P = ctypes.c_void_p
        L.zipf_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, ctypes.c_uint64, P, P]
        _gen = L
    return _gen


def zipf_csr(m: int, n: int, nnz: int, seed: int, s: float = 1.1) -> CSR:
    """Power-law (Zipf s) row and column degrees, values in (0, 1] (see module doc)."""
    rng = np.random.default_rng(seed)
    pr = rng.permutation(m)
    pc = rng.permutation(n)
    w_r = (pr + 1.0) ** (-s)
    w_c = (pc + 1.0) ** (-s)
    deg = _water_fill(w_r, nnz, n)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    cdf = np.cumsum(w_c / w_c.sum())
    cdf[-1] = 1.0
    logw = np.log(w_c)
    total = int(row_ptr[-1])
    col = np.empty(max(total, 1), dtype=np.int32)
    val = np.empty(max(total, 1), dtype=np.float32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _genlib().zipf_fill(m, n, P(row_ptr), P(cdf), P(logw), int(seed), P(col), P(val))
    return CSR(m, n, row_ptr, col[:total], val[:total])


def block_diag_known_sigma(blocks, seed: int, dtype=np.float64):
    """Block-diagonal sparse matrix from small dense blocks, rows and columns
    permuted at random.  Its singular values are the union of the blocks'
    singular values, so exact references exist at any scale.  Returns
    (CSR, sigma_sorted_descending)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals, sig = [], [], [], []
    r0 = c0 = 0
    for B in blocks:
        B = np.asarray(B, dtype=np.float64)
        br, bc = B.shape
        ii, jj = np.nonzero(B)
        rows.append(ii + r0)
        cols.append(jj + c0)
        vals.append(B[ii, jj])
        sig.append(np.linalg.svd(B, compute_uv=False))
        r0 += br
        c0 += bc
    m, n = r0, c0
    pr = rng.permutation(m)
    pc = rng.permutation(n)
    rows = pr[np.concatenate(rows)]
    cols = pc[np.concatenate(cols)]
    vals = np.concatenate(vals).astype(dtype)
    A = _from_coo_sorted(m, n, rows.astype(np.int64), cols.astype(np.int64), vals)
    s = np.sort(np.concatenate(sig))[::-1]
    return A, s


def dense_to_csr(D: np.ndarray, dtype=np.float64) -> CSR:
    D = np.asarray(D)
    m, n = D.shape
    ii, jj = np.nonzero(D)
    return _from_coo_sorted(m, n, ii.astype(np.int64), jj.astype(np.int64),
                            D[ii, jj].astype(dtype))


# ------------------------------------------------------------- named workloads

def config_small(dtype=np.float32) -> CSR:
    """2000 x 1500, 1 % density (30,000 nonzeros), uniform positions, values
    N(0,1) scaled by i^-0.5 for 1-based row i; seed 1001."""
    return uniform_csr(2000, 1500, 30000, seed=1001, row_scale_power=0.5, dtype=dtype)


def config_zipf_200k() -> CSR:
    """200,000 x 100,000, 10M nonzeros, Zipf 1.1 degrees, values in (0,1]; seed 1002."""
    return zipf_csr(200_000, 100_000, 10_000_000, seed=1002)


def config_zipf_2m() -> CSR:
    """2,000,000 x 1,000,000, 100M nonzeros, Zipf 1.1 degrees; seed 1003."""
    return zipf_csr(2_000_000, 1_000_000, 100_000_000, seed=1003)


def batched_zipf_shape(b: int, rows=(1000, 100000), density=(0.0005, 0.01), seed: int = 5000):
    """(m, n, nnz) of member b of batched_zipf, without building it."""
    rng = np.random.default_rng(seed + b)
    m = int(rng.integers(rows[0], rows[1] + 1))
    n = max(1, int(np.floor(rng.uniform(0.5, 1.0) * m)))
    d = float(rng.uniform(density[0], density[1]))
    return m, n, max(m, int(round(d * m * n)))


def batched_zipf_member(b: int, rows=(1000, 100000), density=(0.0005, 0.01), seed: int = 5000) -> CSR:
    """Member b of batched_zipf (independent of the others, so a batch can be
    built in parallel)."""
    m, n, nnz = batched_zipf_shape(b, rows, density, seed)
    return zipf_csr(m, n, nnz, seed=seed + b)


def batched_zipf(count: int, rows=(1000, 100000), density=(0.0005, 0.01), seed: int = 5000) -> list:
    """Batch of independent power-law matrices: matrix b has rows
    U[rows[0], rows[1]], columns floor(U(0.5, 1) * rows), density
    U[density[0], density[1]] and Zipf 1.1 degrees, drawn from seed + b
    (the full-size batched workload is 512 matrices with the default
    ranges)."""
    return [batched_zipf_member(b, rows, density, seed) for b in range(count)]


OMEGA_SEED = {"small": 2001, "zipf_200k": 2002, "zipf_2m": 2003}

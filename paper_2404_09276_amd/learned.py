"""Training data and training loop of the learned shift policy.

The paper sets the shift of every pass by one rule (Alg. 5 step 6: alpha <-
(S_l + alpha)/2 when S_l > alpha).  The LEARNED policy of the library lets a
small MLP choose the multiplier c of alpha_j = c E_l(j-1) for passes 3, 4, ...
from what passes 1 and 2 showed; this module builds its training set and
trains it with the library's HIP kernels (dashsvd_mlp_train_step).

Labels (per training matrix): the method is run with the schedule family
c in {0.5, 0.6, 0.7, 0.8, 0.9}, constant from pass 3 (c = 0.5 is the
paper's rule); each run stops by its own PVE check at tol, and its true
eps_PVE (Sec. 4) is measured against reference singular values.  The label
is the c that meets eps_PVE <= tol in the fewest passes (ties go to the
smaller c), and N* is that pass count.

Training matrices: a pool of power-law matrices (rows U[lo, hi], columns
U(0.5, 1) x rows, mean nonzeros per row log-uniform in [4, 64], Zipf 1.1
degrees), seeds 10^6 + i; held-out matrices use seeds 2 x 10^6 + i.  The
shipped model uses rows U[50k, 500k] and five Omega seeds per matrix (each
seed gives its own features and label).
"""
import math

import numpy as np

import synth

from .dashsvd import DashSVD

C_FAMILY = (0.5, 0.6, 0.7, 0.8, 0.9)


def pool_member(seed: int, rows=(20000, 100000), degree=(4.0, 64.0)):
    """One power-law training / held-out matrix (see the module doc)."""
    rng = np.random.default_rng(seed)
    m = int(rng.integers(rows[0], rows[1] + 1))
    n = max(1, int(np.floor(rng.uniform(0.5, 1.0) * m)))
    deg = math.exp(rng.uniform(math.log(degree[0]), math.log(degree[1])))
    nnz = min(int(round(deg * m)), m * n // 2)
    return synth.zipf_csr(m, n, nnz, seed=seed)


def pool(count: int, seed0: int, rows=(20000, 100000), degree=(4.0, 64.0)) -> list:
    """Power-law training / held-out matrices (see the module doc)."""
    return [pool_member(seed0 + i, rows, degree) for i in range(count)]


def to_device(A, torch):
    """A copy of CSR A whose arrays live on the GPU (the solver then reads
    them in place)."""
    class D:
        pass
    d = D()
    d.m, d.n, d.nnz = A.m, A.n, A.nnz
    d.row_ptr = torch.from_numpy(np.ascontiguousarray(A.row_ptr)).cuda()
    d.col = torch.from_numpy(np.ascontiguousarray(A.col)).cuda()
    d.val = torch.from_numpy(np.ascontiguousarray(A.val)).cuda()
    return d


def reference_sigma(A, k: int, seed: int = 11) -> np.ndarray:
    """sigma_1..sigma_{k+1} from the library's FP64 form run with a wider
    block until the PVE ratio is below 1e-9 (lower bounds by Prop. 1)."""
    h = DashSVD(precision="fp64", p_max=200, seed=seed)
    try:
        h.run(A, k + 1, 24, 1e-9)
        _, S, _ = h.get_usv()
    finally:
        h.close()
    return S


def schedule(c: float, p_max: int) -> np.ndarray:
    """Multipliers indexed by pass: 1/2 for passes 1-2, c afterwards."""
    s = np.full(p_max + 1, c, dtype=np.float64)
    s[:2] = 0.5
    return s


def label(A, k: int, s: int, tol: float, seed: int, sigma_ref, precision: str = "fp32", p_max: int = 40):
    """(features, c*, N*, table) of one matrix; table rows (c, passes,
    eps_PVE).  None when no member of the family meets tol."""
    table = []
    feats = None
    h = DashSVD(precision=precision, p_max=p_max, seed=seed)
    try:
        for c in C_FAMILY:
            h.set_options(precision=precision, p_max=p_max, seed=seed, shift_policy="schedule",
                          schedule=schedule(c, p_max))
            st = h.run(A, k, s, tol)
            info = h.info()
            if feats is None and info.passes >= 2:
                feats = h.learned_features()
            pve, _ = h.evaluate(A, sigma_ref)
            table.append((c, info.passes if st == 0 else p_max + 1, pve))
    finally:
        h.close()
    ok = [(n, c) for c, n, pve in table if pve <= tol and n <= p_max]
    if feats is None or not ok:
        return None
    n_star, c_star = min(ok)
    return feats, c_star, n_star, table


def collect(mats, k: int, s: int, tol: float, seed: int, precision: str = "fp32", log=None, seeds_per_matrix=1):
    """Training arrays X (count x (3l+3)), Y (count x 2: c*, log N*) and the
    per-sample tables; matrix i is run with the Omega seeds
    seed + i * seeds_per_matrix + j, j < seeds_per_matrix, each a sample."""
    X, Y, tables = [], [], []
    for i, A in enumerate(mats):
        sig = reference_sigma(A, k)
        for j in range(seeds_per_matrix):
            r = label(A, k, s, tol, seed + i * seeds_per_matrix + j, sig, precision)
            if r is None:
                continue
            f, c, n, table = r
            X.append(f)
            Y.append((c, math.log(n)))
            tables.append(table)
            if log:
                log(f"  matrix {i} seed {j}: {A.m}x{A.n} nnz {A.nnz}: c*={c} N*={n} "
                    + " ".join(f"({t[0]:.1f}:{t[1]},{t[2]:.1e})" for t in table))
    return np.array(X, dtype=np.float32), np.array(Y, dtype=np.float32), tables


def train(X, Y, l: int, epochs: int = 400, lr: float = 1e-3, batch: int = 32, seed: int = 0,
          c_max: float = 0.9):
    """Adam on the library's HIP kernels; returns (parameters, losses)."""
    h = DashSVD()
    losses = []
    try:
        h.mlp_init(l, seed, c_max)
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        for _ in range(epochs):
            perm = rng.permutation(n)
            tot = 0.0
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                tot += h.mlp_train_step(X[idx], Y[idx], lr) * len(idx)
            losses.append(tot / n)
        params = h.mlp_params()
    finally:
        h.close()
    return params, losses


def save(path: str, params, l: int, c_max: float, **meta):
    np.savez(path, params=np.asarray(params, dtype=np.float32), l=np.int64(l), c_max=np.float64(c_max),
             **{k: np.asarray(v) for k, v in meta.items()})


def load(path: str):
    """(params, l, c_max) of a saved model (no pickled objects)."""
    z = np.load(path, allow_pickle=False)
    return z["params"].astype(np.float32), int(z["l"]), float(z["c_max"])


def attach(h: DashSVD, path: str):
    """Give handle h the saved model (for the LEARNED policy)."""
    params, l, c_max = load(path)
    h.mlp_init(l, 0, c_max)
    h.mlp_set_params(params)

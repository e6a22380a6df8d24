"""The SpMM entry point that allocates nothing (dashsvd_k_spmm_static: its
row-split plan and long-row partials live in the library's static device
scratch) against the allocating dashsvd_k_spmm, through the C ABI.

Both run the same plan and kernels, so their outputs must agree bit for bit;
integer-valued inputs also make them equal to the oracle's FP64 product
exactly.  Two calls in a row, the second on a smaller matrix, check that the
second call is not disturbed by what the first left in the shared scratch;
a plan larger than the scratch is refused before any work is queued."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _int_csr(m, n, nnz, seed, long_rows=()):
    """Integer-valued CSR (values in -3..3) with a few dense rows."""
    rng = np.random.default_rng(seed)
    A = synth.uniform_csr(m, n, nnz, seed=seed, dtype=np.float64)
    D = A.to_dense()
    D[D != 0] = rng.integers(-3, 4, size=int((D != 0).sum()))
    for r in long_rows:
        D[r, :] = rng.integers(1, 3, size=n)
    return synth.dense_to_csr(D)


def _both(torch, A, X, l, long_row, Q=None, alpha=None, dtype=None):
    """(allocating result, static result) of the same product."""
    from paper_2404_09276_amd import k_spmm, k_spmm_static
    dtype = dtype or torch.float32
    vdt = np.float64 if dtype == torch.float64 else np.float32
    ld = X.shape[1]
    rp, col, val = _dev(torch, A.row_ptr), _dev(torch, A.col), _dev(torch, A.val.astype(vdt))
    Xd = _dev(torch, X, dtype)
    Qd = _dev(torch, Q, dtype) if Q is not None else None
    ad = torch.tensor([alpha], dtype=torch.float64, device="cuda") if alpha is not None else None
    out = []
    for fn in (k_spmm, k_spmm_static):
        Y = torch.full((A.m, ld), float("nan"), dtype=dtype, device="cuda")
        fn(A.m, A.n, rp, col, val, Xd, Y, l, Q=Qd, alpha=ad, long_row=long_row)
        torch.cuda.synchronize()
        out.append(Y[:, :l].cpu().numpy())
    return out


def test_static_spmm_matches_allocating_twice_shrinking(torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(5)
    # first call: 2,000 x 1,500 with dense rows (many long-row chunks),
    # l = 120; second call: a smaller matrix, fewer chunks, l = 30
    cases = [(_int_csr(2000, 1500, 40000, seed=11, long_rows=(0, 7, 1999)), 120, 64),
             (_int_csr(300, 250, 3000, seed=12, long_rows=(4,)), 30, 16)]
    for A, l, long_row in cases:
        print(f"static spmm: {A.m} x {A.n}, nnz {A.nnz}, l {l}, long_row {long_row}", flush=True)
        ld = (l + 7) // 8 * 8
        X = np.zeros((A.n, ld))
        X[:, :l] = rng.integers(-4, 5, size=(A.n, l))
        Q = np.zeros((A.m, ld))
        Q[:, :l] = rng.integers(-4, 5, size=(A.m, l))
        ref = oracle.csr_spmm(A.row_ptr, A.col, A.val, X[:, :l])
        y_alloc, y_static = _both(torch, A, X, l, long_row)
        assert np.array_equal(y_static, y_alloc)
        assert np.array_equal(y_static.astype(np.float64), ref)
        c_alloc, c_static = _both(torch, A, X, l, long_row, Q=Q, alpha=3.0)
        assert np.array_equal(c_static, c_alloc)
        assert np.array_equal(c_static.astype(np.float64), ref - 3.0 * Q[:, :l])


def test_static_spmm_power_law_fp32_and_fp64(torch_dev):
    """Real-valued power-law matrices: the same plan and kernels give the same
    bits as the allocating entry point, and the oracle's FP64 product within
    FP32 (or FP64) rounding of the row sums."""
    torch = torch_dev
    A = synth.zipf_csr(20000, 12000, 400000, seed=21)
    for dtype, l, rtol in ((torch.float32, 100, 1e-4), (torch.float64, 40, 1e-12), (torch.float32, 16, 1e-4)):
        print(f"static spmm: zipf 20000 x 12000, {dtype}, l {l}", flush=True)
        ld = (l + 7) // 8 * 8
        X = np.zeros((A.n, ld))
        X[:, :l] = np.random.default_rng(l).standard_normal((A.n, l))
        if dtype == torch.float32:
            X = X.astype(np.float32).astype(np.float64)
        y_alloc, y_static = _both(torch, A, X, l, 0, dtype=dtype)
        assert np.array_equal(y_static, y_alloc)
        ref = oracle.csr_spmm(A.row_ptr, A.col, A.val.astype(np.float64), X[:, :l])
        absref = oracle.csr_spmm(A.row_ptr, A.col, np.abs(A.val.astype(np.float64)), np.abs(X[:, :l]))
        assert np.all(np.abs(y_static - ref) <= rtol * absref + 1e-300)


def test_static_spmm_refuses_plan_beyond_scratch(torch_dev):
    """A plan beyond the 32 MiB scratch is refused with the size in the
    message (host-side sizing: nothing is queued)."""
    torch = torch_dev
    from paper_2404_09276_amd import DashSVDError, k_spmm_static
    A = _int_csr(2000, 1500, 200000, seed=13)
    l, ld = 160, 160
    rp, col, val = _dev(torch, A.row_ptr), _dev(torch, A.col), _dev(torch, A.val.astype(np.float32))
    X = torch.zeros((A.n, ld), dtype=torch.float32, device="cuda")
    Y = torch.zeros((A.m, ld), dtype=torch.float32, device="cuda")
    # long_row 1: 400,001 possible chunks of 656 bytes each
    with pytest.raises(DashSVDError, match="static scratch holds 33554432"):
        k_spmm_static(A.m, A.n, rp, col, val, X, Y, l, long_row=1)
    # the same product with the default chunk length fits and is right
    k_spmm_static(A.m, A.n, rp, col, val, X, Y, l)
    torch.cuda.synchronize()
    assert float(Y.abs().max()) == 0.0

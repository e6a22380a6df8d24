"""Kernel-level parity of the HIP library against the FP64 CPU oracle (and the
library routines the oracle is pinned to), one step of the path at a time,
through the C ABI."""
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


# ------------------------------------------------------------------ Omega

def test_philox_raw_bitwise(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import k_philox_raw
    for seed in (0, 2002, 2**63 + 5):
        out = torch.zeros(10007, dtype=torch.int64, device="cuda")
        k_philox_raw(seed, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle.philox_raw(seed, 10007))


@pytest.mark.parametrize("rows,cols", [(1001, 30), (77, 13), (5, 1)])
def test_gaussian_matches_oracle(torch_dev, rows, cols):
    torch = torch_dev
    from paper_2404_09276_amd import k_gaussian
    ref = oracle.gaussian(2001, rows, cols)
    o64 = torch.empty((rows, cols), dtype=torch.float64, device="cuda")
    k_gaussian(2001, o64)
    o32 = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
    k_gaussian(2001, o32)
    obf = torch.empty((rows, cols), dtype=torch.bfloat16, device="cuda")
    k_gaussian(2001, obf)
    torch.cuda.synchronize()
    g64 = o64.cpu().numpy()
    # device and host libm (log, sqrt, sincos) may differ by a few ulps
    assert np.allclose(g64, ref, rtol=1e-14, atol=1e-14)
    g32 = o32.cpu().numpy()
    assert np.abs(g32 - ref.astype(np.float32)).max() <= 2 * np.spacing(np.float32(8.0))
    gbf = obf.float().cpu().numpy()
    assert np.abs(gbf - ref).max() <= 2.0**-8 * np.abs(ref).max()


def test_gaussian_padded_leading_dimension(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import k_gaussian
    buf = torch.full((50, 40), 7.0, dtype=torch.float64, device="cuda")
    k_gaussian(3, buf[:, :30])
    torch.cuda.synchronize()
    g = buf.cpu().numpy()
    assert np.allclose(g[:, :30], oracle.gaussian(3, 50, 30), rtol=1e-14, atol=1e-14)
    assert np.all(g[:, 30:] == 7.0)


# ------------------------------------------------------------------ CSR(A^T)

def _transpose_case(torch, A, dtype=np.float32):
    from paper_2404_09276_amd import k_transpose
    val = A.val.astype(dtype)
    rp, col, v = _dev(torch, A.row_ptr), _dev(torch, A.col), _dev(torch, val)
    rowT = torch.zeros(A.n + 1, dtype=torch.int64, device="cuda")
    colT = torch.zeros(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    valT = torch.zeros(max(A.nnz, 1), dtype=v.dtype, device="cuda")
    k_transpose(A.m, A.n, rp, col, v, rowT, colT, valT)
    torch.cuda.synchronize()
    rT, cT, vT = oracle.csr_transpose(A.m, A.n, A.row_ptr, A.col, val.astype(np.float64))
    assert np.array_equal(rowT.cpu().numpy(), rT)
    assert np.array_equal(colT.cpu().numpy()[:A.nnz], cT)
    assert np.array_equal(valT.cpu().numpy()[:A.nnz].astype(np.float64), vT)


def test_transpose_bitwise_all_segment_classes(torch_dev):
    # Zipf columns: some with more entries than a sort tile holds (4096),
    # some of 65..2048, many of at most 64 (a wavefront's round), singletons
    # and empty columns.
    A = synth.zipf_csr(30000, 6000, 600000, seed=5)
    cnt = np.bincount(A.col, minlength=A.n)
    assert cnt.max() > 2048 and ((cnt > 64) & (cnt <= 2048)).any() and (cnt <= 64).any()
    _transpose_case(torch_dev, A)
    _transpose_case(torch_dev, A, np.float64)


def test_transpose_radix_pass_counts(torch_dev):
    # 300 columns (9 key bits: one pass of 9-bit digits), 70 000 (17 bits:
    # two passes, 9 + 8), 300 000 (19 bits: three passes, 7 + 6 + 6) and 5
    # (3 bits, one pass of 8 digits)
    _transpose_case(torch_dev, synth.zipf_csr(2000, 300, 40000, seed=6))
    _transpose_case(torch_dev, synth.zipf_csr(50000, 70000, 1000000, seed=7))
    _transpose_case(torch_dev, synth.zipf_csr(40000, 300000, 600000, seed=8))
    _transpose_case(torch_dev, synth.uniform_csr(4000, 5, 9000, seed=9))


@pytest.mark.parametrize("n,bits", [(1, 1), (4095, 3), (4097, 9), (100003, 17), (250000, 20), (30011, 32)])
@pytest.mark.parametrize("desc", [False, True])
def test_radix_sort_stable_against_numpy(torch_dev, n, bits, desc):
    """The radix sort alone: keys on their low bits, ascending or descending,
    equal keys in input order; against NumPy's stable argsort, bit for bit,
    with ragged last tiles, one to four passes and many equal keys."""
    torch = torch_dev
    from paper_2404_09276_amd import k_sort_index
    rng = np.random.default_rng(n + bits)
    hi = min(2 ** bits, 2 ** 31)
    keys = rng.integers(0, hi, size=n, dtype=np.int64)
    keys[: n // 3] = keys[0]  # a long run of one key
    keys = keys.astype(np.uint32).view(np.int32)
    kd = _dev(torch, keys)
    ko = torch.empty_like(kd)
    io = torch.empty(n, dtype=torch.int32, device="cuda")
    k_sort_index(kd, ko, io, bits, desc)
    torch.cuda.synchronize()
    ku = keys.view(np.uint32).astype(np.int64)
    order = np.argsort(-ku if desc else ku, kind="stable")
    assert np.array_equal(io.cpu().numpy(), order.astype(np.int32))
    assert np.array_equal(ko.cpu().numpy(), keys[order])


def test_transpose_small_and_ragged(torch_dev):
    rng = np.random.default_rng(3)
    D = rng.standard_normal((70, 45)) * (rng.random((70, 45)) < 0.2)
    D[4] = 0
    D[:, 9] = 0
    _transpose_case(torch_dev, synth.dense_to_csr(D))
    _transpose_case(torch_dev, synth.dense_to_csr(np.eye(3, 5)))


def test_transpose_rejects_bad_csr(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import DashSVDError, k_transpose
    A = synth.uniform_csr(50, 40, 300, seed=1)
    cases = []
    c = A.col.copy(); c[5] = 40; cases.append((A.row_ptr, c, A.val, -2))           # out of range
    r = A.row_ptr.copy(); r[10], r[11] = r[11], r[10]; cases.append((r, A.col, A.val, -2))  # not monotone
    c = A.col.copy(); i = int(A.row_ptr[3]); c[i + 1] = c[i]; cases.append((A.row_ptr, c, A.val, -2))
    v = A.val.copy(); v[7] = np.nan; cases.append((A.row_ptr, A.col, v, -3))
    v = A.val.copy(); v[9] = np.inf; cases.append((A.row_ptr, A.col, v, -3))
    for rp, col, val, code in cases:
        rowT = torch.zeros(A.n + 1, dtype=torch.int64, device="cuda")
        colT = torch.zeros(A.nnz, dtype=torch.int32, device="cuda")
        valT = torch.zeros(A.nnz, dtype=torch.float32, device="cuda")
        with pytest.raises(DashSVDError) as e:
            k_transpose(A.m, A.n, _dev(torch, rp), _dev(torch, col), _dev(torch, val), rowT, colT, valT)
        assert e.value.status == code


# ------------------------------------------------------------------ SpMM

def _int_csr(m, n, nnz, seed, long_rows=()):
    """Integer-valued CSR (values in -3..3) with a few dense rows."""
    rng = np.random.default_rng(seed)
    A = synth.uniform_csr(m, n, nnz, seed=seed, dtype=np.float64)
    D = A.to_dense()
    D[D != 0] = rng.integers(-3, 4, size=int((D != 0).sum()))
    for r in long_rows:
        D[r, :] = rng.integers(1, 3, size=n)
    return synth.dense_to_csr(D)


@pytest.mark.parametrize("l", [3, 16, 30, 120, 150])
@pytest.mark.parametrize("dt", ["f32", "f64", "bf16"])
def test_spmm_integer_bitwise(torch_dev, l, dt):
    """Integer-valued A, X, Q and alpha make every partial sum exact in the
    accumulator, so the result is independent of summation order: the GPU
    must equal the oracle bit for bit, including long (chunked) rows and the
    fused shift C = A X - alpha Q."""
    torch = torch_dev
    from paper_2404_09276_amd import k_spmm
    A = _int_csr(900, 700, 9000, seed=l, long_rows=(3, 500))
    rng = np.random.default_rng(l + 1)
    ld = (l + 7) // 8 * 8
    X = np.zeros((A.n, ld))
    X[:, :l] = rng.integers(-4, 5, size=(A.n, l))
    Q = np.zeros((A.m, ld))
    Q[:, :l] = rng.integers(-4, 5, size=(A.m, l))
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[dt]
    vdt = np.float64 if dt == "f64" else np.float32
    rp, col, val = _dev(torch, A.row_ptr), _dev(torch, A.col), _dev(torch, A.val.astype(vdt))
    Xd = _dev(torch, X, tdt)
    Qd = _dev(torch, Q, tdt)
    ydt = torch.float64 if dt == "f64" else torch.float32
    alpha = torch.tensor([2.0], dtype=torch.float64, device="cuda")
    # cols = 0: rows of X not given, plain loads instead of buffer loads
    for long_row, xrows in ((0, A.n), (64, A.n), (7, A.n), (0, 0), (7, 0)):
        Y = torch.zeros((A.m, ld), dtype=ydt, device="cuda")
        k_spmm(A.m, xrows, rp, col, val, Xd, Y, l, long_row=long_row)
        Cs = torch.zeros((A.m, ld), dtype=ydt, device="cuda")
        k_spmm(A.m, xrows, rp, col, val, Xd, Cs, l, Q=Qd, alpha=alpha, long_row=long_row)
        torch.cuda.synchronize()
        ref = oracle.csr_spmm(A.row_ptr, A.col, A.val, X[:, :l])
        assert np.array_equal(Y.cpu().numpy()[:, :l].astype(np.float64), ref)
        assert np.array_equal(Cs.cpu().numpy()[:, :l].astype(np.float64), ref - 2.0 * Q[:, :l])


def test_spmm_bf16_output_rounding(torch_dev):
    """BF16 output panel: the FP32 accumulator is rounded to nearest even."""
    torch = torch_dev
    from paper_2404_09276_amd import k_spmm
    A = synth.uniform_csr(400, 300, 6000, seed=9)
    l, ld = 24, 24
    X = np.random.default_rng(2).standard_normal((A.n, ld))
    Xb = _dev(torch, X, torch.bfloat16)
    Y = torch.zeros((A.m, ld), dtype=torch.bfloat16, device="cuda")
    k_spmm(A.m, A.n, _dev(torch, A.row_ptr), _dev(torch, A.col), _dev(torch, A.val), Xb, Y, l)
    torch.cuda.synchronize()
    ref = oracle.csr_spmm(A.row_ptr, A.col, A.val.astype(np.float64),
                          Xb.float().cpu().numpy().astype(np.float64))
    got = Y.float().cpu().numpy()
    assert np.all(np.abs(got - ref) <= 2.0**-8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


def test_spmm_real_values_zipf_f32(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import k_spmm
    A = synth.zipf_csr(20000, 8000, 300000, seed=4)
    l, ld = 120, 120
    X = np.random.default_rng(5).standard_normal((A.n, ld)).astype(np.float32)
    Y = torch.zeros((A.m, ld), dtype=torch.float32, device="cuda")
    k_spmm(A.m, A.n, _dev(torch, A.row_ptr), _dev(torch, A.col), _dev(torch, A.val),
           _dev(torch, X), Y, l)
    torch.cuda.synchronize()
    ref = oracle.csr_spmm(A.row_ptr, A.col, A.val, X.astype(np.float64))
    absA = oracle.csr_spmm(A.row_ptr, A.col, np.abs(A.val), np.abs(X).astype(np.float64))
    rowlen = np.diff(A.row_ptr)[:, None]
    # FP32 accumulation bound: |err| <= (len + 1) u sum |a||x|
    assert np.all(np.abs(Y.cpu().numpy() - ref) <= (rowlen + 2) * 2.0**-24 * absA + 1e-30)


# ------------------------------------------------------------------ Gram / eig / rescale

@pytest.mark.parametrize("r,l", [(1, 1), (300, 8), (300, 16), (2000, 16), (37, 30), (500, 32),
                                 (5000, 120), (20001, 150), (300, 160)])
def test_gram_matches_oracle(torch_dev, r, l):
    torch = torch_dev
    from paper_2404_09276_amd import k_gram
    ld = (l + 7) // 8 * 8
    Cm = np.random.default_rng(r).standard_normal((r, ld)).astype(np.float32)
    G = torch.zeros((l, l), dtype=torch.float64, device="cuda")
    k_gram(_dev(torch, Cm), l, G)
    torch.cuda.synchronize()
    ref = oracle.gram(Cm[:, :l].astype(np.float64))
    g = G.cpu().numpy()
    # FP32 x FP32 products are exact in FP64; only the summation order differs
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.array_equal(g, g.T)


def test_gram_integer_exact_f64(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import k_gram
    Cm = np.random.default_rng(1).integers(-50, 50, size=(3001, 48)).astype(np.float64)
    G = torch.zeros((45, 45), dtype=torch.float64, device="cuda")
    k_gram(_dev(torch, Cm), 45, G)
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), Cm[:, :45].T @ Cm[:, :45])


@pytest.mark.parametrize("r,l,pad", [(1001, 120, 8), (77, 10, 6), (4099, 33, 15)])
def test_gram_ignores_pad_columns(torch_dev, r, l, pad):
    """Pad columns past l may hold anything, NaN included: G must not see them."""
    torch = torch_dev
    from paper_2404_09276_amd import k_gram
    Cm = np.random.default_rng(r + l).standard_normal((r, l + pad)).astype(np.float32)
    Cm[:, l:] = np.nan
    G = torch.zeros((l, l), dtype=torch.float64, device="cuda")
    k_gram(_dev(torch, Cm), l, G)
    torch.cuda.synchronize()
    ref = oracle.gram(Cm[:, :l].astype(np.float64))
    g = G.cpu().numpy()
    assert np.all(np.isfinite(g))
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("l", [1, 2, 3, 5, 16, 24, 30, 75, 120, 150, 160])
def test_eig_matches_lapack(torch_dev, l):
    torch = torch_dev
    from paper_2404_09276_amd import k_eig
    rng = np.random.default_rng(100 + l)
    B = rng.standard_normal((l + 7, l)) @ np.diag(np.logspace(0, -2, l))
    G = B.T @ B
    Gd = _dev(torch, G)
    S = torch.zeros(l, dtype=torch.float64, device="cuda")
    Vs = torch.zeros((l, l), dtype=torch.float64, device="cuda")
    W = torch.zeros((l, l), dtype=torch.float64, device="cuda")
    sw = torch.zeros(1, dtype=torch.int32, device="cuda")
    k_eig(Gd, S, Vs, W, sw)
    torch.cuda.synchronize()
    s, V, Wm = S.cpu().numpy(), Vs.cpu().numpy(), W.cpu().numpy()
    lam = np.linalg.eigvalsh(G)[::-1]
    nrm = lam[0]
    assert np.all(np.diff(s) <= 0)
    assert np.abs(s**2 - lam).max() <= 100 * l * 2.2e-16 * nrm
    assert np.abs(V.T @ V - np.eye(l)).max() < 1e-12
    assert np.linalg.norm(G @ V - V * s**2) <= 100 * l * 2.2e-16 * nrm
    assert np.allclose(Wm, V / s, rtol=1e-14, atol=0)
    assert 0 <= int(sw.cpu()[0]) <= 20
    # agrees with the oracle's cyclic Jacobi (eigenvalues)
    ev, _, _ = oracle.jacobi_eig(G)
    assert np.abs(np.sqrt(np.maximum(ev[::-1], 0)) - s).max() <= 1e-12 * s[0]


def test_eig_diagonal_and_clustered(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import k_eig
    for G in (np.diag([4.0, 9.0, 1.0, 16.0, 25.0]),
              np.diag(np.r_[np.full(6, 2.0), np.full(6, 2.0 + 1e-9), [5.0]]) + 1e-12):
        l = G.shape[0]
        S = torch.zeros(l, dtype=torch.float64, device="cuda")
        Vs = torch.zeros((l, l), dtype=torch.float64, device="cuda")
        W = torch.zeros((l, l), dtype=torch.float64, device="cuda")
        k_eig(_dev(torch, G), S, Vs, W)
        torch.cuda.synchronize()
        lam = np.linalg.eigvalsh(G)[::-1]
        assert np.allclose(S.cpu().numpy() ** 2, lam, rtol=1e-14, atol=1e-15)
        V = Vs.cpu().numpy()
        assert np.abs(V.T @ V - np.eye(l)).max() < 1e-13


def test_eig_rank_deficient_zeroes_w(torch_dev):
    torch = torch_dev
    from paper_2404_09276_amd import k_eig
    B = np.random.default_rng(2).standard_normal((40, 3)) @ np.random.default_rng(3).standard_normal((3, 8))
    G = B.T @ B
    S = torch.zeros(8, dtype=torch.float64, device="cuda")
    Vs = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    W = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    k_eig(_dev(torch, G), S, Vs, W)
    torch.cuda.synchronize()
    assert np.all(W.cpu().numpy()[:, 3:] == 0.0)
    _, So, _, _ = oracle.eigsvd(B)
    assert np.allclose(S.cpu().numpy()[:3], So[:3], rtol=1e-12)


# ------------------------------------------------------------------ one-sided Jacobi eigensolver
def _eig1s(torch, G, skip=2.0**-53):
    from paper_2404_09276_amd import k_eig_onesided
    l = G.shape[0]
    S = torch.full((l,), -1.0, dtype=torch.float64, device="cuda")
    Vs = torch.full((l, l), -1.0, dtype=torch.float64, device="cuda")
    W = torch.full((l, l), -1.0, dtype=torch.float64, device="cuda")
    sw = torch.zeros(1, dtype=torch.int32, device="cuda")
    acc = k_eig_onesided(_dev(torch, G), S, Vs, W, skip, sw)
    return acc, S.cpu().numpy(), Vs.cpu().numpy(), W.cpu().numpy(), int(sw.cpu()[0])


@pytest.mark.parametrize("l", [1, 2, 3, 5, 16, 24, 30, 31, 32, 33, 50, 63, 64, 65, 75, 96, 97, 110, 120, 127, 128])
def test_eig_onesided_matches_lapack(torch_dev, l):
    """Every layout (L = 32, 64, 96, 128) with ragged sizes: eigenvalues
    against LAPACK and the oracle's Jacobi within the rounding of G, Vs
    orthonormal eigenvectors (residual at the same level), W = Vs / S."""
    rng = np.random.default_rng(100 + l)
    B = rng.standard_normal((l + 7, l)) @ np.diag(np.logspace(0, -2, l))
    G = B.T @ B
    acc, s, V, Wm, sw = _eig1s(torch_dev, G)
    assert acc
    lam = np.linalg.eigvalsh(G)[::-1]
    nrm = lam[0]
    assert np.all(np.diff(s) <= 0)
    assert np.abs(s**2 - lam).max() <= 100 * l * 2.2e-16 * nrm
    assert np.abs(V.T @ V - np.eye(l)).max() < 1e-12
    assert np.linalg.norm(G @ V - V * s**2) <= 100 * l * 2.2e-16 * nrm
    assert np.allclose(Wm, V / s, rtol=1e-14, atol=0)
    assert 0 <= sw <= 20
    ev, _, _ = oracle.jacobi_eig(G)
    assert np.abs(np.sqrt(np.maximum(ev[::-1], 0)) - s).max() <= 1e-12 * s[0]


@pytest.mark.parametrize("l", [24, 120])
def test_eig_onesided_fp32_threshold(torch_dev, l):
    """The 2^-23 threshold of the FP32 and BF16 forms: Vs orthonormal to
    about 2^-23 and eigenvalues within O(2^-46) relative, in fewer sweeps."""
    rng = np.random.default_rng(7 + l)
    B = rng.standard_normal((2 * l, l)) @ np.diag(np.logspace(0, -1, l))
    G = B.T @ B
    acc, s, V, Wm, sw = _eig1s(torch_dev, G, 2.0**-23)
    acc64, s64, _, _, sw64 = _eig1s(torch_dev, G)
    assert acc and acc64
    lam = np.linalg.eigvalsh(G)[::-1]
    assert np.abs(V.T @ V - np.eye(l)).max() < 4 * l * 2.0**-23
    assert np.abs(s**2 - lam).max() <= 1e-10 * lam[0]
    assert sw <= sw64


def test_eig_onesided_diagonal_clustered_and_blocks(torch_dev):
    """Diagonal (no rotation: zero sweeps), clustered and block-diagonal G."""
    Gs = [np.diag([4.0, 9.0, 1.0, 16.0, 25.0]),
          np.diag(np.r_[np.full(6, 2.0), np.full(6, 2.0 + 1e-9), [5.0]]) + 1e-12,
          np.kron(np.eye(40), np.array([[2.0, 1.0], [1.0, 3.0]]))]
    for n, G in enumerate(Gs):
        l = G.shape[0]
        acc, s, V, Wm, sw = _eig1s(torch_dev, G)
        assert acc
        lam = np.linalg.eigvalsh(G)[::-1]
        assert np.allclose(s**2, lam, rtol=1e-14, atol=1e-14 * lam[0])
        assert np.abs(V.T @ V - np.eye(l)).max() < 1e-13
        if n == 0:
            assert sw == 0
            assert np.array_equal(np.abs(V) > 0.5, np.eye(5)[:, [4, 3, 1, 0, 2]] > 0.5)


def test_eig_onesided_declines_singular_and_nonfinite(torch_dev):
    """A non-positive or non-finite pivot declines (nothing written); a
    rank-deficient G whose factorisation completes on rounding-level pivots
    gives its nonzero eigenvalues and zero W columns past the rank."""
    for G in (np.diag([1.0, 2.0, -1.0, 3.0]), np.diag([1.0, np.nan, 2.0]), np.diag([1.0, np.inf, 2.0]),
              np.zeros((6, 6))):
        acc, s, V, Wm, _ = _eig1s(torch_dev, G)
        assert not acc
        assert np.all(s == -1.0) and np.all(Wm == -1.0)
    G = np.eye(5)
    G[1, 3] = G[3, 1] = np.nan
    acc, _, _, _, _ = _eig1s(torch_dev, G)
    assert not acc
    B = np.random.default_rng(2).standard_normal((40, 3)) @ np.random.default_rng(3).standard_normal((3, 8))
    acc, s, V, Wm, _ = _eig1s(torch_dev, B.T @ B)
    if acc:
        assert np.all(Wm[:, 3:] == 0.0)
        _, So, _, _ = oracle.eigsvd(B)
        assert np.allclose(s[:3], So[:3], rtol=1e-12)


def test_eig_onesided_rejects_large_l(torch_dev):
    from paper_2404_09276_amd import DashSVDError
    with pytest.raises(DashSVDError):
        _eig1s(torch_dev, np.eye(129))


# ------------------------------------------------------------------ tridiagonal eigensolver
def _eigtri(torch, G):
    from paper_2404_09276_amd import k_eig_tridiag
    l = G.shape[0]
    S = torch.full((l,), -1.0, dtype=torch.float64, device="cuda")
    Vs = torch.full((l, l), -1.0, dtype=torch.float64, device="cuda")
    W = torch.full((l, l), -1.0, dtype=torch.float64, device="cuda")
    acc = k_eig_tridiag(_dev(torch, G), S, Vs, W)
    return acc, S.cpu().numpy(), Vs.cpu().numpy(), W.cpu().numpy()


@pytest.mark.parametrize("l", [1, 2, 3, 5, 16, 24, 30, 31, 32, 33, 64, 65, 75, 96, 110, 120, 127, 128, 129,
                               150, 159, 160])
def test_eig_tridiag_matches_lapack(torch_dev, l):
    """Householder (register tiles of 1 to 5 rows and columns a thread) +
    multisection + twisted factorisations + back-transform, ragged sizes up
    to 160: eigenvalues against LAPACK and the oracle's Jacobi
    within 100 l eps ||G|| (normwise, as the paper's LAPACK eig), Vs
    orthonormal to 1e-8 (graded spectra; the FP32 and BF16 forms that use it
    store Q to 2^-24), residual at the eigenvalue level, W = Vs / S."""
    rng = np.random.default_rng(400 + l)
    B = rng.standard_normal((l + 7, l)) @ np.diag(np.logspace(0, -2, l))
    G = B.T @ B
    acc, s, V, Wm = _eigtri(torch_dev, G)
    assert acc
    lam = np.linalg.eigvalsh(G)[::-1]
    nrm = lam[0]
    assert np.all(np.diff(s) <= 0)
    assert np.abs(s**2 - lam).max() <= 100 * l * 2.2e-16 * nrm
    assert np.abs(V.T @ V - np.eye(l)).max() < 1e-8
    assert np.linalg.norm(G @ V - V * s**2) <= 100 * l * 2.2e-16 * nrm
    assert np.allclose(Wm, V / s, rtol=1e-14, atol=0)
    ev, _, _ = oracle.jacobi_eig(G)
    assert np.abs(np.sqrt(np.maximum(ev[::-1], 0)) ** 2 - s**2).max() <= 100 * l * 2.2e-16 * nrm


def test_eig_tridiag_structured_and_declines(torch_dev):
    """Already-tridiagonal and diagonal G (reflector-free steps), a dense G
    with well separated eigenvalues; clusters (repeated eigenvalues, a
    block-diagonal G with equal blocks), a zero G and non-finite G decline."""
    rng = np.random.default_rng(5)
    T = np.diag(np.arange(1.0, 41.0)) + np.diag(np.full(39, 0.3), 1) + np.diag(np.full(39, 0.3), -1)
    Q, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    for G in (np.diag([4.0, 9.0, 1.0, 16.0, 25.0]), T, (Q * np.linspace(1.0, 50.0, 50)) @ Q.T):
        G = 0.5 * (G + G.T)
        l = G.shape[0]
        acc, s, V, Wm = _eigtri(torch_dev, G)
        assert acc
        lam = np.linalg.eigvalsh(G)[::-1]
        assert np.allclose(s**2, lam, rtol=0, atol=100 * l * 2.2e-16 * lam[0])
        assert np.abs(V.T @ V - np.eye(l)).max() < 1e-12
    for G in (np.diag([1.0, 2.0, 2.0, 3.0]), np.kron(np.eye(4), np.array([[2.0, 1.0], [1.0, 3.0]])),
              np.diag([1.0, np.nan, 2.0]), np.zeros((6, 6)), np.diag(np.r_[np.arange(1.0, 140.0), 7.0])):
        acc, s, V, Wm = _eigtri(torch_dev, G)
        assert not acc


def test_eig_tridiag_rejects_large_l(torch_dev):
    from paper_2404_09276_amd import DashSVDError
    with pytest.raises(DashSVDError):
        _eigtri(torch_dev, np.eye(161))


# ------------------------------------------------------------------ Cholesky-QR pass solver
def _cholqr(torch, G):
    from paper_2404_09276_amd import k_cholqr
    l = G.shape[0]
    S = torch.full((l,), -1.0, dtype=torch.float64, device="cuda")
    W = torch.full((l, l), -1.0, dtype=torch.float64, device="cuda")
    acc = k_cholqr(_dev(torch, G), S, W)
    return acc, S.cpu().numpy(), W.cpu().numpy()


@pytest.mark.parametrize("l", [1, 2, 3, 5, 16, 24, 30, 75, 120, 129, 150, 160])
def test_cholqr_weights_and_values(torch_dev, l):
    """W = R^-1 with G = R^T R (upper triangular, W^T G W = I) and S against
    the oracle's Jacobi eigenvalues, on graded Gram matrices."""
    rng = np.random.default_rng(300 + l)
    B = rng.standard_normal((l + 7, l)) @ np.diag(np.logspace(0, -2, l))
    G = B.T @ B
    acc, s, Wm = _cholqr(torch_dev, G)
    assert acc
    assert np.all(np.tril(Wm, -1) == 0.0)
    assert np.abs(Wm.T @ G @ Wm - np.eye(l)).max() <= 1e-10
    # R = W^-1 is the Cholesky factor: its diagonal is positive
    assert np.all(np.diag(Wm) > 0)
    ev, _, _ = oracle.jacobi_eig(G)
    ref = np.sqrt(np.maximum(ev[::-1], 0))
    assert np.all(np.diff(s) <= 0)
    assert np.abs(s**2 - ref**2).max() <= 100 * l * 2.2e-16 * ref[0] ** 2


def test_cholqr_reduced_and_block_structure(torch_dev):
    """Columns already reduced (diagonal and block-diagonal G) take the
    reflector-free step; clustered eigenvalues keep their multiplicity."""
    Gs = [np.diag([4.0, 9.0, 1.0, 16.0, 25.0]),
          np.diag(np.r_[np.full(6, 2.0), np.full(6, 2.0 + 1e-9), [5.0]]),
          np.kron(np.eye(4), np.array([[2.0, 1.0], [1.0, 3.0]]))]
    for G in Gs:
        l = G.shape[0]
        acc, s, Wm = _cholqr(torch_dev, G)
        assert acc
        ev, _, _ = oracle.jacobi_eig(G)
        assert np.allclose(s**2, ev[::-1], rtol=1e-14, atol=1e-15 * ev.max())
        assert np.abs(Wm.T @ G @ Wm - np.eye(l)).max() <= 1e-13


def test_cholqr_declines_ill_conditioned_and_singular(torch_dev):
    """The kernel declines G with lambda_min <= 2^-32 lambda_max, singular G,
    and G with a non-finite entry (the solver then runs Jacobi)."""
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    for lam_min in (1e-10, 0.0):
        G = (Q * np.r_[np.ones(19), lam_min]) @ Q.T
        G = 0.5 * (G + G.T)
        acc, _, _ = _cholqr(torch_dev, G)
        assert not acc
    B = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 8))
    acc, _, _ = _cholqr(torch_dev, B.T @ B)
    assert not acc
    G = np.eye(6)
    G[2, 2] = np.nan
    acc, _, _ = _cholqr(torch_dev, G)
    assert not acc
    # just inside the accepted range: kappa = 2^30
    G = (Q * np.r_[np.ones(19), 2.0**-30]) @ Q.T
    acc, s, Wm = _cholqr(torch_dev, 0.5 * (G + G.T))
    assert acc
    assert abs(s[-1] ** 2 - 2.0**-30) <= 1e3 * 2.2e-16


@pytest.mark.parametrize("r,l,c", [(70001, 120, 120), (4099, 33, 20), (17, 150, 160)])
def test_rescale_pad_columns_and_many_tiles(torch_dev, r, l, c):
    """Pad columns of C past l may hold anything (NaN here); row counts that
    leave wavefronts with several 16-row tiles and a ragged last tile."""
    torch = torch_dev
    from paper_2404_09276_amd import k_rescale
    ld = (l + 7) // 8 * 8 + 8
    ldo = (c + 7) // 8 * 8
    rng = np.random.default_rng(r + l)
    Cm = rng.standard_normal((r, ld)).astype(np.float32)
    Cm[:, l:] = np.nan
    W = rng.standard_normal((l, c))
    Out = torch.full((r, ldo), 3.0, dtype=torch.float32, device="cuda")
    k_rescale(_dev(torch, Cm), l, _dev(torch, W), c, Out)
    torch.cuda.synchronize()
    ref = Cm[:, :l].astype(np.float64) @ W
    got = Out.cpu().numpy()
    scale = np.abs(Cm[:, :l]).astype(np.float64) @ np.abs(W)
    assert np.all(np.abs(got[:, :c] - ref) <= 4 * l * 2.0**-24 * scale + 1e-300)
    assert np.all(got[:, c:] == 0.0)


@pytest.mark.parametrize("r,l,c,odt", [(1000, 30, 30, "f32"), (777, 120, 120, "f32"), (300, 150, 100, "f32"),
                                       (5000, 150, 150, "bf16"), (500, 30, 20, "f64"), (65, 7, 3, "f32")])
def test_rescale_matches_numpy(torch_dev, r, l, c, odt):
    torch = torch_dev
    from paper_2404_09276_amd import k_rescale
    ld = (l + 7) // 8 * 8
    ldo = (c + 7) // 8 * 8
    rng = np.random.default_rng(r)
    cdt = np.float64 if odt == "f64" else np.float32
    Cm = rng.standard_normal((r, ld)).astype(cdt)
    W = rng.standard_normal((l, c))
    tod = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[odt]
    Out = torch.full((r, ldo), 3.0, dtype=tod, device="cuda")
    k_rescale(_dev(torch, Cm), l, _dev(torch, W), c, Out)
    torch.cuda.synchronize()
    ref = Cm[:, :l].astype(np.float64) @ W
    got = Out.float().cpu().numpy().astype(np.float64) if odt == "bf16" else Out.cpu().numpy()
    scale = np.abs(Cm[:, :l]).astype(np.float64) @ np.abs(W)
    tol = {"f32": 4 * l * 2.0**-24, "f64": 4 * l * 2.0**-53, "bf16": 2.0**-8 + 4 * l * 2.0**-24}[odt]
    assert np.all(np.abs(got[:, :c] - ref) <= tol * scale + 1e-300)
    assert np.all(got[:, c:] == 0.0)

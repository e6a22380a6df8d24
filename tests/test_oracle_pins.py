"""Pins of the FP64 oracle against things other than itself.

Each test ties an oracle function to a library routine written by someone
else (NumPy's Philox, scipy.sparse, LAPACK eigh/svd), to a closed form, to a
hand-derived sequence (tests/golden), or to an invariant the paper proves.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Philox

@pytest.mark.parametrize("seed", [0, 1, 2001, 2002, 2**63 + 12345])
def test_philox_raw_matches_numpy_bitwise(seed):
    """Alg. 5 step 1 draws randn; our reading fixes Philox4x64-10 keyed by
    (seed, 0).  NumPy's Philox is an independent implementation of the same
    published generator: the raw words must match bit for bit."""
    ours = oracle.philox_raw(seed, 4099)
    ref = np.random.Philox(key=seed).random_raw(4099)
    assert np.array_equal(ours, ref)


def test_philox_block_function_with_arbitrary_counter():
    """The block function with every counter and key word nonzero: NumPy's
    generator with counter c emits block f(c + 1, key) first."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ref = np.random.Philox(counter=ctr, key=key).random_raw(4)
        c1 = ctr.copy()
        c1[0] += np.uint64(1)  # no carry: c[0] < 2^63
        assert np.array_equal(oracle.philox4x64_10(c1, key), ref)


def test_gaussian_distribution():
    """Box-Muller output must be N(0,1): mean, variance, KS statistic, and
    independence of the cosine/sine halves of each pair."""
    from scipy import stats
    z = oracle.gaussian(2002, 2000, 500).ravel()
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1.0) < 5e-3
    assert stats.kstest(z, "norm").pvalue > 1e-3
    ev, od = z[0::2], z[1::2]
    assert abs(np.corrcoef(ev, od)[0, 1]) < 5e-3
    # tail mass: P(|z| > 3) = 0.0026998
    assert abs(np.mean(np.abs(z) > 3.0) - 0.0026998) < 4e-4


def test_gaussian_uses_word_pairs_in_order():
    """Element 2t and 2t+1 come from raw words 2t, 2t+1 (radius from the
    first, angle from the second).  Checked through the radius, which the
    pair shares: z[2t]^2 + z[2t+1]^2 = -2 ln(u1)."""
    seed, rows, cols = 99, 7, 6
    z = oracle.gaussian(seed, rows, cols).ravel()
    w = np.random.Philox(key=seed).random_raw(rows * cols)
    u1 = ((w[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53
    r2 = z[0::2] ** 2 + z[1::2] ** 2
    assert np.allclose(r2, -2.0 * np.log(u1), rtol=1e-13, atol=0)
    u2 = (w[1::2] >> np.uint64(11)).astype(np.float64) * 2.0**-53
    ang = np.mod(np.arctan2(z[1::2], z[0::2]), 2 * np.pi)
    d = np.abs(ang - 2 * np.pi * u2)
    d = np.minimum(d, 2 * np.pi - d)
    assert d.max() < 1e-12


def test_gaussian_odd_length_tail():
    z_odd = oracle.gaussian(5, 3, 3).ravel()      # 9 elements
    z_even = oracle.gaussian(5, 2, 5).ravel()     # 10 elements, same stream
    assert np.array_equal(z_odd, z_even[:9])


# ------------------------------------------------------------------ sparse

def _csr_small(seed=3, m=57, n=41, density=0.2):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((m, n)) * (rng.random((m, n)) < density)
    D[5, :] = 0.0  # an empty row
    D[:, 7] = 0.0  # an empty column
    return synth.dense_to_csr(D), D


def test_spmm_matches_scipy():
    A, D = _csr_small()
    X = np.random.default_rng(1).standard_normal((A.n, 13))
    Y = oracle.csr_spmm(A.row_ptr, A.col, A.val, X)
    ref = A.to_scipy() @ X
    assert np.allclose(Y, ref, rtol=1e-14, atol=1e-14)


def test_spmm_integer_values_exact():
    """Integer-valued inputs make every partial sum exact in FP64."""
    rng = np.random.default_rng(2)
    D = rng.integers(-3, 4, size=(40, 30)) * (rng.random((40, 30)) < 0.3)
    A = synth.dense_to_csr(D.astype(np.float64))
    X = rng.integers(-5, 6, size=(30, 9)).astype(np.float64)
    Y = oracle.csr_spmm(A.row_ptr, A.col, A.val, X)
    assert np.array_equal(Y, D @ X)


def test_transpose_matches_scipy_bitwise():
    A, D = _csr_small(seed=4)
    rT, cT, vT = oracle.csr_transpose(A.m, A.n, A.row_ptr, A.col, A.val)
    ref = A.to_scipy().T.tocsr()
    ref.sort_indices()
    assert np.array_equal(rT, ref.indptr)
    assert np.array_equal(cT, ref.indices)
    assert np.array_equal(vT, ref.data)


def test_transpose_zipf_bitwise():
    A = synth.zipf_csr(3000, 2000, 60000, seed=11)
    rT, cT, vT = oracle.csr_transpose(A.m, A.n, A.row_ptr, A.col, A.val)
    ref = A.to_scipy().T.tocsr()
    ref.sort_indices()
    assert np.array_equal(rT, ref.indptr)
    assert np.array_equal(cT, ref.indices)
    assert np.array_equal(vT, ref.data)


# ------------------------------------------------------------------ dense

def test_gram_matches_numpy():
    Cm = np.random.default_rng(5).standard_normal((300, 17))
    G = oracle.gram(Cm)
    assert np.allclose(G, Cm.T @ Cm, rtol=1e-13, atol=1e-12)
    assert np.array_equal(G, G.T)


def test_jacobi_2x2_closed_form():
    """2x2 symmetric: eigenvalues (a+c)/2 -+ sqrt(((a-c)/2)^2 + b^2)."""
    for a, b, c in [(2.0, 1.0, 3.0), (1.0, 1e-3, 1.0), (5.0, -2.0, -1.0), (1.0, 0.0, 4.0)]:
        ev, V, _ = oracle.jacobi_eig(np.array([[a, b], [b, c]]))
        mid, rad = (a + c) / 2, math.sqrt(((a - c) / 2) ** 2 + b * b)
        assert np.allclose(ev, [mid - rad, mid + rad], rtol=1e-15, atol=1e-15)
        G = np.array([[a, b], [b, c]])
        assert np.allclose(G @ V, V * ev, atol=1e-14)


def test_jacobi_diagonal_input():
    d = np.array([3.0, -1.0, 7.0, 0.5, 0.5])
    ev, V, sweeps = oracle.jacobi_eig(np.diag(d))
    assert np.array_equal(ev, np.sort(d))
    assert sweeps == 1
    assert np.array_equal(np.abs(V).sum(axis=0), np.ones(5))


@pytest.mark.parametrize("l", [3, 16, 30, 75, 120])
def test_jacobi_matches_lapack_eigh(l):
    rng = np.random.default_rng(l)
    B = rng.standard_normal((l + 5, l))
    G = B.T @ B
    ev, V, _ = oracle.jacobi_eig(G)
    ref = np.linalg.eigvalsh(G)
    nrm = np.linalg.norm(G, 2)
    assert np.abs(ev - ref).max() <= 50 * l * 2.2e-16 * nrm
    assert np.abs(V.T @ V - np.eye(l)).max() < 1e-13
    assert np.linalg.norm(G @ V - V * ev) <= 10 * l * 2.2e-16 * nrm


def test_eigsvd_matches_lapack_svd():
    """Alg. 3: S descending, U = C V S^-1 orthonormal, C = U S V^T."""
    rng = np.random.default_rng(8)
    Cm = rng.standard_normal((500, 24)) @ np.diag(np.logspace(0, -2, 24))
    U, S, V, deficient = oracle.eigsvd(Cm)
    ref = np.linalg.svd(Cm, compute_uv=False)
    kappa = ref[0] / ref[-1]
    assert not deficient
    assert np.all(np.diff(S) <= 0)
    assert np.abs(S - ref).max() / ref[0] <= 10 * 2.2e-16 * kappa**2 * 24
    assert np.abs(U.T @ U - np.eye(24)).max() < 1e-9
    assert np.allclose(U * S @ V.T, Cm, atol=1e-12)


def test_eigsvd_rank_deficient_zeroes_columns():
    rng = np.random.default_rng(9)
    Cm = rng.standard_normal((50, 3)) @ rng.standard_normal((3, 6))  # rank 3
    U, S, V, deficient = oracle.eigsvd(Cm)
    assert deficient
    assert np.all(U[:, 3:] == 0.0)
    assert np.allclose(U[:, :3] * S[:3] @ V[:, :3].T, Cm, atol=1e-10)


# ------------------------------------------------------------------ check + shift

def test_pve_ratio_hand_values():
    """eq. (19) with the surrogate E = S + alpha (Prop. 3): hand-computed."""
    S = np.array([4.0, 2.0, 1.0])
    Sp = np.array([3.0, 2.0, 0.5])
    # E = [4.5, 2.5], E' = [3.25, 2.25]; |diff| = [1.25, 0.25]; denom 1 + 0.5
    assert oracle.pve_ratio(2, S, Sp, 0.5, 0.25) == pytest.approx(1.25 / 1.5, rel=1e-15)
    # k = 1: only i = 1 counts; denominator S_2 + alpha = 2.5
    assert oracle.pve_ratio(1, S, Sp, 0.5, 0.25) == pytest.approx(1.25 / 2.5, rel=1e-15)


def test_shift_update_hand_values():
    """Alg. 5 step 6: strictly-greater test, midpoint update."""
    assert oracle.shift_update(np.array([5.0, 1.0]), 0.5) == 0.75
    assert oracle.shift_update(np.array([5.0, 0.4]), 0.5) == 0.5
    assert oracle.shift_update(np.array([5.0, 0.5]), 0.5) == 0.5


def _rank_l_matrix(g):
    rng = np.random.default_rng(123)
    m, n = g["m"], g["n"]
    sig = np.array(g["sigma"])
    Uo, _ = np.linalg.qr(rng.standard_normal((m, len(sig))))
    Vo, _ = np.linalg.qr(rng.standard_normal((n, len(sig))))
    D = (Uo * sig) @ Vo.T
    return synth.dense_to_csr(D), D, sig


@pytest.mark.parametrize("mode", ["R2", "R1", "NONE"])
def test_rank_l_shift_sequence_golden(mode):
    g = json.load(open(os.path.join(GOLDEN, "rank_l_shift_sequence.json")))
    A, D, sig = _rank_l_matrix(g)
    pol = oracle.SHIFT_NONE if mode == "NONE" else oracle.SHIFT_PAPER
    pm = oracle.PVE_R1 if mode == "R1" else oracle.PVE_R2
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, g["k"], g["s"], 10, g["tol"],
                       seed=4, shift_policy=pol, pve_mode=pm)
    exp = g[mode]
    assert r.passes == exp["passes"]
    assert np.allclose(r.alpha, exp["alpha_used"], rtol=1e-12, atol=1e-12)
    assert np.allclose(r.ratio, exp["ratio"], rtol=1e-12, atol=1e-12)
    if "s_hat_pass2" in exp:
        assert np.allclose(r.s_hat[1], exp["s_hat_pass2"], rtol=1e-12)
    assert np.allclose(r.S, sig[:g["k"]], rtol=1e-13)


# ------------------------------------------------------------------ end to end

def test_rank_l_exact_for_any_pass_count():
    """rank(A) = l: the sketch spans the row space, sigma_hat = sigma for any p."""
    g = json.load(open(os.path.join(GOLDEN, "rank_l_shift_sequence.json")))
    A, D, sig = _rank_l_matrix(g)
    for p in (0, 1, 3):
        r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 4, 2, p, 0.0, seed=9)
        assert np.allclose(r.S, sig[:4], rtol=1e-13)
        assert np.allclose(D @ r.V, r.U * r.S, atol=1e-12)


def test_small_config_converges_to_lapack():
    """2000 x 1500 uniform config: with many passes sigma_hat -> sigma (LAPACK)."""
    A = synth.config_small(np.float64)
    sv = np.linalg.svd(A.to_dense(), compute_uv=False)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 10, 60, 0.0, seed=2001)
    assert np.abs(r.S - sv[:20]).max() / sv[19] < 1e-10
    # Prop. 1: computed values lie under the exact ones at every pass count
    for p in (0, 2, 5):
        rp = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 10, p, 0.0, seed=2001)
        assert np.all(rp.S <= sv[:20] * (1 + 1e-12))


def test_invariants_props_1_2_3():
    """Prop. 2 via eq. (14): alpha nondecreasing and alpha_j <= sigma_l^2 / 2.
    Prop. 3: E_i(j) = S_i + alpha_j <= sigma_i^2.  Prop. 1: S_hat <= sigma.
    Alg. 3: S descending.  U, V orthonormal."""
    A = synth.config_small(np.float64)
    sv = np.linalg.svd(A.to_dense(), compute_uv=False)
    k, s = 20, 10
    l = k + s
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 12, 0.0, seed=2001)
    assert np.all(np.diff(r.alpha) >= 0)
    assert np.all(r.alpha <= sv[l - 1] ** 2 / 2 * (1 + 1e-12))
    E = r.s_hat + r.alpha[:, None]
    assert np.all(E <= (sv[:l] ** 2)[None, :] * (1 + 1e-12))
    assert np.all(np.diff(r.s_hat, axis=1) <= 0)
    assert np.all(r.S <= sv[:k] * (1 + 1e-12))
    assert np.abs(r.U.T @ r.U - np.eye(k)).max() < 1e-12
    assert np.abs(r.V.T @ r.V - np.eye(k)).max() < 1e-12


def test_known_sigma_block_diagonal():
    """Block-diagonal matrix under random permutations: exact sigma known."""
    rng = np.random.default_rng(21)
    blocks = [rng.standard_normal((int(rng.integers(3, 9)), int(rng.integers(2, 6))))
              * (1.0 / (1 + i)) for i in range(120)]
    A, sig = synth.block_diag_known_sigma(blocks, seed=5)
    assert A.m >= A.n
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 10, 10, 80, 0.0, seed=3)
    assert np.all(r.S <= sig[:10] * (1 + 1e-12))
    gaps_ok = (sig[:10] - sig[1:11]) / sig[:10] > 1e-3
    assert np.abs(r.S - sig[:10])[gaps_ok].max() / sig[0] < 1e-9


def test_wide_matrix_orientation():
    """m < n runs on A^T (Sec. 3.1): U and V exchange roles, sigma unchanged."""
    A, D = _csr_small(seed=12, m=40, n=70, density=0.4)
    sv = np.linalg.svd(D, compute_uv=False)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 5, 5, 40, 0.0, seed=1)
    assert r.U.shape == (40, 5) and r.V.shape == (70, 5)
    assert np.abs(r.S - sv[:5]).max() / sv[0] < 1e-10
    assert np.allclose(D @ r.V, r.U * r.S, atol=1e-10)


def test_tolerance_run_meets_pve():
    """At tol = 1e-2 the true eps_PVE ends about or below 1e-2 (Sec. 4.3)."""
    A = synth.config_small(np.float64)
    sv = np.linalg.svd(A.to_dense(), compute_uv=False)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 10, 64, 1e-2, seed=2001)
    assert r.converged
    pve, es = oracle.metrics(A.m, A.n, A.row_ptr, A.col, A.val, r.U, r.S, sv)
    assert pve <= 1e-2
    # the check cannot pass at the first pass: S' = 0 gives ratio >= 1
    assert r.ratio[0] >= 1.0


def test_theorem_1_bound():
    """Theorem 1, eq. (15) (with A -> A^T for the m >= n form): the basis Q
    after p passes satisfies ||A - A Q Q^T|| <= RHS with the shifts used."""
    rng = np.random.default_rng(31)
    m, n = 400, 300
    sig_t = 1.0 / np.sqrt(np.arange(1, n + 1))
    Uo, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Vo, _ = np.linalg.qr(rng.standard_normal((n, n)))
    D = (Uo * sig_t) @ Vo.T
    A = synth.dense_to_csr(D)
    k, s, p = 10, 10, 4
    l = k + s
    r = oracle.dashsvd(m, n, A.row_ptr, A.col, A.val, k, s, p, 0.0, seed=17)
    Q = r.Q
    err = np.linalg.norm(D - D @ Q @ Q.T, 2)
    # alpha_c for c = 1..p is the shift used in pass c
    al = r.alpha
    j = k // 2
    beta, gamma = 3.0, 3.0
    sig = sig_t
    prod1 = np.prod(((sig[j] ** 2 - al) / (sig[j - 1] ** 2 - al)) ** 2)
    prod2 = np.prod(((sig[k] ** 2 - al) / (sig[j - 1] ** 2 - al)) ** 2)
    rhs = 2 * math.sqrt((2 * l * l * beta**2 * gamma**2 * prod1 + 1) * sig[j] ** 2 +
                        (2 * l * (n - k) * beta**2 * gamma**2 * prod2 + 1) * sig[k] ** 2)
    assert err <= rhs
    # Corollary 2: the shifted bound is no larger than the unshifted one
    p1 = np.prod(((sig[j] ** 2) / (sig[j - 1] ** 2)) ** 2 * np.ones(p))
    p2 = np.prod(((sig[k] ** 2) / (sig[j - 1] ** 2)) ** 2 * np.ones(p))
    rhs0 = 2 * math.sqrt((2 * l * l * beta**2 * gamma**2 * p1 + 1) * sig[j] ** 2 +
                         (2 * l * (n - k) * beta**2 * gamma**2 * p2 + 1) * sig[k] ** 2)
    assert rhs <= rhs0 * (1 + 1e-15)


def test_dynamic_shift_beats_no_shift():
    """Fig. 1's claim: at equal p the dynamically shifted iteration gives
    lower eps_PVE than the unshifted one (Dense2-style sigma_i = 1/sqrt(i))."""
    rng = np.random.default_rng(41)
    m = n = 300
    sig = 1.0 / np.sqrt(np.arange(1, n + 1))
    Uo, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Vo, _ = np.linalg.qr(rng.standard_normal((n, n)))
    D = (Uo * sig) @ Vo.T
    A = synth.dense_to_csr(D)
    wins = 0
    trials = 10
    for sd in range(trials):
        rs = oracle.dashsvd(m, n, A.row_ptr, A.col, A.val, 10, 5, 4, 0.0, seed=100 + sd)
        r0 = oracle.dashsvd(m, n, A.row_ptr, A.col, A.val, 10, 5, 4, 0.0, seed=100 + sd,
                            shift_policy=oracle.SHIFT_NONE)
        e_s, _ = oracle.metrics(m, n, A.row_ptr, A.col, A.val, rs.U, rs.S, sig)
        e_0, _ = oracle.metrics(m, n, A.row_ptr, A.col, A.val, r0.U, r0.S, sig)
        wins += e_s <= e_0
    assert wins >= 9


def test_lapack_mirror_trace():
    """A second route to the same iteration: NumPy with LAPACK eigh in place
    of the Jacobi eig.  The per-pass S, shift and ratio must agree."""
    A = synth.uniform_csr(300, 200, 6000, seed=77, dtype=np.float64)
    D = A.to_dense()
    k, s, P = 8, 4, 6
    l = k + s
    om = oracle.gaussian(55, A.m, l)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, P, 0.0, omega=om)

    def eig_svd(Cm):
        w, V = np.linalg.eigh(Cm.T @ Cm)
        w, V = np.maximum(w[::-1], 0.0), V[:, ::-1]
        S = np.sqrt(w)
        return Cm @ V / S, S, V

    Q, _, _ = eig_svd(D.T @ om)
    alpha = 0.0
    for j in range(P):
        Q, S, _ = eig_svd(D.T @ (D @ Q) - alpha * Q)
        assert np.allclose(S, r.s_hat[j], rtol=1e-10)
        assert alpha == pytest.approx(r.alpha[j], rel=1e-10, abs=1e-14)
        if S[-1] > alpha:
            alpha = (S[-1] + alpha) / 2
    B = D @ Q
    Ub, Sb, Vb = eig_svd(B)
    assert np.allclose(Sb[:k], r.S, rtol=1e-11)


def test_schedule_policy_with_half_is_paper_rule():
    """A schedule of 0.5 everywhere reproduces the paper's shift rule."""
    A = synth.config_small(np.float64)
    r1 = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 10, 8, 0.0, seed=2001)
    r2 = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 10, 8, 0.0, seed=2001,
                        shift_policy=oracle.SHIFT_SCHEDULE, sched=np.full(9, 0.5))
    assert np.allclose(r1.alpha, r2.alpha, rtol=1e-15, atol=0)
    assert np.array_equal(r1.S, r2.S)


def test_invalid_arguments_rejected():
    A = synth.config_small(np.float64)
    with pytest.raises(ValueError):
        oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 0, 5, 0.0)
    with pytest.raises(ValueError):
        oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 1000, 1000, 5, 0.0)


def test_mlp_reference_gradient_matches_finite_differences():
    """The FP64 MLP reference used to check the HIP learned-shift kernels:
    its analytic gradient against central differences of its own loss."""
    from oracle import mlp_ref
    rng = np.random.default_rng(3)
    D, H = 9, 128
    n = H * D + H + H * H + H + 2 * H + 2
    P = rng.standard_normal(n) * 0.2
    X = rng.standard_normal((5, D))
    Y = np.stack([rng.uniform(0.5, 0.9, 5), rng.uniform(1.0, 3.0, 5)], axis=1)
    g = mlp_ref.grad(P, X, Y, D, H, 0.9)
    idx = rng.choice(n, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(n)
        e[i] = h
        fd = (mlp_ref.loss(P + e, X, Y, D, H, 0.9) - mlp_ref.loss(P - e, X, Y, D, H, 0.9)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


# ------------------------------------------------------------------ error metrics

def test_metrics_hand_rotated_vector():
    """Sec. 4 error metrics on a diagonal matrix with hand-known answers.
    A = diag(5, 4, 3, 2, 1) padded to 7 x 5, k = 2.  u_1 is the exact left
    vector e_1 rotated by theta towards e_4 (sigma 2), u_2 = e_2 exactly, so
    ||A^T u_1||^2 = 25 cos^2 + 4 sin^2 and eps_PVE = 21 sin^2 / sigma_3^2.
    Catches a denominator of sigma_k^2 (gives /16), a missing square, or the
    norm of A u instead of A^T u; eps_sigma divides by the exact sigma."""
    sig = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    D = np.zeros((7, 5))
    for i in range(5):
        D[i, i] = sig[i]
    A = synth.dense_to_csr(D)
    th = 0.3
    U = np.zeros((7, 2))
    U[0, 0], U[3, 0] = math.cos(th), math.sin(th)
    U[1, 1] = 1.0
    S = np.array([4.9, 4.1])
    pve, es = oracle.metrics(7, 5, A.row_ptr, A.col, A.val, U, S, sig)
    assert pve == pytest.approx(21.0 * math.sin(th) ** 2 / 9.0, rel=1e-14)
    assert es == pytest.approx(max(0.1 / 5.0, 0.1 / 4.0), rel=1e-13)


def test_metrics_match_dense_numpy():
    """The metrics against a direct dense computation: sigma from LAPACK svd,
    ||A^T u_i||^2 formed with a dense product, denominator sigma_{k+1}^2."""
    A, D = _csr_small(seed=90, m=60, n=45, density=0.3)
    sv = np.linalg.svd(D, compute_uv=False)
    k = 6
    rng = np.random.default_rng(91)
    U, _ = np.linalg.qr(np.linalg.svd(D)[0][:, :k] + 1e-3 * rng.standard_normal((60, k)))
    S = sv[:k] * (1 - 1e-4 * rng.random(k))
    pve, es = oracle.metrics(A.m, A.n, A.row_ptr, A.col, A.val, U, S, sv)
    nrm = np.linalg.norm(D.T @ U, axis=0) ** 2
    assert pve == pytest.approx(np.max(np.abs(sv[:k] ** 2 - nrm)) / sv[k] ** 2, rel=1e-10)
    assert es == pytest.approx(np.max(np.abs(sv[:k] - S) / sv[:k]), rel=1e-10)


# ------------------------------------------------------------------ shift policies

def _mirror(D, om, k, s, P, next_alpha):
    """NumPy/LAPACK route to the pass loop of Alg. 5 (tol = 0, reading R2);
    next_alpha(j, S, alpha, ratio) gives the shift set after pass j."""
    l = k + s

    def eig_svd(Cm):
        w, V = np.linalg.eigh(Cm.T @ Cm)
        w, V = np.maximum(w[::-1], 0.0), V[:, ::-1]
        Sv = np.sqrt(w)
        return Cm @ V / Sv, Sv

    Q, _ = eig_svd(D.T @ om)
    alpha, a_prev, Sp = 0.0, 0.0, np.zeros(l)
    al, ra = [], []
    for j in range(1, P + 1):
        Q, S = eig_svd(D.T @ (D @ Q) - alpha * Q)
        ratio = np.max(np.abs((Sp[:k] + a_prev) - (S[:k] + alpha))) / (S[k] + alpha)
        al.append(alpha)
        ra.append(ratio)
        a_prev, Sp = alpha, S
        alpha = next_alpha(j, S, alpha, ratio)
    return np.array(al), np.array(ra)


def test_fixed_policy_lapack_mirror():
    """Alg. 2* of Sec. 4.1: the shift is set by the rule after the first pass
    and then frozen.  The oracle's FIXED trace against a LAPACK mirror, and
    the trace differs from the paper's rule (which keeps moving the shift),
    so a FIXED branch that fell through to the paper's rule fails here."""
    A = synth.uniform_csr(300, 200, 6000, seed=77, dtype=np.float64)
    D = A.to_dense()
    k, s, P = 8, 4, 6
    om = oracle.gaussian(55, A.m, k + s)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, P, 0.0, omega=om,
                       shift_policy=oracle.SHIFT_FIXED)

    def nxt(j, S, a, ratio):
        return (S[-1] + a) / 2 if (j == 1 and S[-1] > a) else a
    al, ra = _mirror(D, om, k, s, P, nxt)
    assert np.allclose(r.alpha, al, rtol=1e-10, atol=1e-14)
    assert np.allclose(r.ratio, ra, rtol=1e-8)
    assert r.alpha[1] > 0 and np.all(r.alpha[1:] == r.alpha[1])
    rp = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, P, 0.0, omega=om)
    assert rp.alpha[-1] > r.alpha[-1] * 1.1


def test_schedule_lapack_mirror_with_guard_trip():
    """The schedule policy with c = 0.9 from the second pass on, against a
    LAPACK mirror that applies the guard written out independently.  The
    ratio grows at pass 6 (0.007 -> 0.15) so the guard drops the schedule
    there; without the guard the shift would keep rising."""
    A = synth.uniform_csr(300, 200, 6000, seed=77, dtype=np.float64)
    D = A.to_dense()
    k, s, P = 8, 4, 8
    l = k + s
    om = oracle.gaussian(55, A.m, l)
    sched = np.array([0.5] + [0.9] * P)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, P, 0.0, omega=om,
                       shift_policy=oracle.SHIFT_SCHEDULE, sched=sched)
    st = {"off": False, "pr": None, "pe": None, "trip": None}

    def nxt(j, S, a, ratio):
        ek1 = S[k] + a
        if j >= 2 and (ratio > st["pr"] or ek1 < st["pe"]) and not st["off"]:
            st["off"], st["trip"] = True, j
        st["pr"], st["pe"] = ratio, ek1
        c = 0.5 if st["off"] else sched[j]
        return max(a, c * (S[-1] + a))
    al, ra = _mirror(D, om, k, s, P, nxt)
    assert st["trip"] == 6
    assert np.allclose(r.alpha, al, rtol=1e-10, atol=1e-14)
    assert np.allclose(r.ratio, ra, rtol=1e-7)
    # after the trip 0.5 * E_l stays under the shift, which then stays put;
    # the unguarded rule would have moved it to 0.9 * E_l
    assert r.alpha[7] == r.alpha[6] == r.alpha[5]
    E_l6 = r.s_hat[5][-1] + r.alpha[5]
    assert 0.9 * E_l6 > r.alpha[6] * 1.01


def test_schedule_rank_l_hand_derived():
    """Rank exactly l (the golden matrix): every pass's block has singular
    values sigma_i^2 - alpha (Prop. 2).  With c_1 = 0.8 the shift set after
    pass 1 is 0.8 * E_l = 0.8 * 9 = 7.2, not the paper's 4.5, and pass 2's
    S is sigma^2 - 7.2 = [92.8, 56.8, 28.8, 17.8, 8.8, 1.8]."""
    g = json.load(open(os.path.join(GOLDEN, "rank_l_shift_sequence.json")))
    A, D, sig = _rank_l_matrix(g)
    sched = np.array([0.5, 0.8, 0.8])
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, g["k"], g["s"], 2, 0.0, seed=4,
                       shift_policy=oracle.SHIFT_SCHEDULE, sched=sched)
    assert r.passes == 2
    assert np.allclose(r.alpha, [0.0, 7.2], rtol=1e-12, atol=1e-13)
    assert np.allclose(r.s_hat[1], [92.8, 56.8, 28.8, 17.8, 8.8, 1.8], rtol=1e-11)
    assert r.ratio[0] == pytest.approx(6.25, rel=1e-12)
    assert np.allclose(r.S, sig[:g["k"]], rtol=1e-13)


def test_schedule_shift_hand_trajectories():
    """The schedule step on fabricated scalar trajectories: each guard
    criterion fires alone, the guard never fires at pass 1, and once off it
    stays off.  Values computed by hand."""
    f = oracle.schedule_shift
    # pass 1: no guard; 0.8 * 10 = 8 > 1
    assert f(1, 5.0, 0.0, 3.0, 0.0, 10.0, 1.0, 0.8, False) == (8.0, False)
    # pass 2, ratio down and E_{k+1} up: schedule kept, 0.7 * 12 = 8.4
    assert f(2, 0.5, 5.0, 3.5, 3.0, 12.0, 8.0, 0.7, False) == (pytest.approx(8.4), False)
    # candidate below the shift: the shift never decreases
    assert f(2, 0.5, 5.0, 3.5, 3.0, 12.0, 9.0, 0.7, False) == (9.0, False)
    # ratio grows: guard fires, 0.5 * 20 = 10
    assert f(3, 0.6, 0.5, 3.6, 3.5, 20.0, 8.4, 0.9, False) == (10.0, True)
    # E_{k+1} shrinks alone: guard fires, 0.5 * 20 = 10
    assert f(3, 0.4, 0.5, 3.4, 3.5, 20.0, 8.4, 0.9, False) == (10.0, True)
    # once off it stays off even when both criteria are fine
    assert f(4, 0.1, 0.4, 3.7, 3.4, 30.0, 10.0, 0.9, True) == (15.0, True)
    # equal values do not fire the guard (strict comparisons)
    assert f(3, 0.5, 0.5, 3.5, 3.5, 20.0, 8.4, 0.9, False) == (18.0, False)


def test_mlp_reference_forward_hand_values():
    """The MLP reference's forward pass on weights chosen so every layer can
    be done by hand (D = 2, H = 2): W1 = [[1, -1], [2, 0]], b1 = [0, -1],
    W2 = I, b2 = [0.5, 0], W3 = [[1, 1], [0, 2]], b3 = [0, 0.25].  For
    x = (3, 1): h1 = relu(2, 5) = (2, 5); h2 = (2.5, 5); o = (7.5, 10.25).
    For x = (0, 1): h1 = relu(-1, -1) = 0; h2 = (0.5, 0); o = (0.5, 0.25)."""
    from oracle import mlp_ref
    P = np.array([1, -1, 2, 0, 0, -1, 1, 0, 0, 1, 0.5, 0, 1, 1, 0, 2, 0, 0.25], dtype=float)
    X = np.array([[3.0, 1.0], [0.0, 1.0]])
    o = mlp_ref.forward(P, X, 2, 2)[2]
    assert np.array_equal(o, [[7.5, 10.25], [0.5, 0.25]])
    c = mlp_ref.outputs(P, X, 2, 2, 0.9)[:, 0]
    assert np.allclose(c, 0.5 + 0.4 / (1 + np.exp(-np.array([7.5, 0.5]))), rtol=1e-15)


# ------------------------------------------------------------------ control without the surrogate

def test_nosurr_lapack_mirror():
    """Accuracy control without the surrogate (Sec. 4.3, Table 3): after
    each pass the singular values of B = A Q are computed and eq. (18) is
    checked on their squares, E' starting at zero.  A NumPy mirror that takes
    sigma(B) from LAPACK's SVD of B itself (not from the eig of its Gram)
    must give the same per-pass ratios, stopping pass and final sigma.  A
    ratio on sigma instead of sigma^2, on the surrogate S + alpha, with
    E_k in place of E_{k+1} in the denominator, or with B formed from the
    Q before the pass instead of after it, fails here."""
    A = synth.uniform_csr(300, 200, 6000, seed=77, dtype=np.float64)
    D = A.to_dense()
    k, s, tol = 8, 4, 1e-3
    l = k + s
    om = oracle.gaussian(55, A.m, l)
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 30, tol, omega=om,
                       pve_mode=oracle.PVE_NOSURR)

    def eig_svd(Cm):
        w, V = np.linalg.eigh(Cm.T @ Cm)
        w, V = np.maximum(w[::-1], 0.0), V[:, ::-1]
        Sv = np.sqrt(w)
        return Cm @ V / Sv, Sv

    Q, _ = eig_svd(D.T @ om)
    alpha, Ep, ratios = 0.0, np.zeros(l), []
    for j in range(1, 31):
        Q, S = eig_svd(D.T @ (D @ Q) - alpha * Q)
        E = np.linalg.svd(D @ Q, compute_uv=False) ** 2
        ratio = np.max(np.abs(Ep[:k] - E[:k])) / E[k]
        ratios.append(ratio)
        assert r.alpha[j - 1] == pytest.approx(alpha, rel=1e-10, abs=1e-14)
        if ratio <= tol:
            break
        Ep = E
        if S[-1] > alpha:
            alpha = (S[-1] + alpha) / 2
    assert r.converged and r.passes == len(ratios) >= 3
    assert np.allclose(r.ratio, ratios, rtol=1e-7, atol=1e-15)
    assert min(abs(np.log(np.array(ratios) / tol))) > 0.05  # no borderline pass
    sb = np.linalg.svd(D @ Q, compute_uv=False)
    assert np.allclose(r.S, sb[:k], rtol=1e-11)


def test_nosurr_rank_l_closed_form():
    """rank(A) = l: the sketch already spans the row space, so sigma(A Q) =
    sigma(A) from the first pass on.  The first check compares with E' = 0:
    ratio_1 = sigma_1^2 / sigma_{k+1}^2 exactly; the second finds no change
    (ratio_2 ~ 0) and stops, N_p = 2 at any tol."""
    g = json.load(open(os.path.join(GOLDEN, "rank_l_shift_sequence.json")))
    A, D, sig = _rank_l_matrix(g)
    k, s = g["k"], g["s"]
    for tol in (1e-2, 1e-8):
        r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 10, tol, seed=4,
                           pve_mode=oracle.PVE_NOSURR)
        assert r.passes == 2 and r.converged
        assert r.ratio[0] == pytest.approx(sig[0] ** 2 / sig[k] ** 2, rel=1e-12)
        assert r.ratio[1] <= 1e-11
        assert np.allclose(r.S, sig[:k], rtol=1e-13)


def test_nosurr_stops_at_or_one_before_the_surrogate():
    """Table 3's observation: without the surrogate, N_p is the same or one
    smaller (the surrogate lags sigma(A Q)^2 by about a pass, Prop. 3).
    Checked on the 2000 x 1500 workload and a power-law matrix at three
    tolerances."""
    cases = [(synth.config_small(np.float64), 20, 10, 2001),
             (synth.zipf_csr(20000, 12000, 400000, seed=21), 50, 25, 3)]
    for A, k, s, seed in cases:
        for tol in (1e-1, 1e-2, 1e-3):
            r2 = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 30, tol, seed=seed)
            rn = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 30, tol, seed=seed,
                                pve_mode=oracle.PVE_NOSURR)
            assert r2.converged and rn.converged
            assert r2.passes - 1 <= rn.passes <= r2.passes, (tol, r2.passes, rn.passes)


# ------------------------------------------------------------------ residual and spectral metrics

def test_residual_metrics_hand_diagonal():
    """A = diag(5, 4, 3, 2, 1) padded to 7 x 5, k = 2, v_1 = e_1, v_2 = e_2,
    u_1 = e_1 rotated by theta towards e_4, u_2 = e_2, s = (4.9, 4):
      A^T u_1 - s_1 v_1 = (5 cos - 4.9) e_1 + 2 sin e_4, so
      eps_res = sqrt((5 cos - 4.9)^2 + 4 sin^2) / 5;
    with theta = 0 the rank-2 part is exact but for s_1: E = diag(0.1, 0, 3,
    2, 1) and ||E||_2 = 3 = sigma_3, eps_spec = 0.  Catches a residual
    divided by s_i instead of sigma_i, A u in place of A^T u, and a norm
    of the wrong residual."""
    sig = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    D = np.zeros((7, 5))
    for i in range(5):
        D[i, i] = sig[i]
    A = synth.dense_to_csr(D)
    V = np.zeros((5, 2))
    V[0, 0] = V[1, 1] = 1.0
    S = np.array([4.9, 4.0])
    for th in (0.0, 0.3):
        U = np.zeros((7, 2))
        U[0, 0], U[3, 0] = math.cos(th), math.sin(th)
        U[1, 1] = 1.0
        er, es, en, _ = oracle.residual_metrics(7, 5, A.row_ptr, A.col, A.val, U, S, V, sig)
        assert er == pytest.approx(math.sqrt((5 * math.cos(th) - 4.9) ** 2 + 4 * math.sin(th) ** 2) / 5.0,
                                   rel=1e-13)
        E = D - (U * S) @ V.T
        assert en == pytest.approx(np.linalg.norm(E, 2), rel=1e-12)
        if th == 0.0:
            assert en == pytest.approx(3.0, rel=1e-14) and abs(es) <= 1e-14


@pytest.mark.parametrize("shape", [(60, 45), (45, 60), (300, 200)])
def test_residual_metrics_match_dense_numpy(shape):
    """Both metrics against a direct dense computation: ||A^T u_i - s_i v_i||
    from dense products, ||A - U S V^T||_2 from LAPACK's SVD of the dense
    residual, sigma from LAPACK."""
    m, n = shape
    A, D = _csr_small(seed=m + n, m=m, n=n, density=0.3)
    Uf, sv, Vt = np.linalg.svd(D)
    k = 6
    rng = np.random.default_rng(92)
    U, _ = np.linalg.qr(Uf[:, :k] + 1e-3 * rng.standard_normal((m, k)))
    V, _ = np.linalg.qr(Vt[:k].T + 1e-3 * rng.standard_normal((n, k)))
    S = sv[:k] * (1 - 1e-4 * rng.random(k))
    er, es, en, steps = oracle.residual_metrics(m, n, A.row_ptr, A.col, A.val, U, S, V, sv)
    res = np.linalg.norm(D.T @ U - V * S, axis=0) / sv[:k]
    assert er == pytest.approx(res.max(), rel=1e-10)
    ref = np.linalg.norm(D - (U * S) @ V.T, 2)
    assert en == pytest.approx(ref, rel=1e-11)
    assert es == pytest.approx((ref - sv[k]) / sv[k], rel=1e-8, abs=1e-12)
    assert es > 0 and steps <= min(m, n)


def test_spectral_norm_lanczos_clustered_spectrum():
    """Lanczos on E^T E when the top of the residual's spectrum is a tight
    cluster (sigma_{k+1} and sigma_{k+2} 1e-6 apart): the estimate is a
    lower bound and reaches ||E||_2 to 1e-12 within the step budget."""
    rng = np.random.default_rng(31)
    m, n = 120, 90
    sig = np.concatenate([[9.0, 8.0, 7.0], [3.0, 3.0 - 3e-6], np.linspace(2.5, 0.1, n - 5)])
    Uo, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Vo, _ = np.linalg.qr(rng.standard_normal((n, n)))
    D = (Uo * sig) @ Vo.T
    A = synth.dense_to_csr(D)
    k = 3
    er, es, en, steps = oracle.residual_metrics(m, n, A.row_ptr, A.col, A.val, Uo[:, :k], sig[:k],
                                                Vo[:, :k], sig, steps=90)
    assert en <= 3.0 * (1 + 1e-13)
    assert en == pytest.approx(3.0, rel=1e-12)
    assert abs(es) <= 1e-12 and er <= 1e-13

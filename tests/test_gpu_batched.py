"""Batched form (dashsvd_run_batched): every matrix of the batch must give
what Alg. 5 gives on it alone.  Matrix i draws Omega from the Philox stream
keyed (seed + i, 0), so the oracle (and the single-matrix library path) can
reproduce each member; the batch mixes sizes, power-law and uniform
structure, long rows and ragged tails."""
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


def _batch(dtype=np.float64):
    mats = [
        synth.uniform_csr(700, 500, 9000, seed=51, dtype=dtype),
        synth.zipf_csr(3000, 1200, 40000, seed=52),
        synth.uniform_csr(129, 64, 2000, seed=53, dtype=dtype),
        synth.zipf_csr(1500, 1500, 30000, seed=54),
        synth.uniform_csr(2049, 333, 12000, seed=55, dtype=dtype),
        synth.zipf_csr(900, 450, 20000, seed=56),
    ]
    for A in mats:
        A.val = A.val.astype(dtype)
    return mats


def _vec_close(X, Xref, tol):
    d = np.minimum(np.abs(X - Xref).max(axis=0), np.abs(X + Xref).max(axis=0))
    return d.max() <= tol


def _run(mats, k, s, pmax, tol, seed, precision, **kw):
    from paper_2404_09276_amd import DashSVD
    h = DashSVD(precision=precision, p_max=pmax, seed=seed, **kw)
    st = h.run_batched(mats, k, s, tol)
    out = [(h.get_usv_batched(i), h.info_batched(i)) for i in range(len(mats))]
    summary = h.info_batched(-1)
    h.close()
    return st, out, summary


def test_batched_fp64_matches_oracle_per_matrix(torch_dev):
    mats = _batch(np.float64)
    st, out, summary = _run(mats, 8, 4, 4, 0.0, 300, "fp64")
    assert st == 0 and summary.passes == 4
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 8, 4, 4, 0.0, seed=300 + i)
        assert info.passes == 4
        assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-10, i
        assert np.allclose(info.alpha_used, ref.alpha, rtol=1e-10, atol=0), i
        assert _vec_close(U, ref.U, 1e-8) and _vec_close(V, ref.V, 1e-8), i


def test_batched_onesided_matches_oracle_per_matrix(torch_dev):
    """eig_method ONESIDED in the batched form (one workgroup of the one-sided
    kernel per member, the two-sided kernel gated on each member's decline
    flag): every member against the oracle, FP64, fixed passes."""
    mats = _batch(np.float64)
    st, out, summary = _run(mats, 8, 4, 4, 0.0, 300, "fp64", eig_method="onesided")
    assert st == 0 and summary.passes == 4
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 8, 4, 4, 0.0, seed=300 + i)
        assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-10, i
        assert np.allclose(info.alpha_used, ref.alpha, rtol=1e-10, atol=0), i
        assert _vec_close(U, ref.U, 1e-8) and _vec_close(V, ref.V, 1e-8), i


def _groups(mats, lim):
    """The library's grouping rule: consecutive members, at most lim nonzeros."""
    g, z = [], 0
    for A in mats:
        if not g or z + A.nnz > lim:
            g.append(0)
            z = 0
        g[-1] += 1
        z += A.nnz
    return g


@pytest.mark.parametrize("lim", [45000, 70000])
def test_batched_sub_batches_match_oracle_and_whole_batch(torch_dev, lim):
    """batch_nnz_max below the batch's total: the members run in consecutive
    sub-batches (each its own stacked operator in the arena) and their
    results are gathered; every member still draws Omega from seed + its
    index in the whole batch, so it matches the oracle and the one-group run."""
    mats = _batch(np.float64)
    groups = _groups(mats, lim)
    assert len(groups) > 1
    st, out, summary = _run(mats, 8, 4, 4, 0.0, 300, "fp64", batch_nnz_max=lim)
    st1, out1, summary1 = _run(mats, 8, 4, 4, 0.0, 300, "fp64")
    assert st == 0 and st1 == 0
    assert summary.sub_batches == len(groups) and summary1.sub_batches == 1
    assert summary.passes == 4
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        (U1, S1, V1), info1 = out1[i]
        ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 8, 4, 4, 0.0, seed=300 + i)
        assert info.passes == 4
        assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-10, i
        assert np.abs(S - S1).max() / S1.max() <= 1e-12, i
        assert np.allclose(info.alpha_used, ref.alpha, rtol=1e-10, atol=0), i
        assert _vec_close(U, ref.U, 1e-8) and _vec_close(V, ref.V, 1e-8), i


def test_batched_sub_batches_tolerance_and_oversized_member(torch_dev):
    """Tolerance runs stop each member at its own pass across sub-batches;
    a member above the limit is an argument error."""
    from paper_2404_09276_amd import DashSVD, DashSVDError
    mats = _batch(np.float64)
    st, out, summary = _run(mats, 8, 4, 30, 1e-3, 400, "fp64", batch_nnz_max=45000)
    assert st == 0 and summary.converged and summary.sub_batches > 1
    passes = []
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 8, 4, 30, 1e-3, seed=400 + i)
        if not np.any(np.abs(ref.ratio - 1e-3) < 1e-6 * 1e-3):
            assert info.passes == ref.passes, i
        assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-10, i
        passes.append(info.passes)
    assert summary.passes == max(passes)
    h = DashSVD(precision="fp64", p_max=4, seed=1, batch_nnz_max=10000)
    with pytest.raises(DashSVDError):
        h.run_batched(mats, 8, 4, 0.0)
    h.close()


@pytest.mark.parametrize("every", [3, 100])
def test_batched_passes_per_graph_launch(torch_dev, every):
    """check_interval passes captured as one graph (all p_max passes in one
    launch when check_interval >= p_max, a shorter last chunk captured
    again): the same results as one pass per launch, bit for bit."""
    mats = _batch(np.float32)
    st1, out1, s1 = _run(mats, 8, 4, 7, 0.0, 600, "fp32", check_interval=1)
    st, out, s = _run(mats, 8, 4, 7, 0.0, 600, "fp32", check_interval=every)
    assert st == st1 == 0
    assert s1.graph_launches == 7 and s.graph_launches == -(-7 // every)
    for i in range(len(mats)):
        (U, S, V), _ = out[i]
        (U1, S1, V1), _ = out1[i]
        assert np.array_equal(S, S1) and np.array_equal(U, U1) and np.array_equal(V, V1), i


@pytest.mark.parametrize("mode", ["r2", "r1"])
def test_batched_tolerance_each_matrix_stops_at_its_own_pass(torch_dev, mode):
    mats = _batch(np.float64)
    pm = oracle.PVE_R1 if mode == "r1" else oracle.PVE_R2
    st, out, summary = _run(mats, 8, 4, 30, 1e-3, 400, "fp64", pve_mode=mode)
    assert st == 0 and summary.converged
    passes = []
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 8, 4, 30, 1e-3, seed=400 + i, pve_mode=pm)
        borderline = np.any(np.abs(ref.ratio - 1e-3) < 1e-6 * 1e-3)
        if not borderline:
            assert info.passes == ref.passes, i
            assert np.allclose(info.ratio, ref.ratio, rtol=1e-8, atol=0), i
        assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-10, i
        passes.append(info.passes)
    assert summary.passes == max(passes)


def test_batched_fp32_matches_single_matrix_runs(torch_dev):
    """Members of an FP32 batch against dashsvd_run on each matrix alone with
    the same Omega stream (same algorithm, different kernels for the small
    dense steps)."""
    from paper_2404_09276_amd import DashSVD
    mats = _batch(np.float32)
    st, out, summary = _run(mats, 10, 6, 40, 1e-2, 500, "fp32")
    assert st == 0
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        h = DashSVD(precision="fp32", p_max=40, seed=500 + i)
        U1, S1, V1, st1, info1 = h.solve(A, 10, 6, 1e-2)
        h.close()
        assert info.passes == info1.passes, i
        assert np.all(np.abs(S - S1) / S1 <= 1e-5), i
        assert np.abs(U.T @ U - np.eye(10)).max() < 1e-5


@pytest.mark.parametrize("prec,bar", [("fp32", 1e-5), ("bf16", 5e-3)])
def test_batched_members_match_oracle(torch_dev, prec, bar):
    """Every member of an FP32 or BF16 batch against the FP64 oracle on that
    matrix alone with the member's Omega stream (seed + i).  FP32: the same
    pass count as the oracle's tolerance run and sigma within 1e-5 relative.
    BF16 panels (8-bit significand, relative rounding 2^-9 on every panel
    entry): sigma within 5e-3 (2.5 x 2^-9) relative of the oracle run for the member's own
    pass count, and every member converged."""
    mats = _batch(np.float32) + synth.batched_zipf(6, rows=(1000, 6000), seed=5100)
    st, out, summary = _run(mats, 10, 6, 40, 1e-2, 500, prec)
    assert st in (0, 2) and summary.converged
    worst = 0.0
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        assert info.converged, i
        if prec == "fp32":
            ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 10, 6, 40, 1e-2, seed=500 + i)
            borderline = np.any(np.abs(ref.ratio - 1e-2) < 1e-6 * 1e-2)
            if not borderline:
                assert info.passes == ref.passes, i
        else:
            ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 10, 6, info.passes, 0.0,
                                 seed=500 + i)
        rel = np.abs(S - ref.S) / ref.S
        worst = max(worst, float(rel.max()))
        assert np.all(rel <= bar), (i, rel.max())
    print(f"batched {prec}: worst member sigma rel err vs oracle {worst:.2e}", flush=True)


def test_batched_bf16_power_law_batch(torch_dev):
    """A batch shaped like the paper-scale batched workload (rows 1k-10k,
    columns 0.5-1 x rows, density 0.05-1 %, Zipf 1.1 degrees), k = 16,
    oversampling 8, BF16 panels, tol 1e-2: every member converges and meets
    the output identity A V = U diag(S) of the final Rayleigh-Ritz step."""
    mats = synth.batched_zipf(24, rows=(1000, 10000), seed=5000)
    st, out, summary = _run(mats, 16, 8, 16, 1e-2, 700, "bf16")
    assert st == 0 and summary.converged
    for i, A in enumerate(mats):
        (U, S, V), info = out[i]
        assert info.converged and 2 <= info.passes <= 16
        AV = oracle.csr_spmm(A.row_ptr, A.col, A.val, V)
        err = np.abs(AV - U * S[None, :]).max(axis=0) / S
        assert err.max() <= 5e-3, (i, err.max())
        assert np.all(np.diff(S) <= 0)


def test_batched_graph_replays_match_eager_fixed_passes(torch_dev):
    """p_max passes run as p_max replays of one captured pass: results after 1,
    2 and 5 replays each match the oracle at that pass count."""
    mats = _batch(np.float64)[:3]
    for p in (1, 2, 5):
        st, out, summary = _run(mats, 8, 4, p, 0.0, 900, "fp64")
        for i, A in enumerate(mats):
            (U, S, V), info = out[i]
            ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 8, 4, p, 0.0, seed=900 + i)
            assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-10, (p, i)


def test_batched_errors(torch_dev):
    from paper_2404_09276_amd import DashSVD, DashSVDError
    mats = _batch(np.float64)
    h = DashSVD(precision="fp64", p_max=3)
    wide = synth.uniform_csr(300, 700, 5000, seed=3, dtype=np.float64)
    with pytest.raises(DashSVDError) as e:
        h.run_batched(mats[:2] + [wide], 8, 4, 0.0)
    assert e.value.status == -1
    with pytest.raises(DashSVDError) as e:
        h.run_batched(mats[:2], 40, 30, 0.0)
    assert e.value.status == -1
    bad = synth.CSR(mats[0].m, mats[0].n, mats[0].row_ptr, mats[0].col.copy(), mats[0].val)
    bad.col[5] = mats[0].n  # inside the stacked column range, outside its own
    with pytest.raises(DashSVDError) as e:
        h.run_batched([mats[1], bad], 8, 4, 0.0)
    assert e.value.status == -2
    # still usable
    assert h.run_batched(mats[:2], 8, 4, 0.0) == 0
    h.close()


def test_autotune_writes_and_applies_database(torch_dev, tmp_path):
    """dashsvd_autotune searches the chunk length, the lane vectors, the
    column slabs and (single matrix) the degree order for a single matrix and
    for a batch, appends "key T lanes slab_kib reorder" to the database, and
    a handle that reads the database runs with those knobs; results stay
    within rounding of the default configuration.  Options that fix a knob
    keep it."""
    from paper_2404_09276_amd import DashSVD
    db = str(tmp_path / "tune.txt")
    A = synth.zipf_csr(20000, 9000, 400000, seed=61)
    mats = synth.batched_zipf(8, rows=(1000, 4000), seed=6100)
    h = DashSVD(precision="fp32", p_max=6, seed=3)
    t1 = h.autotune(A, 16, 8, db)
    t2 = h.autotune(mats, 16, 8, db)
    h.close()
    cands = {32, 64, 128, 256, 512, 768, 1024}
    assert t1 in cands and t2 in cands
    lines = [ln.split() for ln in open(db).read().split("\n") if ln]
    assert len(lines) == 2 and lines[0][0].endswith("_s") and lines[1][0].endswith("_b")
    (T1, v1, s1, r1), (T2, v2, s2, r2) = [tuple(int(x) for x in ln[1:]) for ln in lines]
    assert (T1, T2) == (t1, t2) and v1 in (1, 2) and v2 in (1, 2) and s1 in (0, 2048) and s2 in (0, 2048)
    assert r1 in (1, -1) and r2 == 0
    h = DashSVD(precision="fp32", p_max=6, seed=3, tuning_db=db)
    U, S, V, st, info = h.solve(A, 16, 8, 0.0)
    assert (info.long_row_used, info.lane_vectors_used, info.slab_kib_used) == (T1, v1, s1)
    assert info.reordered == (r1 > 0)
    h.run_batched(mats, 16, 8, 0.0)
    sb = h.info_batched(-1)
    assert (sb.long_row_used, sb.lane_vectors_used, sb.slab_kib_used) == (T2, v2, s2)
    h.close()
    h = DashSVD(precision="fp32", p_max=6, seed=3)
    U0, S0, V0, st0, info0 = h.solve(A, 16, 8, 0.0)
    h.close()
    assert info0.long_row_used == 128 and info0.lane_vectors_used == 1 and info0.slab_kib_used == 0
    assert np.all(np.abs(S - S0) / S0 <= 1e-5)
    # a fixed knob stays fixed
    h = DashSVD(precision="fp32", p_max=6, seed=3, lane_vectors=2, long_row=256)
    assert h.autotune(A, 16, 8, None) == 256
    U2, S2, V2, st2, info2 = h.solve(A, 16, 8, 0.0)
    assert info2.lane_vectors_used == 2 and info2.long_row_used == 256
    assert np.all(np.abs(S2 - S0) / S0 <= 1e-5)
    h.close()


def test_batched_bf16_promotion_guard(torch_dev):
    """A batch whose member plateaus above tol with BF16 panels (a very sparse
    power-law matrix, about 2 nonzeros per row): the stagnation guard moves the
    batch to FP32 panels, every member then meets tol, and the stagnant member
    matches its single-matrix FP32 run."""
    from paper_2404_09276_amd import DashSVD
    mats = synth.batched_zipf(1, rows=(1000, 10000), seed=5230) + synth.batched_zipf(5, rows=(1000, 4000), seed=5600)
    assert mats[0].nnz < 3 * mats[0].m
    st, out, summary = _run(mats, 16, 8, 24, 1e-2, 800, "bf16")
    # status 2 (RANK_DEFICIENT, results valid) is allowed: the sparse member
    # has numerically zero singular values inside its block
    assert st in (0, 2) and summary.converged and summary.promoted
    (U, S, V), info = out[0]
    h = DashSVD(precision="fp32", p_max=24, seed=800)
    U1, S1, V1, st1, info1 = h.solve(mats[0], 16, 8, 1e-2)
    h.close()
    assert info1.converged
    assert np.all(np.abs(S - S1) / S1 <= 2e-2)

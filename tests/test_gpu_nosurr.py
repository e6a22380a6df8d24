"""Accuracy control without the surrogate (pve_mode NOSURR, the comparison of
Sec. 4.3 / Table 3) on the GPU against the FP64 oracle: after every pass the
singular values of B = A Q, eq. (18) on their squares.

Bars: equal N_p (unless a ratio lies within 1e-6 tol of tol), sigma within
1e-10 (FP64) / 1e-5 (FP32) relative, per-pass shifts within the same bars,
per-pass ratios within 1e-9 relative (FP64) or, in FP32, within
1e-4 E_1 / E_k absolute (the ratio is a difference of squared singular
values of size up to E_1 divided by E_{k+1}, each carrying the FP32 panels'
~1e-6 relative rounding; E_1 / E_k stands in for E_1 / E_{k+1}, which the
returned k values do not give, hence the extra factor)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _solve(A, k, s, p_max, tol, seed, precision, **kw):
    from paper_2404_09276_amd import DashSVD
    h = DashSVD(precision=precision, p_max=p_max, seed=seed, **kw)
    U, S, V, st, info = h.solve(A, k, s, tol)
    h.close()
    return U, S, V, st, info


def _ratio_bar(ref, k, prec):
    if prec == "fp64":
        return 1e-9 * np.abs(ref.ratio) + 1e-14
    E = ref.S[0] ** 2 / ref.S[k - 1] ** 2
    return np.full(ref.ratio.shape, 1e-4 * E)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("eig", ["auto", "jacobi"])
@pytest.mark.parametrize("tol", [1e-2, 1e-3])
def test_nosurr_small_matches_oracle(torch_dev, prec, eig, tol):
    A = synth.config_small(np.float64 if prec == "fp64" else np.float32)
    k, s = 20, 10
    ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 64, tol, seed=2001,
                         pve_mode=oracle.PVE_NOSURR)
    U, S, V, st, info = _solve(A, k, s, 64, tol, 2001, prec, pve_mode="nosurr", eig_method=eig)
    assert st == 0 and info.converged and ref.converged
    assert info.passes == ref.passes
    bar = 1e-10 if prec == "fp64" else 1e-5
    assert np.all(np.abs(S - ref.S) / ref.S <= bar)
    assert np.allclose(info.alpha_used, ref.alpha, rtol=bar, atol=0)
    assert np.all(np.abs(info.ratio - ref.ratio) <= _ratio_bar(ref, k, prec))


def test_nosurr_degree_ordered_power_law_fp32(torch_dev):
    """A power-law matrix through the degree order and the long-row chunks."""
    A = synth.zipf_csr(30000, 12000, 500000, seed=42012)
    k, s, tol = 20, 10, 1e-2
    ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, 64, tol, seed=23,
                         pve_mode=oracle.PVE_NOSURR)
    U, S, V, st, info = _solve(A, k, s, 64, tol, 23, "fp32", pve_mode="nosurr", reorder=True)
    assert st == 0 and info.converged and info.passes == ref.passes
    assert np.all(np.abs(S - ref.S) / ref.S <= 1e-5)
    assert np.all(np.abs(info.ratio - ref.ratio) <= _ratio_bar(ref, k, "fp32"))


def test_nosurr_rank_l_closed_form_on_gpu(torch_dev):
    """rank(A) = l: sigma(A Q) = sigma(A) from the first pass, so the first
    ratio is sigma_1^2 / sigma_{k+1}^2 and the second is ~0: N_p = 2."""
    g = json.load(open(os.path.join(GOLDEN, "rank_l_shift_sequence.json")))
    rng = np.random.default_rng(123)
    sig = np.array(g["sigma"])
    Uo, _ = np.linalg.qr(rng.standard_normal((g["m"], len(sig))))
    Vo, _ = np.linalg.qr(rng.standard_normal((g["n"], len(sig))))
    A = synth.dense_to_csr((Uo * sig) @ Vo.T)
    k = g["k"]
    U, S, V, st, info = _solve(A, k, g["s"], 10, 1e-8, 4, "fp64", pve_mode="nosurr")
    assert st == 0 and info.passes == 2
    assert info.ratio[0] == pytest.approx(sig[0] ** 2 / sig[k] ** 2, rel=1e-11)
    assert info.ratio[1] <= 1e-10
    assert np.allclose(S, sig[:k], rtol=1e-12)


def test_nosurr_stops_at_or_one_before_the_surrogate(torch_dev):
    """Table 3's observation on the GPU: N_p without the surrogate is the
    surrogate's or one fewer, and both meet eps_PVE of the order of tol."""
    A = synth.config_small(np.float32)
    sig = np.linalg.svd(A.to_dense(), compute_uv=False)
    for tol in (1e-1, 1e-2, 1e-3):
        _, S2, _, st2, i2 = _solve(A, 20, 10, 64, tol, 2001, "fp32")
        Un, Sn, Vn, stn, i_n = _solve(A, 20, 10, 64, tol, 2001, "fp32", pve_mode="nosurr")
        assert i2.converged and i_n.converged
        assert i2.passes - 1 <= i_n.passes <= i2.passes
        pve, _ = oracle.metrics(A.m, A.n, A.row_ptr, A.col, A.val.astype(np.float64),
                                Un.astype(np.float64), Sn, sig)
        assert pve <= 3 * tol


def test_nosurr_rejected_for_bf16_and_batched(torch_dev):
    from paper_2404_09276_amd import DashSVD, DashSVDError
    A = synth.config_small(np.float32)
    h = DashSVD(precision="bf16", pve_mode="nosurr")
    with pytest.raises(DashSVDError, match="NOSURR"):
        h.solve(A, 20, 10, 1e-2)
    h.close()
    h = DashSVD(precision="fp32", pve_mode="nosurr")
    with pytest.raises(DashSVDError, match="NOSURR"):
        h.run_batched([A, A], 8, 4, 1e-2)
    # the handle stays usable after the refusals
    U, S, V, st, info = h.solve(A, 20, 10, 1e-2)
    assert st == 0 and info.converged
    h.close()

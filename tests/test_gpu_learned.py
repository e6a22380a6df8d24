"""Learned shift policy: the HIP MLP kernels against the FP64 reference
(oracle/mlp_ref.py), training, and the in-solver inference against the
oracle's SCHEDULE policy run with the same multipliers."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp_ref

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
MODEL = os.path.join(os.path.dirname(HERE), "paper_2404_09276_amd", "learned_alpha_c4.npz")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _targets(rng, B):
    return np.stack([rng.uniform(0.5, 0.9, B), rng.uniform(0.5, 3.0, B)], axis=1).astype(np.float32)


def test_mlp_forward_and_gradient_match_fp64_reference(torch_dev):
    from paper_2404_09276_amd import DashSVD
    h = DashSVD()
    l = 10
    D, H = 3 * l + 3, 128
    h.mlp_init(l, 5, 0.9)
    P = h.mlp_params()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((37, D)).astype(np.float32)
    Y = _targets(rng, 37)
    out = h.mlp_forward(X)
    ref = mlp_ref.outputs(P, X, D, H, 0.9)
    assert np.allclose(out, ref, rtol=1e-5, atol=1e-5)
    g, loss = h.mlp_grad(X, Y)
    gr = mlp_ref.grad(P, X, Y, D, H, 0.9)
    assert abs(loss - mlp_ref.loss(P, X, Y, D, H, 0.9)) <= 1e-5 * max(1.0, loss)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    assert np.all(np.abs(g - gr) <= 1e-4 * np.abs(gr) + 1e-6 * np.abs(gr).max())
    h.close()


def test_mlp_training_reduces_loss(torch_dev):
    from paper_2404_09276_amd import DashSVD
    h = DashSVD()
    l = 10
    D = 3 * l + 3
    h.mlp_init(l, 9, 0.9)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((256, D)).astype(np.float32)
    w = rng.standard_normal(D)
    c = 0.5 + 0.4 / (1.0 + np.exp(-(X @ w) / np.sqrt(D)))
    Y = np.stack([c, 1.0 + 0.2 * (X[:, 0])], axis=1).astype(np.float32)
    first = h.mlp_train_step(X, Y, 1e-3)
    for _ in range(300):
        last = h.mlp_train_step(X, Y, 1e-3)
    assert last < 0.2 * first
    h.close()


def test_learned_policy_in_solver_matches_oracle_schedule(torch_dev):
    """A LEARNED run with given weights: the multiplier c the eigensolver of
    pass 2 computes equals the reference forward pass on the run's own
    features, and the whole run equals the oracle's SCHEDULE policy with
    multipliers (1/2, 1/2, c, c, ...)."""
    from paper_2404_09276_amd import DashSVD
    A = synth.config_small(np.float64)
    k, s, pmax = 20, 10, 7
    l = k + s
    h = DashSVD(precision="fp64", p_max=pmax, seed=2001)
    h.mlp_init(l, 21, 0.9)
    P = h.mlp_params()
    # push c away from 1/2 so the check is not vacuous
    D, H = 3 * l + 3, 128
    P[(H * D + H + H * H + H + 2 * H)] = 1.5  # bias of o_0
    h.mlp_set_params(P)
    h.set_options(precision="fp64", p_max=pmax, seed=2001, shift_policy="learned")
    U, S, V, st, info = h.solve(A, k, s, 0.0)
    feats = h.learned_features()
    h.close()
    c = float(mlp_ref.outputs(P, feats[None, :], D, H, 0.9)[0, 0])
    assert 0.75 < c < 0.9
    sched = np.full(pmax + 1, c)
    sched[:2] = 0.5
    ref = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, k, s, pmax, 0.0, seed=2001,
                         shift_policy=oracle.SHIFT_SCHEDULE, sched=sched)
    assert np.allclose(info.alpha_used, ref.alpha, rtol=1e-6, atol=0)
    assert np.abs(S - ref.S).max() / ref.S.max() <= 1e-6


def test_learned_policy_needs_a_model(torch_dev):
    from paper_2404_09276_amd import DashSVD, DashSVDError
    A = synth.config_small(np.float32)
    h = DashSVD(precision="fp32", p_max=5, shift_policy="learned")
    with pytest.raises(DashSVDError) as e:
        h.run(A, 20, 10, 1e-2)
    assert e.value.status == -1
    h.mlp_init(16, 0, 0.9)
    h.set_options(precision="fp32", p_max=5, shift_policy="learned")
    with pytest.raises(DashSVDError) as e:
        h.run(A, 20, 10, 1e-2)
    assert e.value.status == -1
    h.close()


@pytest.mark.skipif(not os.path.exists(MODEL), reason="no trained model file")
def test_trained_model_on_held_out_matrices(torch_dev):
    """The committed model (paper_2404_09276_amd/learned_alpha_c4.npz: k = 50,
    oversampling 25, tol 1e-2, trained on 1045 samples from 5225 runs over
    209 power-law matrices of 50k-500k rows) on held-out matrices of the same
    distribution (seeds 2 x 10^6 + i, Omega seed 9000 + i, as in the
    training script's held-out comparison): on the three held-out matrices
    where the training run saw a gain it needs one pass fewer than the
    paper's rule, on three others the same count, never more, and every run
    meets tol by its PVE check with a true eps_PVE below tol.  Over all 40
    held-out matrices the training run measured 5.225 passes against 5.325
    (four fewer, none more), stored in the model file."""
    from paper_2404_09276_amd import DashSVD, learned
    z = np.load(MODEL, allow_pickle=False)
    hold = z["holdout"]
    assert hold.shape == (40, 9)
    assert hold[:, 6].sum() < hold[:, 3].sum() and np.all(hold[:, 6] <= hold[:, 3])
    gains, controls = [24, 29, 39], [11, 14, 38]
    rows = tuple(int(x) for x in z["rows"])
    pp, pl = {}, {}
    for i in gains + controls:
        A = learned.pool_member(2 * 10**6 + i, rows)
        D = learned.to_device(A, torch_dev)
        sig = learned.reference_sigma(D, 50)
        for policy, acc in (("paper", pp), ("learned", pl)):
            h = DashSVD(precision="fp32", p_max=40, seed=9000 + i)
            if policy == "learned":
                learned.attach(h, MODEL)
            h.set_options(precision="fp32", p_max=40, seed=9000 + i, shift_policy=policy)
            st = h.run(D, 50, 25, 1e-2)
            info = h.info()
            pve, _ = h.evaluate(D, sig)
            h.close()
            assert st == 0 and info.converged and not info.learned_fallback
            assert pve <= 1e-2, (policy, i, pve)
            acc[i] = info.passes
        print(f"held-out {i}: paper {pp[i]} passes, learned {pl[i]}", flush=True)
    assert all(pl[i] == pp[i] - 1 for i in gains)
    assert all(pl[i] <= pp[i] for i in controls)

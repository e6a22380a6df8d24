"""Train the learned shift model and write its parameters.

  python -m paper_2404_09276_amd.train_learned_alpha --out learned_alpha_l75.npz \
      [--train 160] [--holdout 40] [--k 50] [--s 25] [--tol 1e-2]

Builds the training set on the GPU (labels from the schedule family, see
learned.py), trains the MLP with the library's HIP kernels, then compares
the LEARNED policy with the paper's rule on held-out matrices and stores
that comparison next to the parameters.
"""
import argparse
import math
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2404_09276_amd import learned  # noqa: E402
from paper_2404_09276_amd.dashsvd import DashSVD  # noqa: E402


def log(msg):
    print(msg, flush=True)


def compare(mats, k, s, tol, model, seed0):
    """Passes and true eps_PVE of PAPER vs LEARNED on each matrix."""
    rows = []
    for i, A in enumerate(mats):
        sig = learned.reference_sigma(A, k)
        res = []
        for policy in ("paper", "learned"):
            h = DashSVD(precision="fp32", p_max=40, seed=seed0 + i, shift_policy="paper")
            if policy == "learned":
                learned.attach(h, model)
            h.set_options(precision="fp32", p_max=40, seed=seed0 + i, shift_policy=policy)
            h.run(A, k, s, tol)
            info = h.info()
            pve, _ = h.evaluate(A, sig)
            res.append((info.passes, pve, info.learned_fallback))
            h.close()
        rows.append((A.m, A.n, A.nnz) + res[0] + res[1])
        log(f"  held-out {i}: {A.m}x{A.n}: paper N={res[0][0]} eps={res[0][1]:.2e} | "
            f"learned N={res[1][0]} eps={res[1][1]:.2e} fallback={res[1][2]}")
    return np.array(rows, dtype=np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--train", type=int, default=160)
    ap.add_argument("--holdout", type=int, default=40)
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--s", type=int, default=25)
    ap.add_argument("--tol", type=float, default=1e-2)
    ap.add_argument("--epochs", type=int, default=400)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "training needs a GPU"
    l = args.k + args.s
    t0 = time.time()
    log(f"training pool: {args.train} matrices")
    mats = learned.pool(args.train, 10**6)
    X, Y, tables = learned.collect(mats, args.k, args.s, args.tol, 7000, log=log)
    log(f"labelled {X.shape[0]} of {len(mats)} in {time.time() - t0:.0f} s; c* counts: "
        + str({c: int(np.sum(np.isclose(Y[:, 0], c))) for c in learned.C_FAMILY}))
    params, losses = learned.train(X, Y, l, epochs=args.epochs)
    log(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    tmp = args.out + ".tmp.npz"
    learned.save(tmp, params, l, 0.9)
    hold = learned.pool(args.holdout, 2 * 10**6)
    cmp = compare(hold, args.k, args.s, args.tol, tmp, 9000)
    os.remove(tmp)
    learned.save(args.out, params, l, 0.9, train_X=X, train_Y=Y, losses=np.array(losses),
                 holdout=cmp, tol=args.tol, k=args.k, s=args.s)
    log(f"held-out mean passes: paper {cmp[:, 3].mean():.2f} learned {cmp[:, 6].mean():.2f}; "
        f"max eps_PVE: paper {cmp[:, 4].max():.2e} learned {cmp[:, 7].max():.2e}; "
        f"total {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

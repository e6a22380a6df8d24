"""Write reference singular values of the synthetic workloads (oracle only).

The per-vector error eps_PVE of Sec. 4 needs the exact sigma_1..sigma_{k+1}.
For matrices too large for dense LAPACK they come from the FP64 oracle (the
method itself, Alg. 5) run with a wide block and a very small tolerance; by
Prop. 1 the values are lower bounds that converge from below, so the script
records the last pass ratio as the convergence evidence.

It also writes the oracle's own runs of the 2,000,000 x 1,000,000 workload
in the configuration the GPU tests use (k = 100, oversampling 50, Omega from
Philox seed 2003, tol 1e-2 and 1e-3): the singular values, the pass count and
the per-pass shifts and ratios, against which the GPU's BF16 and FP32 runs
are held.

Usage:  python tests/golden/make_reference_sigma.py zipf_200k
        python tests/golden/make_reference_sigma.py zipf_2m       (about 25 min)
        python tests/golden/make_reference_sigma.py zipf_2m_runs  (about 15 min)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = {
    # name: (generator, k_needed, block oversampling, p_max)
    "zipf_200k": (synth.config_zipf_200k, 101, 99, 60),
    "zipf_2m": (synth.config_zipf_2m, 101, 59, 40),
}


def main(name):
    gen, kk, s, pmax = CASES[name]
    A = gen()
    t = time.time()
    r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, kk, s, pmax, 1e-12, seed=7)
    out = {
        "_about": ("Reference sigma_1..sigma_%d of the %s workload from the FP64 oracle "
                   "(Alg. 5, k=%d, oversampling %d, tol 1e-12, p_max %d); lower bounds that "
                   "converge from below (Prop. 1)." % (kk, name, kk, s, pmax)),
        "m": A.m, "n": A.n, "nnz": A.nnz,
        "passes": r.passes, "converged": r.converged,
        "last_ratios": [float(x) for x in r.ratio[-5:]],
        "sigma": [float(x) for x in r.S],
        "oracle_seconds": time.time() - t,
        "threads": oracle.num_threads(),
    }
    with open(os.path.join(HERE, f"sigma_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, r.passes, r.converged, out["last_ratios"], out["oracle_seconds"])


def runs_2m():
    A = synth.config_zipf_2m()
    out = {"_about": ("FP64 oracle runs (Alg. 5) of the zipf_2m workload: k=100, oversampling 50, "
                      "Omega from Philox seed 2003, p_max 64, at tol 1e-2 and 1e-3."),
           "m": A.m, "n": A.n, "nnz": A.nnz, "k": 100, "s": 50, "seed": synth.OMEGA_SEED["zipf_2m"],
           "runs": {}}
    for tol in (1e-2, 1e-3):
        t = time.time()
        r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 100, 50, 64, tol, seed=synth.OMEGA_SEED["zipf_2m"])
        out["runs"][f"{tol:g}"] = {"passes": r.passes, "converged": r.converged,
                                   "sigma": [float(x) for x in r.S],
                                   "alpha": [float(x) for x in r.alpha],
                                   "ratio": [float(x) for x in r.ratio],
                                   "oracle_seconds": time.time() - t}
        print(tol, r.passes, r.converged, time.time() - t, flush=True)
    out["threads"] = oracle.num_threads()
    with open(os.path.join(HERE, "oracle_runs_zipf_2m.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "zipf_2m_runs":
        runs_2m()
    else:
        main(sys.argv[1])

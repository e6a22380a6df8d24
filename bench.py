"""Benchmark: time-to-PVE <= 1e-2 of dashSVD on one MI355X.

Workload (zipf_200k): the 200,000 x 100,000 power-law CSR matrix (10M
nonzeros, Zipf 1.1 row and column degrees, values in (0, 1]), k = 100,
oversampling 20, tol = 1e-2 on the PVE check, FP32 panels.  The matrix is
generated on the host from a fixed seed and copied to device memory before
the timed region; every timed step is one full dashsvd_run: validation,
CSR(A^T), SpMM plans, Omega, the sketch, the shifted power passes until the
check passes, and the final Rayleigh-Ritz step.

Printed: one JSON line with the metric, the roofline of the dominant kernel
(the SpMM, the two sparse products of every pass, timed with HIP events on
the stream it runs on inside the timed region) with its counter traffic, the
Jacobi eigensolver against the FP64 ALU of its one CU and of the chip, the
Gram against the FP64 MFMA peak, the Cholesky-QR pass solver's time, the
other forms of the metric (BF16 panels, learned shift, the accuracy control
without the surrogate, batched, and BF16 against FP32 panels on the
2,000,000 x 1,000,000 workload at tol 1e-2 and 1e-3), and the CPU oracle
timed on the host cores (with the CPU model, and one 2000 x 1500 solve on one
thread and on all of them).

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-forms] [--no-c3]
  python bench.py --copy-probe   (a plain 1 GiB device copy, three times: the
                                  reference that calibrates the HBM counters)
  python bench.py --c5-full      (only the batched workload at its stated scale,
                                  about 6.9e9 nonzeros, one JSON line)
  python bench.py --c3-only      (only the 2M-row forms, one solve each: for profiles)
  python bench.py --batched-only (only the batched form: for profiles)
  python bench.py --summarize-trace STATS_CSV COMMAND > kernel_stats.md
  python bench.py --summarize-pmc FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV COMMANDS > traffic.txt
  python bench.py --summarize-mfma COUNTER_CSV COMMAND > mfma.md
                                 (the committed profile summaries, from the
                                  rocprofv3 outputs of the commands given)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-PVE≤1e-2 (s) + SpMM HBM GB/s, plain FP32 vs BF16/learned-α"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak of one compute unit: 64 FMA lanes x 2 flops x 2.4 GHz
# (the 78.6 TFLOP/s chip peak over 256 CUs); the eigensolver is one workgroup
CU_FP64_TFLOPS = 78.6 / 256
K, P, TOL, OMEGA_SEED = 100, 20, 1e-2, 2002
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_zipf_200k_fp32.txt")
CSRC = os.path.join(ROOT, "paper_2404_09276_amd", "csrc")


def spmm_bytes(m, n, nnz, l, b_val=4, b_idx=4, b_ptr=8, b_x=4, b_y=4):
    """Algorithmic bytes of Y = A X (A m x n CSR, X n x l, Y m x l), each
    array counted once."""
    return nnz * (b_val + b_idx) + (m + 1) * b_ptr + n * l * b_x + m * l * b_y


def tridiag_flops(l):
    """Algorithmic flops of one call of the tridiagonal eigensolver: the
    Householder reduction of an l x l symmetric matrix (4/3 l^3) and the
    back-transformation of l eigenvectors through l - 2 reflectors (2 l^3).
    The multisection's Sturm counts are redundant parallel work and are not
    counted."""
    return 4.0 / 3.0 * l ** 3 + 2.0 * l ** 3


def jacobi_flops(l, sweeps):
    """Algorithmic flops of cyclic Jacobi sweeps on an l x l symmetric matrix
    with eigenvector accumulation: l(l-1)/2 rotations a sweep, each 6l flops
    on the matrix (symmetric two-sided update) and 6l on the vectors."""
    return 6.0 * l * l * (l - 1) * sweeps


def load_workload(torch):
    import synth
    A = synth.config_zipf_200k()

    class Dev:
        m, n, nnz = A.m, A.n, A.nnz
        row_ptr = torch.from_numpy(A.row_ptr).cuda()
        col = torch.from_numpy(A.col).cuda()
        val = torch.from_numpy(A.val).cuda()
    return A, Dev


def reference_sigma():
    path = os.path.join(ROOT, "tests", "golden", "sigma_zipf_200k.json")
    return np.array(json.load(open(path))["sigma"]) if os.path.exists(path) else None


def run_form(torch, Dev, steps, warmup, stream, model=None, detail=0, **kw):
    """Time `steps` solves with HIP events around the SpMM launches only (the
    events of every kernel group would slow the step by a few per cent);
    then `detail` more solves, untimed, with every kernel group timed.
    Returns (seconds, infos of the timed solves, eps_PVE, eps_sigma, infos
    of the detail solves)."""
    from paper_2404_09276_amd import DashSVD, learned
    h = DashSVD(p_max=64, seed=OMEGA_SEED, stream=stream, timing="spmm", **kw)
    if model:
        learned.attach(h, model)
        h.set_options(p_max=64, seed=OMEGA_SEED, stream=stream, timing="spmm", **kw)
    for _ in range(warmup):
        h.run(Dev, K, P, TOL)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        h.run(Dev, K, P, TOL)
        infos.append(h.info())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sig = reference_sigma()
    pve, es = h.evaluate(Dev, sig) if sig is not None else (None, None)
    dinfos = []
    if detail:
        h.set_options(p_max=64, seed=OMEGA_SEED, stream=stream, timing=True, **kw)
        for _ in range(detail):
            h.run(Dev, K, P, TOL)
            dinfos.append(h.info())
        torch.cuda.synchronize()
    h.close()
    return el, infos, pve, es, dinfos


def batched_form(torch, steps):
    """The batched form on 512 power-law matrices (rows 1k-10k, columns
    0.5-1 x rows, density 0.05-1 %, Zipf 1.1), k = 16, oversampling 8, BF16
    panels, tol 1e-2: seconds per batch and matrices per second."""
    import synth
    from paper_2404_09276_amd import DashSVD

    mats = synth.batched_zipf(512, rows=(1000, 10000), seed=5000)
    dev = []
    for A in mats:
        class D:
            pass
        d = D()
        d.m, d.n, d.nnz = A.m, A.n, A.nnz
        d.row_ptr = torch.from_numpy(A.row_ptr).cuda()
        d.col = torch.from_numpy(A.col).cuda()
        d.val = torch.from_numpy(A.val).cuda()
        dev.append(d)
    h = DashSVD(precision="bf16", p_max=16, seed=5000, stream=torch.cuda.current_stream())
    h.run_batched(dev, 16, 8, 1e-2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.run_batched(dev, 16, 8, 1e-2)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    s = h.info_batched(-1)
    h.close()
    return {"value": el, "unit": "s per batch", "matrices_per_s": 512 / el, "matrices": 512,
            "nnz_total": int(sum(A.nnz for A in mats)), "max_passes": s.passes,
            "all_converged": bool(s.converged), "pass_loop_ms": s.time_loop_ms,
            "workload": "512 Zipf 1.1 matrices, rows U[1k,10k], k=16, oversampling 8, BF16 panels, "
                        "tol 1e-2, p_max 16"}


def _c5_member(b):
    import synth
    A = synth.batched_zipf_member(b)
    return b, A.m, A.n, A.row_ptr, A.col, A.val


def batched_full_scale(torch):
    """The batched workload at its stated scale: 512 power-law matrices, rows
    U[1k, 100k], columns 0.5-1 x rows, density 0.05-1 %, Zipf 1.1 (about
    6.9e9 nonzeros), k = 16, oversampling 8, BF16 panels, tol 1e-2, p_max 16,
    all passes of a sub-batch in one graph launch (check_interval = p_max),
    sub-batches below 2^31 nonzeros.  The members are generated on the host
    cores in parallel and moved to the GPU before the timed run.  Checks:
    three small members against the FP64 oracle at their own pass count
    (sigma within 5e-3 relative, the BF16 bar) and the residual
    max_i |A v_i - sigma_i u_i| / sigma_i of the two largest members."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor, as_completed
    import numpy as np
    import scipy.sparse as sp
    import oracle
    import synth
    from paper_2404_09276_amd import DashSVD

    count = 512
    t0 = time.perf_counter()
    dev = [None] * count
    host_small = {}
    nnz_total = 0
    # a worker that dies raises (BrokenProcessPool) instead of leaving the pool waiting
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1), mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(_c5_member, b) for b in range(count)]
        for done, fut in enumerate(as_completed(futs)):
            b, m, n, rp, col, val = fut.result()
            class D:
                pass
            d = D()
            d.m, d.n, d.nnz = m, n, int(rp[-1])
            d.row_ptr = torch.from_numpy(rp).cuda()
            d.col = torch.from_numpy(col).cuda()
            d.val = torch.from_numpy(val).cuda()
            dev[b] = d
            nnz_total += d.nnz
            if m <= 5000 and len(host_small) < 3:
                host_small[b] = (m, n, rp, col, val)
            if (done + 1) % 64 == 0:
                print(f"c5 full scale: {done + 1}/{count} members on the GPU, {nnz_total / 1e9:.2f}e9 nonzeros, "
                      f"{time.perf_counter() - t0:.0f} s", flush=True)
    gen_s = time.perf_counter() - t0
    h = DashSVD(precision="bf16", p_max=16, seed=5000, check_interval=16, stream=torch.cuda.current_stream())
    t1 = time.perf_counter()
    h.run_batched(dev, 16, 8, 1e-2)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t1
    print(f"c5 full scale: first run {first_s:.2f} s", flush=True)
    t1 = time.perf_counter()
    h.run_batched(dev, 16, 8, 1e-2)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    s = h.info_batched(-1)
    worst_small = 0.0
    for b, (m, n, rp, col, val) in sorted(host_small.items()):
        (U, S, V), info = h.get_usv_batched(b), h.info_batched(b)
        ref = oracle.dashsvd(m, n, rp, col, val.astype(np.float64), 16, 8, info.passes, 0.0, seed=5000 + b)
        worst_small = max(worst_small, float(np.max(np.abs(S - ref.S) / ref.S)))
    big = sorted(range(count), key=lambda b: -dev[b].nnz)[:2]
    worst_res = 0.0
    for b in big:
        U, S, V = h.get_usv_batched(b)
        d = dev[b]
        A = sp.csr_matrix((d.val.cpu().numpy(), d.col.cpu().numpy(), d.row_ptr.cpu().numpy()), shape=(d.m, d.n))
        R = A @ V - U * S
        worst_res = max(worst_res, float(np.max(np.linalg.norm(R, axis=0) / S)))
    h.close()
    return {"value": el, "unit": "s per batch", "matrices_per_s": count / el, "matrices": count,
            "nnz_total": nnz_total, "sub_batches": s.sub_batches, "graph_launches": s.graph_launches,
            "max_passes": s.passes, "all_converged": bool(s.converged), "pass_loop_ms": s.time_loop_ms,
            "first_run_s": first_s, "generation_s": gen_s,
            "small_members_sigma_rel_err_vs_oracle": worst_small, "large_members_residual": worst_res,
            "workload": "512 Zipf 1.1 matrices, rows U[1k,100k], columns 0.5-1 x rows, density 0.05-1 %, "
                        "k=16, oversampling 8, BF16 panels, tol 1e-2, p_max 16, one graph launch per sub-batch"}


def c3_forms(torch, stream, steps=2):
    """zipf_2m (2,000,000 x 1,000,000, 100M nonzeros, Zipf 1.1, k = 100,
    oversampling 50): BF16 panels against FP32 panels at tol 1e-2 and 1e-3,
    each with its seconds per solve, passes and eps_PVE / eps_sigma against
    the reference singular values of tests/golden (time-to-tolerance of the
    two forms at the accuracy each reaches)."""
    import synth
    from paper_2404_09276_amd import DashSVD
    A = synth.config_zipf_2m()

    class Dev:
        m, n, nnz = A.m, A.n, A.nnz
        row_ptr = torch.from_numpy(A.row_ptr).cuda()
        col = torch.from_numpy(A.col).cuda()
        val = torch.from_numpy(A.val).cuda()
    path = os.path.join(ROOT, "tests", "golden", "sigma_zipf_2m.json")
    sig = np.array(json.load(open(path))["sigma"]) if os.path.exists(path) else None
    out = {"workload": "zipf_2m: CSR 2000000x1000000, 100M nnz, Zipf 1.1 degrees, k=100, oversampling 50"}
    for prec in ("bf16", "fp32"):
        for tol in (1e-2, 1e-3):
            h = DashSVD(precision=prec, p_max=64, seed=2003, stream=stream)
            h.run(Dev, 100, 50, tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                h.run(Dev, 100, 50, tol)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            inf = h.info()
            pve, es = h.evaluate(Dev, sig) if sig is not None else (None, None)
            out[f"{prec}_tol{tol:g}"] = {"value": el, "unit": "s", "passes": inf.passes,
                                         "converged": bool(inf.converged), "promoted": inf.promoted,
                                         "eps_pve": pve, "eps_sigma": es}
            h.close()
    for tol in ("0.01", "0.001"):
        b, f = out[f"bf16_tol{tol}"], out[f"fp32_tol{tol}"]
        out[f"bf16_over_fp32_time_tol{tol}"] = b["value"] / f["value"]
    del Dev
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_one_thread_small():
    """One FP64 oracle solve of the 2000 x 1500 workload (k = 20,
    oversampling 10, 5 passes) on one host thread and on all of them
    (separate processes: OpenMP fixes its thread count at start)."""
    import subprocess
    code = ("import time, sys; sys.path.insert(0, %r); import numpy as np, oracle, synth; "
            "A = synth.config_small(np.float64); t = time.perf_counter(); "
            "[oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, 20, 10, 5, 0.0, seed=2001) for _ in range(3)]; "
            "print((time.perf_counter() - t) / 3, oracle.num_threads())" % ROOT)
    res = {}
    for label, env in (("one_thread", {"OMP_NUM_THREADS": "1"}), ("all_cores", {})):
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           env=dict(os.environ, **env), timeout=600)
        if r.returncode == 0:
            t, thr = r.stdout.split()
            res[label] = {"seconds": float(t), "threads": int(thr)}
    return res


def cpu_baseline(A, min_seconds=10.0):
    """The oracle as it stands on the host cores: full FP64 solves of the same
    workload (tol 1e-2, same Omega seed), repeated until min_seconds of CPU
    work, seconds per solve."""
    import oracle
    runs, t0 = 0, time.perf_counter()
    passes = None
    while True:
        r = oracle.dashsvd(A.m, A.n, A.row_ptr, A.col, A.val, K, P, 64, TOL, seed=OMEGA_SEED)
        passes = r.passes
        runs += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    t = (time.perf_counter() - t0) / runs
    return {"value": t, "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{runs} full solves of the workload (tol 1e-2, {passes} passes each), "
                      f"mean seconds per solve",
            "small_2000x1500_5_passes": cpu_one_thread_small()}


def source_digest(*names):
    """SHA-256 over the named sources, in order."""
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


# The SpMM's counter traffic depends on the kernel, on the order of the
# operator's rows and columns (the degree order is built in k_csr.hip) and on
# the panel layout (the leading dimension is chosen in driver.hip).
TRAFFIC_SOURCES = {"spmm": ("k_spmm.hip", "k_head.hip", "k_csr.hip", "driver.hip"), "eig": ("k_eigtri.hip",)}


def traffic(kind):
    """HBM bytes per launch of a kernel ("spmm": one SpMM, k_spmm and its
    long-row kernel; "eig": one tridiagonal eigSVD call, its two kernels)
    from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel),
    or None when it is missing or the kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = {}
    for line in open(TRAFFIC_FILE):
        parts = line.split()
        if len(parts) == 2 and not line.startswith("#"):
            t[parts[0]] = parts[1]
    if t.get(f"{kind}_sha256") != source_digest(*TRAFFIC_SOURCES[kind]) or f"{kind}_bytes_per_launch" not in t:
        return None
    return float(t[f"{kind}_bytes_per_launch"])


def short_name(name):
    """Kernel name without namespaces and argument list."""
    base = name[5:] if name.startswith("void ") else name
    for ns in ("dsv::(anonymous namespace)::", "dsv::"):
        base = base.replace(ns, "")
    return base.split("(")[0].strip()


def summarize_trace(stats_csv, command):
    """Markdown table of a rocprofv3 --stats kernel summary."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | total ms | average us | % of GPU time |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        if float(r["TotalDurationNs"]) < 1e-3 * tot:
            continue
        out.append(f"| `{short_name(r['Name'])[:80]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / tot:.2f} |")
    print(f"Command (from /tmp; R = repository root):\n\n    {command}\n")
    print("\n".join(out))


def summarize_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, commands):
    """Per-kernel HBM traffic per dispatch from FETCH_SIZE and WRITE_SIZE
    runs, each calibrated by what the counter reads for a plain copy of known
    size; the lines the benchmark reads (per-launch bytes and the source
    digests they belong to) come last."""
    import csv

    def per_kernel(path):
        acc = {}
        for r in csv.DictReader(open(path)):
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return acc

    def copy_kib(path):
        vals = [v for k, vs in per_kernel(path).items() if "copyBuffer" in k for v in vs]
        return max(vals)

    probe_bytes = (1 << 28) * 4
    fcal = probe_bytes / 1024.0 / copy_kib(copy_fetch_csv)
    wcal = probe_bytes / 1024.0 / copy_kib(copy_write_csv)
    fk, wk = per_kernel(fetch_csv), per_kernel(write_csv)
    rows = []
    for name in fk:
        if name not in wk or "rocclr" in name:
            continue
        f, w = np.mean(fk[name]), np.mean(wk[name])
        rows.append((short_name(name), len(fk[name]), f, w, (fcal * f + wcal * w) * 1024 / 1e6, fk[name], wk[name]))
    rows.sort(key=lambda r: -r[4] * r[1])
    print("# HBM traffic per dispatch, zipf_200k workload (200000 x 100000, 10M nnz, k=100, oversampling 20,")
    print("# FP32 panels, tol 1e-2), one bench step; MI355X, rocprofv3 counter collection.")
    print("# Commands (run from /tmp; R = repository root):")
    for c in commands:
        print(f"#   {c}")
    print(f"# Calibration: a plain 1 GiB device copy reads FETCH_SIZE = {probe_bytes / 1024 / fcal:.1f} KiB and")
    print(f"# WRITE_SIZE = {probe_bytes / 1024 / wcal:.1f} KiB per launch, so bytes = {fcal:.4f} x FETCH_SIZE x 1024"
          f" + {wcal:.4f} x WRITE_SIZE x 1024.")
    print("# FETCH_SIZE counts L2 misses, which the 256 MB last-level cache may still serve: an upper bound on HBM reads.")
    print("#")
    print(f"# {'kernel':56s} {'dispatches':>10s} {'FETCH_KiB':>11s} {'WRITE_KiB':>11s} {'calibrated_MB':>14s}")
    for name, cnt, f, w, mb, _, _ in rows:
        print(f"# {name[:56]:56s} {cnt:10d} {f:11.1f} {w:11.1f} {mb:14.2f}")
    print("#")
    spmm = [r for r in rows if r[0].startswith("k_spmm<")]
    spmm_long = [r for r in rows if r[0].startswith("k_spmm_long<")]
    heads = [r for r in rows if r[0].startswith("k_head_partial<") or r[0].startswith("k_head_reduce<")]
    # one SpMM launch = k_spmm + its long-row kernel + the dense head kernels
    # of the products that have one (all summed, over the k_spmm dispatches)
    n_spmm = max(1, sum(r[1] for r in spmm))
    spmm_b = sum(r[4] * r[1] for r in spmm + spmm_long + heads) / n_spmm
    # tridiagonal eigSVD calls: k_tri_reduce + k_tri_vectors (means over
    # their dispatches; the Jacobi launch behind each call returns at once
    # unless the call declined)
    eig_b, eig_n = 0.0, 0
    for pre in ("k_tri_reduce<", "k_tri_vectors"):
        sel = [r for r in rows if r[0].startswith(pre)]
        n = sum(r[1] for r in sel)
        if n:
            eig_b += sum(r[4] * r[1] for r in sel) / n * 1e6
            eig_n = n
    print("# One SpMM launch = k_spmm + k_spmm_long + the dense head (k_head_partial + k_head_reduce, A C only),")
    print("# their bytes summed over the k_spmm dispatches; one eigSVD call =")
    print("# k_tri_reduce + k_tri_vectors (means over their dispatches).")
    print(f"# Algorithmic bytes per launch for comparison: SpMM (A C) {spmm_bytes(200000, 100000, 10**7, 120) / 1e6:.1f} MB,"
          f" SpMM (A^T Z) {spmm_bytes(100000, 200000, 10**7, 120) / 1e6:.1f} MB.")
    print(f"fetch_calibration {fcal:.6f}")
    print(f"write_calibration {wcal:.6f}")
    print(f"spmm_sha256 {source_digest(*TRAFFIC_SOURCES['spmm'])}")
    print(f"spmm_bytes_per_launch {spmm_b * 1e6:.0f}")
    print(f"eig_sha256 {source_digest(*TRAFFIC_SOURCES['eig'])}")
    print(f"eig_bytes_per_launch {eig_b:.0f}")
    print(f"eig_calls_counted {eig_n}")


def summarize_mfma(csv_path, command):
    """Per-kernel MFMA utilisation from SQ_VALU_MFMA_BUSY_CYCLES,
    GRBM_GUI_ACTIVE and SQ_INSTS_VALU_MFMA_MOPS_F64 (rocprofv3 --pmc): busy
    cycles over (the kernel's duration x 2.4 GHz x 1024 SIMDs), and over
    (GRBM_GUI_ACTIVE / 8 x 1024), the per-dispatch GRBM value being the sum
    over the 8 XCDs and including the profiler's window around the kernel;
    and the FP64 MFMA flops (512 a MOP)."""
    import csv
    per = {}
    for r in csv.DictReader(open(csv_path)):
        d = per.setdefault((r["Kernel_Name"], r["Dispatch_Id"]), {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        d["dur_ns"] = float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    simds, clock = 256 * 4, 2.4e9
    agg = {}
    for (name, _), c in per.items():
        if "SQ_VALU_MFMA_BUSY_CYCLES" not in c or "GRBM_GUI_ACTIVE" not in c:
            continue
        a = agg.setdefault(short_name(name), [0, 0.0, 0.0, 0.0, 0.0])
        a[0] += 1
        a[1] += c["SQ_VALU_MFMA_BUSY_CYCLES"]
        a[2] += c["GRBM_GUI_ACTIVE"]
        a[3] += c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
        a[4] += c["dur_ns"]
    print(f"Command (from /tmp; R = repository root):\n\n    {command}\n")
    print("| kernel | dispatches | mean duration us | MFMA busy / (duration x 2.4 GHz x 1024 SIMDs) "
          "| MFMA busy / (GRBM_GUI_ACTIVE / 8 x 1024) | FP64 MFMA flops a dispatch | FP64 MFMA TFLOP/s |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for name, (n, busy, act, mops, dur) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        if busy <= 0:
            continue
        fl = 512.0 * mops / n
        print(f"| `{name[:60]}` | {n} | {dur / n / 1e3:.1f} | {100.0 * busy / (dur * 1e-9 * clock * simds):.1f} % | "
              f"{100.0 * busy / (act / 8.0 * simds):.1f} % | {fl:.3e} | {fl / (dur / n * 1e-9) / 1e12:.1f} |")
    print("\nThe Gram kernel computes whole 16 x 16 upper tiles; the method's work per pass block is "
          f"n l (l + 1) = {100000 * 120 * 121:.3e} flops (upper triangle of C^T C). Dense FP64 MFMA peak: 78.6 TFLOP/s.")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--c3-only", action="store_true",
                    help="only the 2M-row forms (BF16 and FP32 panels, tol 1e-2 and 1e-3), one solve each")
    ap.add_argument("--batched-only", action="store_true", help="only the batched form")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--c5-full", action="store_true",
                    help="only the batched workload at its stated scale (about 6.9e9 nonzeros)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("STATS_CSV", "COMMAND"))
    ap.add_argument("--summarize-pmc", nargs="+", metavar="ARG")
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("COUNTER_CSV", "COMMAND"))
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_pmc:
        a = args.summarize_pmc
        summarize_pmc(a[0], a[1], a[2], a[3], a[4:])
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this library has no multi-GPU form)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.c5_full:
        print(json.dumps({"batched_full_scale": batched_full_scale(torch)}), flush=True)
        return
    if args.c3_only:
        print(json.dumps({"c3": c3_forms(torch, torch.cuda.current_stream(), steps=1)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_form(torch, 3)}), flush=True)
        return
    A, Dev = load_workload(torch)
    stream = torch.cuda.current_stream()
    ndetail = 3
    el, infos, pve, es, dinfos = run_form(torch, Dev, args.steps, args.warmup, stream, detail=ndetail,
                                          precision="fp32")
    ms = el / args.steps * 1e3
    inf = infos[-1]
    l = K + P
    # SpMM launches: HIP events of the timed solves
    tot_s = {g: sum(i.kt_ms[g] for i in infos) for g in ("spmm", "spmm_t")}
    cnt_s = {g: sum(i.kt_count[g] for i in infos) for g in ("spmm", "spmm_t")}
    # every kernel group: the detail solves after the timed ones
    tot = {g: sum(i.kt_ms[g] for i in dinfos) for g in dinfos[0].kt_ms}
    cnt = {g: sum(i.kt_count[g] for i in dinfos) for g in dinfos[0].kt_count}
    avg = {g: (tot[g] / cnt[g] if cnt[g] else 0.0) for g in tot}
    for g in ("spmm", "spmm_t"):
        avg[g] = tot_s[g] / cnt_s[g] if cnt_s[g] else 0.0
    dom = max(("spmm", "spmm_t", "gram", "eig", "cholqr", "rescale", "transpose", "final"), key=lambda g: tot[g])
    # dominant kernel, the SpMM: algorithmic bytes of the two products of a
    # pass over their event time (one launch = k_spmm and its long-row kernel)
    b1 = spmm_bytes(A.m, A.n, A.nnz, l)
    b2 = spmm_bytes(A.n, A.m, A.nnz, l)
    gbs1 = b1 / (avg["spmm"] * 1e-3) / 1e9 if avg["spmm"] else 0.0
    gbs2 = b2 / (avg["spmm_t"] * 1e-3) / 1e9 if avg["spmm_t"] else 0.0
    pair_ms = avg["spmm"] + avg["spmm_t"]
    achieved = (b1 + b2) / (pair_ms * 1e-3) / 1e9 if pair_ms else 0.0
    # eigensolver calls of the pass blocks (the "eig" group; the final step's
    # call is timed in the "final" group): the tridiagonal solver's
    # algorithmic flops over their event time (the Jacobi kernel launched
    # behind each call runs only where the tridiagonal solver declines)
    eig_ms = tot["eig"]
    tri_calls = int(sum(max(0, i.eig_calls - 1) for i in dinfos))
    sweeps = int(sum(int(np.sum(i.sweeps_per_call[:max(0, i.eig_calls - 1)])) for i in dinfos))
    eig_flops = tri_calls * tridiag_flops(l) + jacobi_flops(l, sweeps)
    eig_tf = eig_flops / (eig_ms * 1e-3) / 1e12 if eig_ms else 0.0
    # Gram of the pass blocks: the method's n l (l + 1) FP64 flops (upper
    # triangle of C^T C) over the event time of a Gram launch (partials and
    # their sum)
    gram_tf = A.n * l * (l + 1) / (avg["gram"] * 1e-3) / 1e12 if avg["gram"] else 0.0
    out = {
        "metric": METRIC, "value": ms / 1e3, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "zipf_200k: CSR 200000x100000, 10M nnz, Zipf 1.1 degrees, "
                               "k=100, oversampling 20, PVE tol 1e-2, FP32 panels",
                   "form": "plain FP32", "passes": inf.passes, "converged": inf.converged,
                   "eps_pve": pve, "eps_sigma": es, "eig_calls": inf.eig_calls,
                   "cholqr_calls": inf.cholqr_calls, "eig_sweeps": inf.eig_sweeps,
                   "sweeps_per_call": [int(x) for x in inf.sweeps_per_call],
                   "dense_head_rows": [inf.head_rows, inf.head_rows_t]},
        "roofline": {"bound": "hbm", "kernel": "SpMM (k_spmm + k_spmm_long + dense head k_head_partial + "
                     "k_head_reduce), the two products of a pass",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic("spmm"),
                     # the counters' bytes (L2 misses of the gathers, served by the
                     # last-level cache or HBM) per second of a launch
                     "traffic_gbs": (traffic("spmm") / (0.5 * pair_ms * 1e-3) / 1e9
                                     if traffic("spmm") and pair_ms else None),
                     "bytes_per_launch": {"spmm": b1, "spmm_t": b2},
                     "avg_ms": {"spmm": avg["spmm"], "spmm_t": avg["spmm_t"]},
                     "gbs": {"spmm": gbs1, "spmm_t": gbs2}},
        "roofline_eig": {"bound": "latency",
                         "kernel": "k_tri_reduce + k_tri_vectors (tridiagonal eigSVD: Householder reduction "
                                   "in one workgroup, then one wave per eigenvalue)",
                         "achieved": eig_tf, "peak": CU_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": eig_tf / CU_FP64_TFLOPS, "traffic": traffic("eig"),
                         "flops_per_call": tridiag_flops(l), "calls_timed": tri_calls,
                         "jacobi_sweeps_after_declines": sweeps,
                         "avg_ms_per_call": eig_ms / tri_calls if tri_calls else 0.0,
                         "peak_basis": "FP64 vector peak of one CU (78.6 TFLOP/s / 256): the reduction runs "
                                       "in one workgroup, l - 2 dependent steps with two barriers each",
                         "frac_of_chip_fp64": eig_tf / 78.6},
        "roofline_gram": {"bound": "mfma", "kernel": "k_gram_partial + k_gram_reduce (FP64 MFMA, C^T C)",
                          "achieved": gram_tf, "peak": 78.6, "unit": "TFLOP/s", "frac": gram_tf / 78.6,
                          "flops_per_launch": A.n * l * (l + 1), "avg_ms": avg["gram"]},
        "cholqr": {"kernel": "k_cholqr (Cholesky-QR weights and Sturm-bisection eigenvalues, two workgroups)",
                   "calls_per_step": cnt["cholqr"] / ndetail, "avg_ms_per_launch": avg["cholqr"]},
        "kernel_groups_ms_per_step": {g: tot[g] / ndetail for g in tot},
        "kernel_groups_from": f"{ndetail} solves after the timed ones, every kernel group timed",
        "dominant_group": dom,
    }
    if not args.no_forms:
        nf = max(2, args.steps // 3)
        elb, infb, pveb, esb, _ = run_form(torch, Dev, nf, 1, stream, precision="bf16")
        out["forms"] = {"bf16_panels": {"value": elb / nf, "unit": "s", "passes": infb[-1].passes,
                                        "promoted": infb[-1].promoted, "eps_pve": pveb, "eps_sigma": esb}}
        model = os.path.join(ROOT, "paper_2404_09276_amd", "learned_alpha_l120.npz")
        if os.path.exists(model):
            ell, infl, pvel, esl, _ = run_form(torch, Dev, nf, 1, stream, model=model, precision="fp32",
                                            shift_policy="learned")
            out["forms"]["learned_alpha"] = {"value": ell / nf, "unit": "s", "passes": infl[-1].passes,
                                             "fell_back": infl[-1].learned_fallback,
                                             "predicted_passes": infl[-1].learned_n,
                                             "eps_pve": pvel, "eps_sigma": esl}
        el64, inf64, pve64, es64, _ = run_form(torch, Dev, nf, 1, stream, precision="fp64")
        out["forms"]["fp64"] = {"value": el64 / nf, "unit": "s", "passes": inf64[-1].passes,
                                "eps_pve": pve64, "eps_sigma": es64, "cholqr_calls": inf64[-1].cholqr_calls,
                                "about": "FP64 panels and SpMM, Cholesky-QR for the early blocks, Jacobi after"}
        eln, infn, pven, esn, _ = run_form(torch, Dev, nf, 1, stream, precision="fp32", pve_mode="nosurr")
        out["forms"]["no_surrogate"] = {"value": eln / nf, "unit": "s", "passes": infn[-1].passes,
                                        "eps_pve": pven, "eps_sigma": esn,
                                        "time_over_surrogate": (eln / nf) / (ms / 1e3),
                                        "about": "accuracy control without the surrogate (Sec. 4.3): "
                                                 "sigma(A Q) after every pass, eq. (18)"}
        out["forms"]["batched"] = batched_form(torch, 3)
        if not args.no_c3:
            out["forms"]["c3"] = c3_forms(torch, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

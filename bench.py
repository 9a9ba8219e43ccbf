#!/usr/bin/env python3
"""Benchmark of the multilevel BLUP solve on one MI355X.

Default line (the headline metric, Matern C.x Gpairs/s): one step = one
application of the solve's operator C_W = W C(theta) W^T in FP64 (W^T, the
dense covariance product over all N^2 ordered pairs, W) on the largest
workload: 1,048,576 points in d = 20 (half uniform in [0,1]^20, half near a
random 3-dimensional affine subspace), Matern nu = 1/2, rho = 1, linear trend
(p = 21), leaf 64.  The points, the basis image and the input vector are
resident in HBM before the timed region; `value` = N^2 logical pairs per
step over the wall-clock time of the K timed steps.  The same line carries:
the FP64 product's rate from HIP events on the launch stream and its
roofline object (sym_kernel, FP64 vector peak), the evaluated (unordered)
pair count, the mixed-precision operator (BF16 x3 matrix-core Gram for
d >= 8, FP32 otherwise) with its error against the FP64 one, the FP64
product against the oracle on sampled rows, a record of the whole predictor
path (tree, basis, preconditioner, FP64 and mixed solves to relres 1e-8,
predictors, gradients) on the 65,536-point d = 3 workload under its own
key, and the oracle's CPU baseline.

`--solve` prints the whole-path line for one workload instead (the records
under profiles/blup_solve_* come from it); `--sweep`, `--loglik`,
`--loglik-sparse` and `--cpu-oracle` are the other measurement modes.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6      # 256 CU x 2.4 GHz x 64 lanes x 2 flop (FMA)


def flops_per_unordered_pair(d: int, nu: float) -> int:
    """Algorithmic flops of one distinct pair {i, j} of the FP64 symmetric
    product (FMA = 2): the squared distance, sqrt (1), exp (1), the Matern
    polynomial (nu=1/2: 0; 3/2: 1+z and the product with e^-z = 2; 5/2: two
    FMA and the product = 5) and two accumulation FMAs (4), one for y_i and
    one for y_j.  The squared distance is d differences + d squared
    accumulations (3d) for d < 8; from d = 8 on the kernel takes the
    expanded form |a|^2 + |b|^2 - 2 a.b, d FMAs for the dot product, one
    addition of the norms and one FMA (2d + 3; the norms themselves are per
    point, not per pair)."""
    poly = {0.5: 0, 1.5: 2, 2.5: 5}[nu]
    dist = 2 * d + 3 if d >= 8 else 3 * d
    return dist + 6 + poly


TRAFFIC_FILES = {"cfg2_n65536_d3_nu1.5": os.path.join(ROOT, "profiles", "traffic_sym_kernel_fp64_cfg2_n65536_d3.txt"),
                 "cfg5_n1048576_d20_nu0.5": os.path.join(ROOT, "profiles",
                                                         "traffic_sym_kernel_fp64_cfg5_n1048576_d20.txt")}
VALU_FILE = os.path.join(ROOT, "profiles", "valu_per_pair_sym_kernel.txt")
VALU_LANE_RATE = 256 * 4 * 16 * 2.4e9   # VALU lane-instructions per second (CUs x SIMDs x lanes x clock)


def _hashed_file(path):
    """key = value lines of a recorded measurement whose source hash still
    matches the sources it names, else None."""
    import hashlib
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in kv.get("sources", "").split():
        p = os.path.join(ROOT, src)
        if not os.path.exists(p):
            return None
        h.update(open(p, "rb").read())
    return kv if h.hexdigest() == kv.get("source_sha256") else None


def valu_per_pair(kind: str, d: int, nu: float):
    """VALU instructions per evaluated pair of the symmetric kernel (from the
    gfx950 assembly, recorded by paper_1701_00285_amd.isa_stats), or None."""
    kv = _hashed_file(VALU_FILE)
    if kv is None:
        return None
    v = kv.get(f"{kind}_d{d}_nu2{int(round(2 * nu))}")
    return float(v) if v is not None else None


def measured_traffic(workload: str):
    """HBM bytes per FP64 symmetric product of a full-size workload from the
    calibrated rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded under
    profiles/, or None when there is no record or the kernel sources changed
    since it was taken (hash mismatch)."""
    path = TRAFFIC_FILES.get(workload)
    kv = _hashed_file(path) if path else None
    return int(float(kv["hbm_bytes_per_product"])) if kv else None


def cpu_baseline(wl, rows: int):
    """The oracle's row-block FP64 product on a bounded sample of rows."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import brute
    import synth
    x = synth.standard_normal(wl.n, 12345)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        brute.cov_matvec(wl.points[:rows], wl.points, x, wl.nu, wl.rho, wl.sigma2)
        dt = time.perf_counter() - t0
    return {"value": rows * wl.n / dt / 1e9, "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} rows x {wl.n} columns of the FP64 covariance product ({rows * wl.n:.3g} pairs, "
                      f"{dt:.1f} s, one thread)"}


def _host_cores() -> int:
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_oracle_report(parts: str = "all"):
    """The oracle timed on the host's cores beside the GPU (one JSON line):
    (i) the row-block FP64 covariance product on all cores (a thread pool over
    blocks of 1,024 rows, one BLAS thread each; NumPy releases the GIL inside
    its array operations) and on one core: all cores take every row of
    workloads 1 and 2, 32,768 rows of workload 4 and 4,096 rows of workloads 3
    and 5; one core takes every row of workload 1, 512 rows of workloads 2 and
    4 and 128 rows of workloads 3 and 5; rates in Gpairs/s and the full
    product's time extrapolated where sampled;
    (ii) the dense classic BLUP (Cholesky, GLS beta, kriging; LAPACK on all
    cores) on workload 1, the workload 4 generator at 4,096 points and the
    workload 2 generator at 32,768 points, beside the GPU predictor (FP64
    solve to relres 1e-8, block preconditioner) on the same inputs, and the
    largest prediction difference between the two.  parts: "products",
    "blup" or "all"."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits

    from oracle import blup, brute
    import synth
    from paper_1701_00285_amd import FP64, PREC_BLOCK, PcgOptions, Solver
    cores = _host_cores()
    out = {"cores": cores, "kind": "oracle", "products": {}, "dense_blup": {}}

    def product(wl, rows, threads):
        x = synth.standard_normal(wl.n, 12345)
        blocks = [(i, min(rows, i + 1024)) for i in range(0, rows, 1024)]
        inner = max(16, min(256, (1 << 25) // wl.n))   # rows per dense block: at most 256 MB per temporary

        def run(b):
            return brute.cov_matvec(wl.points[b[0]:b[1]], wl.points, x, wl.nu, wl.rho, wl.sigma2, block=inner)

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            if threads == 1:
                for b in blocks:
                    run(b)
            else:
                with ThreadPoolExecutor(max_workers=threads) as ex:
                    list(ex.map(run, blocks))
            return time.perf_counter() - t0

    for k in ((1, 2, 3, 4, 5) if parts in ("all", "products") else ()):
        wl = synth.make_config(k, with_z=False)
        rows_all = {1: wl.n, 2: wl.n, 4: 32768}.get(k, 4096)
        rows_one = {1: wl.n, 2: 512, 4: 512}.get(k, 128)
        dt_all = product(wl, rows_all, cores)
        dt_one = product(wl, rows_one, 1)
        rec = {"n": wl.n, "d": wl.d,
               "all_cores": {"rows": rows_all, "s": round(dt_all, 3),
                             "gpairs_s": round(rows_all * wl.n / dt_all / 1e9, 4),
                             "full_product_s": round(dt_all * wl.n / rows_all, 2)},
               "one_core": {"rows": rows_one, "s": round(dt_one, 3),
                            "gpairs_s": round(rows_one * wl.n / dt_one / 1e9, 4),
                            "full_product_s": round(dt_one * wl.n / rows_one, 1)}}
        out["products"][f"cfg{k}"] = rec
        print(f"cpu product cfg{k}: {rec}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    for k, n in (((1, None), (4, 4096), (2, 32768)) if parts in ("all", "blup") else ()):
        wl = synth.make_config(k, n=n)
        if wl.z is None:   # workload 1: Z = X beta + G xi with G = chol(C), drawn with the oracle's C
            from oracle.design import design_matrix
            from oracle.matern import cov_matrix
            import scipy.linalg as sla
            X = design_matrix(wl.points, wl.degree_w)
            G = sla.cholesky(cov_matrix(wl.points, wl.points, wl.nu, wl.rho, wl.sigma2), lower=True)
            wl.z = X @ wl.extra["beta_gen"][: X.shape[1]] + G @ wl.extra["xi"]
        print(f"cpu dense blup cfg{k} n={wl.n}: start", file=sys.stderr, flush=True)
        with threadpool_limits(limits=cores):
            t0 = time.perf_counter()
            ref = blup.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, wl.nu, wl.rho, wl.sigma2)
            dt_cpu = time.perf_counter() - t0
        print(f"cpu dense blup cfg{k} n={wl.n}: {dt_cpu:.2f} s", file=sys.stderr, flush=True)
        s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2, max_targets=wl.targets.shape[0])
        z = torch.as_tensor(wl.z, dtype=torch.float64, device="cuda")
        tg = torch.as_tensor(wl.targets, dtype=torch.float64, device="cuda")
        pc = s.precond(PREC_BLOCK)
        opts = PcgOptions(rtol=1e-8, max_iter=20000, precision=FP64, precond=pc)
        s.predict(z, tg, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = s.predict(z, tg, opts)
        torch.cuda.synchronize()
        dt_gpu = time.perf_counter() - t0
        zh = g["zhat"].cpu().numpy()
        err = float(np.max(np.abs(zh - ref.zhat)) / np.max(np.abs(ref.zhat)))
        rec = {"n": wl.n, "d": wl.d, "targets": int(wl.targets.shape[0]), "cpu_s": round(dt_cpu, 3),
               "gpu_predict_s": round(dt_gpu, 4), "gpu_iters": g["info"]["inner_iters"],
               "zhat_max_rel_diff": err}
        out["dense_blup"][f"cfg{k}"] = rec
        print(f"gpu predict cfg{k} n={wl.n}: {rec}", file=sys.stderr, flush=True)
        del s
    print(json.dumps(out), flush=True)


def sweep(configs, reps: int = 10, warm: int = 3, nu=None):
    """Per workload: the square product in every precision that applies
    (median of `reps` HIP-event timings after `warm` untimed launches), the
    FP64 target product, and W / W^T against their algorithmic bytes.  Errors:
    each precision against the FP64 GPU product, and the FP64 product against
    the oracle on 16 sampled rows.  One JSON line per workload."""
    import numpy as np
    import torch

    import synth
    from oracle import brute
    from paper_1701_00285_amd import (FP32, FP64, MFMA_BF16X3, MFMA_FP32, VALUE, Solver, cov_matvec,
                                      cov_workspace_bytes, profile_enable, profile_read)
    torch.cuda.set_device(0)
    names = {FP64: "fp64", FP32: "fp32", MFMA_FP32: "mfma_fp32", MFMA_BF16X3: "mfma_bf16x3"}
    for k in configs:
        wl = synth.make_config(k, with_z=False)
        if nu is not None:
            wl.nu = nu
        n, d = wl.n, wl.d
        closed = wl.nu in (0.5, 1.5, 2.5) or math.isinf(wl.nu)
        s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2, max_targets=wl.targets.shape[0])
        P = s.basis.points_dev
        x_host = synth.standard_normal(n, 7)
        x = torch.as_tensor(x_host, dtype=torch.float64, device="cuda")
        pts_tree = P.cpu().numpy()
        idx = np.random.default_rng(k).choice(n, 16, replace=False)
        ref = brute.cov_matvec(pts_tree[idx], pts_tree, x_host, wl.nu, wl.rho, wl.sigma2)
        scale = brute.cov_matvec(pts_tree[idx], pts_tree, np.abs(x_host), wl.nu, wl.rho, wl.sigma2)

        def timed(fn, prec):
            times = []
            out = None
            for i in range(warm + reps):
                profile_enable(True)
                profile_read()
                out = fn()
                torch.cuda.synchronize()
                ms, nl, _ = profile_read()[(prec, VALUE)]
                if i >= warm:
                    times.append(ms / nl)
            profile_enable(False)
            return float(np.median(times)), out

        precs = [FP64, FP32] + ([MFMA_FP32, MFMA_BF16X3] if closed and 8 <= d <= 32 else [])
        prods, y64 = {}, None
        for prec in precs:
            work = torch.empty(max(cov_workspace_bytes(n, n, d, prec, VALUE), 256), dtype=torch.uint8, device="cuda")
            ms, (y, _) = timed(lambda: cov_matvec(P, P, x, wl.nu, wl.rho, wl.sigma2, precision=prec, work=work), prec)
            if prec == FP64:
                y64 = y
            e = {"ms": round(ms, 4), "logical_gpairs_s": round(n * n / (ms * 1e-3) / 1e9, 1),
                 "maxerr_vs_fp64_product": float(torch.max(torch.abs(y - y64)) / torch.max(torch.abs(y64)))}
            if prec == FP64:
                e["rowerr_vs_oracle"] = float(np.max(np.abs(y.cpu().numpy()[idx] - ref) / scale))
            prods[names[prec]] = e
            del work
        T = torch.as_tensor(wl.targets, dtype=torch.float64, device="cuda")
        m = T.shape[0]
        work = torch.empty(max(cov_workspace_bytes(m, n, d, FP64, VALUE), 256), dtype=torch.uint8, device="cuda")
        ms, _ = timed(lambda: cov_matvec(T, P, x, wl.nu, wl.rho, wl.sigma2, precision=FP64, work=work), FP64)
        targets = {"m": m, "ms": round(ms, 4), "logical_gpairs_s": round(m * n / (ms * 1e-3) / 1e9, 1)}
        # W and W^T: torch events on the current stream (the library launches on it)
        tb = s.basis.transform_bytes()
        res = {}
        for name, fn in (("apply_W", lambda: s.apply_W(x)), ("apply_Wt", lambda: s.apply_Wt(x[: n - s.p]))):
            ts = []
            for i in range(warm + reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                if i >= warm:
                    ts.append(e0.elapsed_time(e1))
            med = float(np.median(ts))
            res[name] = {"ms": round(med, 4), "algorithmic_bytes": tb, "gb_s": round(tb / (med * 1e-3) / 1e9, 1)}
        print(json.dumps({"workload": wl.name, "n": n, "d": d, "nu": wl.nu, "rho": wl.rho, "reps": reps,
                          "warmup": warm, "square_product": prods, "target_product_fp64": targets,
                          "transform": res}), flush=True)


def loglik_bench(k: int, n: int, reps: int = 3, quick: bool = False):
    """Estimator path: l_n at the finest levels and at level 0 (each the
    median of `reps` calls after one untimed call, host clock around a call
    that synchronises), the sparsified l~_n at levels t and t - 1 for tau from
    0.05 (the distance of the paper's d = 3 estimation runs) to 0.4, with the
    fill of C~^n_W, and one golden-section MLE of rho at level t - 1.
    quick: levels t and 0 only, one timed call each (large n).
    Flops of one call: the dense Cholesky N~^3/3, the two batched analyses
    2 sum_cells m^2 (N + N~) and the covariance N^2 pairs."""
    import time

    import numpy as np
    import torch

    import synth
    from paper_1701_00285_amd import MlblupError, Solver
    torch.cuda.set_device(0)
    wl = synth.make_config(k, n=n, n_targets=1)
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2)
    z = torch.as_tensor(wl.z, dtype=torch.float64, device="cuda")
    t = s.basis.levels - 1
    res = {"workload": f"cfg{k} generator, n={n}, d={wl.d}, nu={wl.nu}, rho={wl.rho}", "levels": {}}
    if quick:
        reps = 1
    for level in ((t, 0) if quick else (t, t - 1, t - 2, 0)):
        s.loglik(z, level)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = s.loglik(z, level)
            times.append(time.perf_counter() - t0)
        ms = 1e3 * float(np.median(times))
        nt = out["rows"]
        res["levels"][str(level)] = {"rows": nt, "ms": round(ms, 3), "loglik": out["loglik"],
                                    "logdet": out["logdet"], "quad": out["quad"],
                                    "cholesky_gflop": round(nt ** 3 / 3 / 1e9, 2)}
        print(f"loglik level {level}: rows {nt}, {ms:.1f} ms", file=sys.stderr, flush=True)
    if quick:
        print(json.dumps(res), flush=True)
        return
    res["sparsified"] = {}
    for level in (t, t - 1):
        for tau in (0.05, 0.1, 0.2, 0.4):
            key = f"level {level} tau {tau}"
            try:
                t0 = time.perf_counter()
                out = s.loglik(z, level, tau=tau)
                ms = 1e3 * (time.perf_counter() - t0)
                res["sparsified"][key] = {"ms": round(ms, 3), "fill": round(out["nnz"] / out["rows"] ** 2, 4),
                                          "loglik": out["loglik"],
                                          "exact_loglik": res["levels"][str(level)]["loglik"]}
            except MlblupError as e:   # C~ not positive definite for this tau
                res["sparsified"][key] = {"fill": round(s.basis.sparsity_pattern(level, tau) /
                                                        res["levels"][str(level)]["rows"] ** 2, 4),
                                          "error": str(e).split(":")[0]}
            print(f"sparsified loglik {key}: {res['sparsified'][key]}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    m = s.mle_rho(z, t - 1, wl.rho / 10, wl.rho * 10, 1e-4)
    res["mle_rho_level_t_minus_1"] = {"rho_hat": m["rho"], "loglik": m["loglik"], "evals": m["evals"],
                                      "s": round(time.perf_counter() - t0, 3), "rho_workload": wl.rho}
    print(json.dumps(res), flush=True)


def loglik_sparse_bench(k: int, n: int, reps: int = 3, dense: bool = True, nu: float = 0.0, rho: float = 0.0,
                        taus=(0.02, 0.05, 0.1), levels: int = 2):
    """Estimator with the sparse block factorization: l~_n at levels t and
    t - 1 for several tau, only the kept blocks formed and factored (host
    analysis timed on its own: pattern, minimum-degree order, block
    structure, wavelet vectors), each the median of `reps` calls after one
    untimed call; with `dense`, the dense sparsified path on the same matrix
    beside it (the N x N covariance must fit).  Flops: the block
    factorization's (w^3/3 per diagonal block, w_i w_k^2 per block below it,
    2 w_i w_j w_k per update) and the dense tail's T^3/3; the assembly,
    2 |S_a| |S_b| (w_b + 1) + 2 |S_a| w_a w_b per kept block pair, is not
    counted in TFLOP/s."""
    import time

    import numpy as np
    import torch

    import synth
    from paper_1701_00285_amd import MlblupError, Solver
    torch.cuda.set_device(0)
    wl = synth.make_config(k, n=n, n_targets=1)
    nu = nu or wl.nu
    rho = rho or wl.rho
    t0 = time.perf_counter()
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, nu, rho, wl.sigma2)
    setup = time.perf_counter() - t0
    z = torch.as_tensor(wl.z, dtype=torch.float64, device="cuda")
    top = s.basis.levels - 1
    res = {"workload": f"cfg{k} generator, n={n}, d={wl.d}, nu={nu}, rho={rho}, leaf={wl.leaf_max}, "
                       f"p={s.p}", "setup_s": round(setup, 3), "cases": {}}
    for level in (top, top - 1)[:levels]:
        for tau in taus:
            key = f"level {level} tau {tau}"
            t0 = time.perf_counter()
            info = s.loglik_sparse_info(level, tau)
            ana = time.perf_counter() - t0
            row = {"rows": info["rows"], "kept_fill": round(info["kept"] / info["rows"] ** 2, 5),
                   "factor_entries": info["factor_entries"], "block_columns": info["block_columns"],
                   "heights": info["heights"], "block_gflop": round(info["flops"] / 1e9, 3),
                   "tail_rows": info["tail_rows"], "tail_gflop": round(info["tail_flops"] / 1e9, 3),
                   "analysis_s": round(ana, 3)}
            try:
                s.loglik_sparse(z, level, tau)
                times = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    out = s.loglik_sparse(z, level, tau)
                    times.append(time.perf_counter() - t0)
                ms = 1e3 * float(np.median(times))
                row.update(ms=round(ms, 3), loglik=float(out["loglik"]), logdet=float(out["logdet"]),
                           quad=float(out["quad"]),
                           factor_tflops=round((info["flops"] + info["tail_flops"]) / (ms * 1e-3) / 1e12, 3))
            except MlblupError as e:   # C~ not positive definite for this tau
                row["error"] = str(e).split(":")[0]
            if dense and "error" not in row:
                s.loglik(z, level, tau=tau)
                times = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    d = s.loglik(z, level, tau=tau)
                    times.append(time.perf_counter() - t0)
                row.update(dense_ms=round(1e3 * float(np.median(times)), 3),
                           rel_diff_loglik=float(abs(d["loglik"] - row["loglik"]) / abs(d["loglik"])))
            res["cases"][key] = row
            print(f"sparse loglik {key}: {row}", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


def solve_bench(a):
    """The whole predictor path on one workload (a.config), a.warmup untimed
    and a.steps timed steps; returns the result dict (one JSON line):
    kd-tree and multilevel basis (host C++), basis upload, the
    preconditioner, W Z, the FP64 PCG solve of C_W gamma_W = Z_W to relres
    1e-8, the mixed-precision solve of the same system to the same FP64
    relres, the predictor of each path (warm-started from its own solution:
    true FP64 residual, gamma, beta-hat, predictions at the targets with FP64
    products) and Q, dQ/dlog rho of each.  `value` = logical covariance
    pairs of every product per second over the step."""
    import numpy as np
    import torch

    import synth
    from paper_1701_00285_amd import (FP32, FP64, MFMA_BF16X3, MIXED_FLEXIBLE, MIXED_RELIABLE, PREC_BLOCK,
                                      PREC_COARSE, PREC_JACOBI, VALUE, PcgOptions, Solver, profile_enable,
                                      profile_read)

    torch.cuda.set_device(0)
    wl = synth.make_config(a.config, n=a.n or None, n_targets=a.targets or None)
    wname = wl.name if not a.n else f"{wl.name}, generator at n={wl.n}"
    mixed = a.mixed if a.mixed >= 0 else (FP32 if wl.d < 8 else MFMA_BF16X3)
    if a.precond == "auto":
        # the coarse space for the smooth low-dimensional workloads; the rough
        # nu = 1/2 kernels in 10 and 20 dimensions converge fastest without one
        a.precond = "coarse" if wl.d < 8 else "none"
    scheme = {"flexible": MIXED_FLEXIBLE, "reliable": MIXED_RELIABLE}[a.scheme]
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda")
    P, Z, T = dev(wl.points), dev(wl.z), dev(wl.targets)
    torch.cuda.synchronize()

    def step(rec):
        t = [time.perf_counter()]
        pts_host = P.cpu().numpy()
        s = Solver(pts_host, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2, max_targets=T.shape[0])
        pc = {"block": PREC_BLOCK, "jacobi": PREC_JACOBI, "coarse": PREC_COARSE}.get(a.precond)
        pc = s.precond(pc) if pc is not None else None
        zt = s.to_tree(Z)
        zw, _ = s.apply_W(zt)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        o64 = PcgOptions(rtol=1e-8, max_iter=a.max_iter, precision=FP64, precond=pc)
        om = PcgOptions(rtol=1e-8, max_iter=a.max_iter, precision=mixed, inner_rtol=a.inner_rtol, precond=pc,
                        mixed_scheme=scheme)
        r = dict(solve_fp64=None, reference_fp64=None)
        if a.fp64_solve == "full":
            gw64, info64, st64 = s.solve(zw, o64, allow_noconv=True)
            torch.cuda.synchronize()
            t.append(time.perf_counter())
            r["solve_fp64"] = t[-1] - t[-2]
        gwm, infom, stm = s.solve(zw, om, allow_noconv=True)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        r["solve_mixed"] = t[-1] - t[-2]
        if a.fp64_solve == "refine":
            o_ref = PcgOptions(rtol=1e-10, max_iter=a.max_iter, precision=FP64, precond=pc)
            gw64, info64, st64 = s.solve(zw, o_ref, x0=gwm, allow_noconv=True)
            torch.cuda.synchronize()
            t.append(time.perf_counter())
            r["reference_fp64"] = t[-1] - t[-2]
        have64 = a.fp64_solve != "skip"
        # predictor of each path: FP64 residual check of its gamma_W, gamma,
        # beta-hat and the target products in FP64
        out = s.predict(Z, T, o64, gamma_w0=gw64, allow_noconv=True) if have64 else None
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        r["predict"] = t[-1] - t[-2]
        outm = s.predict(Z, T, om, gamma_w0=gwm, allow_noconv=True)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        r["predict_mixed"] = t[-1] - t[-2]
        q, dq = s.quad_grad(zt, out["gamma_tree"]) if have64 else (None, None)
        qm, dqm = s.quad_grad(zt, outm["gamma_tree"])
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        r["grad"] = t[-1] - t[-2]
        r["total"] = t[-1] - t[0]
        # for the record: the same results with low-precision kernel values in
        # the target products and in the gradient product (outside the timed
        # phases above)
        outl = s.predict(Z, T, om, predict_precision=mixed, gamma_w0=gwm, allow_noconv=True)
        _, dql = s.quad_grad(zt, outm["gamma_tree"], precision=mixed)
        mx = lambda u, v: float(torch.max(torch.abs(u - v)) / torch.max(torch.abs(v)))
        err = {}
        if have64:
            err = {"gamma_w_reldiff_mixed_vs_fp64": float(torch.linalg.norm(gwm - gw64) / torch.linalg.norm(gw64)),
                   "zhat_maxrelerr_mixed_vs_fp64": mx(outm["zhat"], out["zhat"]),
                   "beta_maxrelerr_mixed_vs_fp64": float(np.max(np.abs(outm["beta"] - out["beta"])) /
                                                         np.max(np.abs(out["beta"]))),
                   "dQ_relerr_mixed_vs_fp64": abs(dqm - dq) / abs(dq),
                   "zhat_maxrelerr_lowp_target_products": mx(outl["zhat"], out["zhat"]),
                   "dQ_relerr_lowp_grad_product": abs(dql - dq) / abs(dq)}
        rec.append(dict(r, setup=t[1] - t[0], info64=info64 if have64 else None, infom=infom,
                        infop=out["info"] if have64 else None, q=q, dq=dq, qm=qm, dqm=dqm, err=err, p=s.p,
                        converged=(stm == 0 and outm["status"] == 0 and
                                   (not have64 or (st64 == 0 and out["status"] == 0)))))

    warm = []
    for _ in range(a.warmup):
        step(warm)
    warm.clear()
    profile_enable(True)
    profile_read()
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(recs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = profile_read()
    profile_enable(False)

    total_pairs = sum(v[2] for v in prof.values())
    value = total_pairs / elapsed / 1e9
    n = wl.n
    ms64, n64, pairs64 = prof.get((FP64, VALUE), (0.0, 0, 0.0))
    msm, nm, pairsm = prof.get((mixed, VALUE), (0.0, 0, 0.0))
    last = recs[-1]
    have64 = a.fp64_solve != "skip"
    # the square launches of the FP64 product (the dominant kernel): logical
    # pairs n^2 each; the FP64 target launches (m x n: one per predictor that
    # runs, i.e. FP64 and mixed paths) are counted apart
    rect64 = a.steps * (2 if have64 else 1) * T.shape[0] * n
    sq64 = int(round((pairs64 - rect64) / (n * n))) if n64 else 0
    fpp = flops_per_unordered_pair(wl.d, wl.nu)
    i64, im, ip = last["info64"], last["infom"], last["infop"]
    rnd = lambda v, k=4: None if v is None else round(v, k)
    out = {
        "metric": "Matern C.x Gpairs/s (whole predictor step); BLUP solve time to relres 1e-8, FP64 vs mixed",
        "value": round(value, 3),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": wname, "n": n, "d": wl.d, "nu": wl.nu, "rho": wl.rho, "trend_p": last["p"],
                   "leaf": wl.leaf_max, "targets": int(T.shape[0]), "rtol": 1e-8,
                   "preconditioner": {"block": "cell blocks of C_W", "jacobi": "diag(C_W)",
                                      "coarse": "cell blocks of the finest level + dense coarse block of C_W",
                                      "none": "none"}[a.precond],
                   "mixed_precision": mixed, "mixed_scheme": a.scheme, "inner_rtol": a.inner_rtol,
                   "fp64_solve": a.fp64_solve},
        "phases_s": {k: rnd(last[k]) for k in ("setup", "solve_fp64", "solve_mixed", "reference_fp64", "predict",
                                                "predict_mixed", "grad", "total")},
        "solve": dict({"converged": last["converged"],
                       "fp64_s": rnd(last["solve_fp64"], 3), "mixed_s": round(last["solve_mixed"], 3),
                       "speedup": (round(last["solve_fp64"] / last["solve_mixed"], 3)
                                   if last["solve_fp64"] is not None else None),
                       "fp64_iters": i64["inner_iters"] if i64 else None,
                       "fp64_relres": i64["relres_fp64"] if i64 else None,
                       "mixed_outer": im["outer_iters"], "mixed_inner": im["inner_iters"],
                       "mixed_fp64_matvecs": im["fp64_matvecs"], "mixed_lowp_matvecs": im["lowp_matvecs"],
                       "mixed_relres_fp64": im["relres_fp64"],
                       "predict_warm_iters": ip["inner_iters"] if ip else None,
                       "predict_relres": ip["relres_fp64"] if ip else None}, **last["err"]),
        "pair_kernel": {
            "fp64_logical_gpairs_s": round(pairs64 / (ms64 * 1e-3) / 1e9, 2) if ms64 else None,
            "fp64_launches": n64, "fp64_avg_launch_ms": round(ms64 / n64, 4) if n64 else None,
            "mixed_logical_gpairs_s": round(pairsm / (msm * 1e-3) / 1e9, 2) if msm else None,
            "mixed_launches": nm, "mixed_avg_launch_ms": round(msm / nm, 4) if nm else None,
            "pairs_per_step": total_pairs / a.steps,
        },
    }
    # roofline of the dominant kernel: the FP64 square product (symmetric
    # kernel).  Algorithmic flops per launch = n(n+1)/2 distinct pairs x
    # flops_per_unordered_pair; the event time of those launches is the
    # bucket time minus the target launches' share (estimated at the same
    # per-pair rate as the bucket, which overstates their cost: conservative).
    if n64 and sq64 > 0:
        frac_sq = sq64 * n * n / pairs64
        t_sq = ms64 * 1e-3 * frac_sq
        achieved = sq64 * (n * (n + 1) / 2) * fpp / t_sq / 1e12
        traffic = measured_traffic(wl.name) if not a.n else None
        out["roofline"] = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 4),
                           "traffic": traffic,
                           "kernel": "sym_kernel FP64 value (square C x)", "launches": sq64,
                           "avg_launch_ms": round(t_sq / sq64 * 1e3, 4), "flops_per_unordered_pair": fpp}
        # the same launches against the VALU instruction-issue ceiling of the
        # kernel's own instruction mix (one lane evaluates one pair)
        vpp = valu_per_pair("fp64", wl.d, wl.nu)
        if vpp:
            ceil = 2 * VALU_LANE_RATE / vpp / 1e9   # logical (ordered) pairs per second
            got = sq64 * n * n / t_sq / 1e9
            out["roofline"]["issue_ceiling"] = {"valu_instr_per_pair": vpp, "ceiling_logical_gpairs_s": round(ceil, 1),
                                                "achieved_logical_gpairs_s": round(got, 1),
                                                "frac": round(got / ceil, 4)}
    out["grad"] = {"Q": last["q"], "dQ_dlogrho": last["dq"], "Q_mixed": last["qm"], "dQ_dlogrho_mixed": last["dqm"]}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_rows or default_cpu_rows(wl))
    return out




def segment_bench(a):
    """FP64 vs mixed solve to relres 1e-8 on a workload whose FP64 solve is
    longer than one run may last, in separate runs (a.segment):
      fp64-start:  the FP64 PCG from gamma_W = 0 for a.max_iter iterations;
                   gamma_W and the Krylov state (r, p, r.z) go to a.ckpt_out;
      fp64-resume: the same recurrence continued from a.ckpt_in to relres 1e-8
                   (an exact continuation: the iterates are those of one
                   uninterrupted solve), then the FP64 predictor at the targets
                   and Q, dQ/dlog rho; all of it to a.ckpt_out;
      mixed:       the mixed-precision solve (flexible CG, inner products on the
                   matrix cores or FP32), its predictor and gradient, compared
                   with the FP64 results in a.ckpt_in.
    Each run times its own solve with the host clock around synchronised calls
    (setup excluded) and prints one JSON line."""
    import numpy as np
    import torch

    import synth
    from paper_1701_00285_amd import (FP32, FP64, MFMA_BF16X3, MIXED_FLEXIBLE, MIXED_RELIABLE, PREC_COARSE,
                                      PcgOptions, Solver)
    torch.cuda.set_device(0)
    wl = synth.make_config(a.config, n=a.n or None, n_targets=a.targets or None)
    mixed = a.mixed if a.mixed >= 0 else (FP32 if wl.d < 8 else MFMA_BF16X3)
    scheme = {"flexible": MIXED_FLEXIBLE, "reliable": MIXED_RELIABLE}[a.scheme]
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2, max_targets=wl.targets.shape[0])
    pc = s.precond(PREC_COARSE) if a.precond == "coarse" else None
    Z, T = dev(wl.z), dev(wl.targets)
    zt = s.to_tree(Z)
    zw, _ = s.apply_W(zt)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    nw = s.n - s.p
    out = {"mode": f"segmented solve: {a.segment}", "workload": wl.name, "n": wl.n, "d": wl.d, "nu": wl.nu,
           "rho": wl.rho, "targets": int(T.shape[0]), "rtol": 1e-8,
           "preconditioner": "coarse" if pc is not None else "none", "setup_s": round(setup, 3)}
    if a.segment in ("fp64-start", "fp64-resume"):
        state = torch.empty(2 * nw + 8, dtype=torch.float64, device="cuda")
        x0, done_iters, done_s = None, 0, 0.0
        if a.segment == "fp64-resume":
            ck = np.load(os.path.join(a.ckpt_in, "fp64_state.npz"))
            x0 = dev(ck["gamma_w"])
            state.copy_(dev(ck["state"]))
            done_iters, done_s = int(ck["iters"]), float(ck["solve_s"])
        opts = PcgOptions(rtol=1e-8, max_iter=a.max_iter, precision=FP64, precond=pc, state=state,
                          resume=x0 is not None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gw, info, st = s.solve(zw, opts, x0=x0, allow_noconv=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        os.makedirs(a.ckpt_out, exist_ok=True)
        out.update({"segment_s": round(dt, 3), "segment_iters": info["inner_iters"],
                    "fp64_s_total": round(done_s + dt, 3), "fp64_iters_total": done_iters + info["inner_iters"],
                    "relres_fp64": info["relres_fp64"], "converged": st == 0})
        rec = dict(gamma_w=gw.cpu().numpy(), state=state.cpu().numpy(), iters=done_iters + info["inner_iters"],
                   solve_s=done_s + dt)
        if st == 0:
            o64 = PcgOptions(rtol=1e-8, max_iter=a.max_iter, precision=FP64, precond=pc)
            t2 = time.perf_counter()
            pr = s.predict(Z, T, o64, gamma_w0=gw, allow_noconv=True)
            q, dq = s.quad_grad(zt, pr["gamma_tree"])
            torch.cuda.synchronize()
            out.update({"predict_grad_s": round(time.perf_counter() - t2, 3), "Q": q, "dQ_dlogrho": dq})
            rec.update(zhat=pr["zhat"].cpu().numpy(), beta=pr["beta"], Q=q, dQ=dq)
        np.savez(os.path.join(a.ckpt_out, "fp64_state.npz"), **rec)
        return out
    # mixed
    om = PcgOptions(rtol=1e-8, max_iter=a.max_iter, precision=mixed, inner_rtol=a.inner_rtol, precond=pc,
                    mixed_scheme=scheme)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gwm, infom, stm = s.solve(zw, om, allow_noconv=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    o64 = PcgOptions(rtol=1e-8, max_iter=a.max_iter, precision=FP64, precond=pc)
    pr = s.predict(Z, T, o64, gamma_w0=gwm, allow_noconv=True)
    qm, dqm = s.quad_grad(zt, pr["gamma_tree"])
    torch.cuda.synchronize()
    out.update({"mixed_precision": mixed, "mixed_scheme": a.scheme, "inner_rtol": a.inner_rtol, "mixed_s": round(dt, 3),
                "mixed_inner": infom["inner_iters"], "mixed_outer": infom["outer_iters"],
                "mixed_fp64_matvecs": infom["fp64_matvecs"], "mixed_lowp_matvecs": infom["lowp_matvecs"],
                "relres_fp64": infom["relres_fp64"], "converged": stm == 0, "Q_mixed": qm, "dQ_dlogrho_mixed": dqm})
    if a.ckpt_in:
        ck = np.load(os.path.join(a.ckpt_in, "fp64_state.npz"))
        zh = pr["zhat"].cpu().numpy()
        g64 = ck["gamma_w"]
        out.update({"fp64_s": round(float(ck["solve_s"]), 3), "fp64_iters": int(ck["iters"]),
                    "speedup": round(float(ck["solve_s"]) / dt, 3),
                    "zhat_maxrelerr_mixed_vs_fp64": float(np.max(np.abs(zh - ck["zhat"])) / np.max(np.abs(ck["zhat"]))),
                    "beta_maxrelerr_mixed_vs_fp64": float(np.max(np.abs(pr["beta"] - ck["beta"])) /
                                                          np.max(np.abs(ck["beta"]))),
                    "gamma_w_reldiff_mixed_vs_fp64": float(np.linalg.norm(gwm.cpu().numpy() - g64) /
                                                           np.linalg.norm(g64)),
                    "dQ_relerr_mixed_vs_fp64": abs(dqm - float(ck["dQ"])) / abs(float(ck["dQ"]))})
    return out


def default_cpu_rows(wl) -> int:
    """Rows of the oracle's CPU product sample: about 4e9 / (n (d + 3))
    (10-20 s of one host core at the oracle's measured rates)."""
    return int(max(16, min(wl.n, 4e9 / (wl.n * (wl.d + 3)))))


def product_bench(a):
    """The headline line: a.warmup untimed and a.steps timed applications of
    the FP64 operator C_W of the solve on workload a.config (full size unless
    a.n), plus the records described in the module docstring."""
    import numpy as np
    import torch

    import synth
    from oracle import brute
    from paper_1701_00285_amd import (FP32, FP64, MFMA_BF16X3, VALUE, Solver, profile_enable, profile_read)

    torch.cuda.set_device(0)
    wl = synth.make_config(a.config, n=a.n or None, n_targets=1, with_z=False)
    wname = wl.name if not a.n else f"{wl.name}, generator at n={wl.n}"
    n, d = wl.n, wl.d
    print(f"bench: product line, {wname}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nw = n - s.p
    x = torch.as_tensor(synth.standard_normal(nw, 11), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    mixed = a.mixed if a.mixed >= 0 else (FP32 if d < 8 else MFMA_BF16X3)
    for _ in range(a.warmup):
        s.cw_matvec(x, FP64, out=y)
    torch.cuda.synchronize()
    profile_enable(True)
    profile_read()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s.cw_matvec(x, FP64, out=y)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = profile_read()
    ms64, n64, _ = prof[(FP64, VALUE)]
    print(f"bench: {a.steps} FP64 operator applications in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # the mixed-precision operator (the inner products of the mixed solve)
    ym = torch.empty_like(x)
    for _ in range(2):
        s.cw_matvec(x, mixed, out=ym)
    torch.cuda.synchronize()
    profile_read()
    reps = 5
    for _ in range(reps):
        s.cw_matvec(x, mixed, out=ym)
    torch.cuda.synchronize()
    msm, nm, _ = profile_read()[(mixed, VALUE)]
    profile_enable(False)
    err_mixed = float(torch.max(torch.abs(ym - y)) / torch.max(torch.abs(y)))
    # the FP64 covariance product itself against the oracle on 16 sampled rows
    av = s.apply_Wt(x)
    cv, _ = s.cov_matvec_tree(av, FP64)
    pts = s.basis.points_dev.cpu().numpy()
    a_host = av.cpu().numpy()
    idx = np.random.default_rng(a.config).choice(n, 16, replace=False)
    ref = brute.cov_matvec(pts[idx], pts, a_host, wl.nu, wl.rho, wl.sigma2)
    scale = brute.cov_matvec(pts[idx], pts, np.abs(a_host), wl.nu, wl.rho, wl.sigma2)
    rowerr = float(np.max(np.abs(cv.cpu().numpy()[idx] - ref) / scale))
    value = a.steps * n * n / elapsed / 1e9
    fpp = flops_per_unordered_pair(d, wl.nu)
    t_prod = ms64 * 1e-3 / n64                      # HIP-event time of one FP64 square product
    evaluated = n * (n + 1) / 2
    achieved = evaluated * fpp / t_prod / 1e12
    out = {
        "metric": "Matern C.x Gpairs/s; BLUP solve time to relres 1e-8, FP64 vs mixed",
        "value": round(value, 3),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": wname, "n": n, "d": d, "nu": wl.nu, "rho": wl.rho, "trend_p": s.p,
                   "leaf": wl.leaf_max,
                   "step": "one FP64 application of C_W = W C W^T (W^T, dense N x N covariance product, W)",
                   "pairs_per_step": "N^2 logical (ordered) pairs"},
        "setup_s": round(setup_s, 3),
        "fp64_product": {"events_ms": round(t_prod * 1e3, 3), "launches": n64,
                         "logical_gpairs_s": round(n * n / t_prod / 1e9, 2),
                         "evaluated_pairs_per_product": evaluated,
                         "evaluated_gpairs_s": round(evaluated / t_prod / 1e9, 2),
                         "rowerr_vs_oracle": rowerr},
        "mixed_product": {"precision": {FP32: "fp32", MFMA_BF16X3: "mfma_bf16x3"}.get(mixed, str(mixed)),
                          "events_ms": round(msm / nm, 3), "launches": nm,
                          "logical_gpairs_s": round(n * n / (msm / nm * 1e-3) / 1e9, 2),
                          "maxrelerr_vs_fp64_operator": err_mixed},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 4),
                     "traffic": measured_traffic(wl.name) if not a.n else None,
                     "kernel": "sym_kernel FP64 value (square C x; all dispatches of one product)",
                     "avg_launch_ms": round(t_prod * 1e3, 3), "flops_per_unordered_pair": fpp,
                     "unordered_pairs_per_launch": evaluated},
    }
    vpp = valu_per_pair("fp64", d, wl.nu)
    if vpp:
        ceil = 2 * VALU_LANE_RATE / vpp / 1e9
        got = n * n / t_prod / 1e9
        out["roofline"]["issue_ceiling"] = {"valu_instr_per_pair": vpp, "ceiling_logical_gpairs_s": round(ceil, 1),
                                            "achieved_logical_gpairs_s": round(got, 1), "frac": round(got / ceil, 4)}
    del s, x, y, ym, av, cv
    torch.cuda.empty_cache()
    if a.record_config:
        # the whole predictor path on its own workload, one warm and one timed step
        import argparse as _ap
        ra = _ap.Namespace(**vars(a))
        ra.config, ra.n, ra.targets, ra.steps, ra.warmup, ra.no_cpu = a.record_config, 0, 0, 1, 1, True
        ra.mixed = -1
        print(f"bench: whole-path record on workload {ra.config}", file=sys.stderr, flush=True)
        r = solve_bench(ra)
        out["solve_record"] = {"workload": r["config"]["workload"], "preconditioner": r["config"]["preconditioner"],
                               "mixed_precision": r["config"]["mixed_precision"],
                               "inner_rtol": r["config"]["inner_rtol"], "phases_s": r["phases_s"],
                               "solve": r["solve"], "grad": r["grad"],
                               "fp64_product_logical_gpairs_s": r["pair_kernel"]["fp64_logical_gpairs_s"]}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_rows or default_cpu_rows(wl))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=0,
                    help="workload 1-5 (default: 5 for the product line, 2 for --solve and --loglik)")
    ap.add_argument("--solve", action="store_true",
                    help="time the whole predictor path (tree, basis, preconditioner, FP64 and mixed solves to relres "
                         "1e-8, predictors, gradients) on --config instead of the product line")
    ap.add_argument("--record-config", type=int, default=2,
                    help="workload of the whole-path record carried by the product line (0: none)")
    ap.add_argument("--n", type=int, default=0, help="number of points drawn from the workload generator (0: its full size)")
    ap.add_argument("--targets", type=int, default=0, help="number of targets (0: the workload's)")
    ap.add_argument("--nu", type=float, default=0.0,
                    help="smoothness in place of the workload's (sweep: products only; a nu other than 1/2, 3/2, "
                         "5/2 or +inf takes the general-nu tables, FP64 and FP32)")
    ap.add_argument("--mixed", type=int, default=-1, help="precision of the mixed solve (default: FP32 for d<8, "
                                                          "matrix-core BF16 x3 for d>=8)")
    ap.add_argument("--scheme", choices=("flexible", "reliable"), default="flexible",
                    help="mixed-precision scheme: flexible CG around inner solves, or one recurrence with reliable "
                         "updates")
    ap.add_argument("--inner-rtol", type=float, default=0.35,
                    help="inner tolerance (flexible) or residual-replacement factor (reliable)")
    ap.add_argument("--fp64-solve", choices=("full", "refine", "skip"), default="full",
                    help="full: independent FP64 solve (timed against the mixed one); refine: FP64 PCG from the mixed "
                         "solution to relres 1e-10 as the error reference (for workloads where a full FP64 solve "
                         "does not fit the time budget); skip: none")
    ap.add_argument("--precond", choices=("auto", "block", "jacobi", "coarse", "none"), default="auto",
                    help="preconditioner of both solves: cell blocks of the finest level and one dense "
                         "coarse block of C_W (coarse; 2 N nc doubles of workspace while it is built), the cell "
                         "blocks of every level (block), diag(C_W) (jacobi), none, or auto (coarse for d < 8, "
                         "none otherwise)")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the oracle's CPU product sample (0: about 15 s of one core's work)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-iter", type=int, default=40000,
                    help="Krylov iteration cap (lower it only for short profiling runs)")
    ap.add_argument("--sweep", default="",
                    help="comma-separated workloads: time every precision's product, the target product and W / W^T "
                         "(one JSON line each) instead of the step")
    ap.add_argument("--reps", type=int, default=10,
                    help="with --sweep: timed launches per product (after min(3, reps) untimed ones)")
    ap.add_argument("--loglik", type=int, default=0,
                    help="estimator: time the multilevel log-likelihood (dense C^n_W, blocked Cholesky) and the "
                         "rho MLE on this many points of the workload's generator (one JSON line) instead of the step")
    ap.add_argument("--cpu-oracle", choices=("all", "products", "blup"), default=None,
                    help="time the oracle on the host's cores (covariance products, dense classic BLUP) beside "
                         "the GPU predictor; one JSON line instead of the step")
    ap.add_argument("--loglik-quick", action="store_true",
                    help="with --loglik: levels t and 0 only, one timed call each")
    ap.add_argument("--loglik-sparse", type=int, default=0,
                    help="estimator with the sparse block factorization of the kept blocks: levels t and t - 1, "
                         "several tau, on this many points of the workload's generator (one JSON line)")
    ap.add_argument("--rho", type=float, default=0.0,
                    help="with --loglik-sparse: range of the covariance (default: the workload's)")
    ap.add_argument("--taus", default="0.02,0.05,0.1", help="with --loglik-sparse: comma-separated tau values")
    ap.add_argument("--no-dense", action="store_true",
                    help="with --loglik-sparse: skip the dense sparsified path beside it (large n)")
    ap.add_argument("--sparse-levels", type=int, choices=(1, 2), default=2,
                    help="with --loglik-sparse: level t only (1) or levels t and t - 1 (2)")
    ap.add_argument("--segment", choices=("fp64-start", "fp64-resume", "mixed"), default=None,
                    help="one segment of a FP64 vs mixed comparison split over several runs (default workload 5): "
                         "the FP64 solve for --max-iter iterations, its exact continuation, or the mixed solve")
    ap.add_argument("--ckpt-in", default="", help="directory of the FP64 segment to continue or compare with")
    ap.add_argument("--ckpt-out", default="", help="directory receiving the FP64 segment's state")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 512 MiB three times with a plain device copy (reference for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: the path runs on one GPU; --gpus {a.gpus} is not supported (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if a.sweep:
        sweep([int(v) for v in a.sweep.split(",")], reps=a.reps, warm=min(3, a.reps), nu=a.nu or None)
        return

    if a.loglik:
        loglik_bench(a.config or 2, a.loglik, quick=a.loglik_quick)
        return

    if a.loglik_sparse:
        loglik_sparse_bench(a.config or 2, a.loglik_sparse, dense=not a.no_dense, nu=a.nu, rho=a.rho,
                            taus=tuple(float(v) for v in a.taus.split(",")), levels=a.sparse_levels)
        return

    if a.cpu_oracle:
        cpu_oracle_report(a.cpu_oracle)
        return

    if a.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 8, "launches": 3}), flush=True)
        return

    if a.segment:
        a.config = a.config or 5
        if a.precond == "auto":
            a.precond = "none"
        print(json.dumps(segment_bench(a)), flush=True)
        return

    if a.solve:
        a.config = a.config or 2
        print(json.dumps(solve_bench(a)), flush=True)
        return
    a.config = a.config or 5
    print(json.dumps(product_bench(a)), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the multilevel BLUP solve on one MI355X.

One step = one pass of the whole hot path over one synthetic workload:
kd-tree and multilevel basis (host C++), basis upload, W Z, the FP64 PCG
solve of C_W gamma_W = Z_W to relres 1e-8, the mixed-precision solve of
the same system to the same FP64 relres (iterative refinement), beta-hat,
predictions at the targets, Q and dQ/dlog rho.  Inputs (points, Z,
targets) are resident in HBM when the timed region starts.

The default workload is 65,536 uniform points in [0,1]^3, Matern nu=3/2,
rho=0.2, quadratic trend (p=10), leaf 64, 4,096 targets.

Prints ONE JSON line.  `value` = logical covariance pairs evaluated per
second over the whole step (Gpairs/s); the per-phase times, the solve
times (FP64 vs mixed), the pair-kernel rates measured with HIP events on
the launch stream, the roofline object of the dominant kernel (the FP64
pair kernel) and the CPU oracle baseline are added to the same line.
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


def flops_per_pair(d: int, nu: float) -> int:
    """Algorithmic flops of one pair (FMA = 2): d differences + d squared
    accumulations (3d), sqrt (1), exp (1), the Matern polynomial (nu=1/2: 0,
    3/2: 1+z and the product with e^-z = 2, 5/2: 1+z+z^2/3 (two FMA) and the
    product = 5) and the accumulation FMA (2)."""
    poly = {0.5: 0, 1.5: 2, 2.5: 5}[nu]
    return 3 * d + 4 + poly


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--mixed", type=int, default=-1, help="precision of the mixed solve (default: FP32 for d<8, "
                                                          "MFMA FP32 for d>=8)")
    ap.add_argument("--cpu-rows", type=int, default=3072)
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {a.gpus} is not supported (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1701_00285_amd import (DLOGRHO, FP32, FP64, MFMA_FP32, VALUE, PcgOptions, Solver, profile_enable,
                                      profile_read)

    torch.cuda.set_device(0)
    wl = synth.make_config(a.config)
    mixed = a.mixed if a.mixed >= 0 else (FP32 if wl.d < 8 else MFMA_FP32)
    dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda")
    P, Z, T = dev(wl.points), dev(wl.z), dev(wl.targets)
    torch.cuda.synchronize()

    def step(rec):
        t = [time.perf_counter()]
        pts_host = P.cpu().numpy()
        s = Solver(pts_host, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2, max_targets=T.shape[0])
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        out = s.predict(Z, T, PcgOptions(rtol=1e-8, precision=FP64))
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        zt = s.to_tree(Z)
        zw, _ = s.apply_W(zt)
        gw_m, info_m, _ = s.solve(zw, PcgOptions(rtol=1e-8, precision=mixed, inner_rtol=1e-4))
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        q, dq = s.quad_grad(zt, out["gamma_tree"])
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        rec.append(dict(setup=t[1] - t[0], predict_fp64=t[2] - t[1], solve_mixed=t[3] - t[2], grad=t[4] - t[3],
                        total=t[4] - t[0], info64=out["info"], infom=info_m, q=q, dq=dq,
                        gamma_w64=out["gamma_w"], gamma_wm=gw_m, solver=s))

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

    # FP64-only solve time (separately timed, same system): the predict phase
    # contains extra products (beta, targets)
    s = recs[-1]["solver"]
    zw, _ = s.apply_W(s.to_tree(Z))
    torch.cuda.synchronize()
    ts = time.perf_counter()
    gw64, info64s, _ = s.solve(zw, PcgOptions(rtol=1e-8, precision=FP64))
    torch.cuda.synchronize()
    solve64 = time.perf_counter() - ts
    ts = time.perf_counter()
    gwm, infoms, _ = s.solve(zw, PcgOptions(rtol=1e-8, precision=mixed, inner_rtol=1e-4))
    torch.cuda.synchronize()
    solvem = time.perf_counter() - ts
    rel_diff = float(torch.linalg.norm(gwm - gw64) / torch.linalg.norm(gw64))

    total_pairs = sum(v[2] for v in prof.values())
    value = total_pairs / elapsed / 1e9
    ms64, n64, pairs64 = prof.get((FP64, VALUE), (0.0, 0, 0.0))
    msm, nm, pairsm = prof.get((mixed, VALUE), (0.0, 0, 0.0))
    fpp = flops_per_pair(wl.d, wl.nu)
    achieved = pairs64 * fpp / (ms64 * 1e-3) / 1e12 if ms64 > 0 else 0.0
    last = recs[-1]
    out = {
        "metric": "Matern C.x Gpairs/s (whole step); BLUP solve time to relres 1e-8, FP64 vs mixed",
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
        "config": {"workload": wl.name, "n": wl.n, "d": wl.d, "nu": wl.nu, "rho": wl.rho, "trend_p": s.p,
                   "leaf": wl.leaf_max, "targets": int(T.shape[0]), "rtol": 1e-8, "mixed_precision": mixed},
        "phases_s": {k: round(last[k], 4) for k in ("setup", "predict_fp64", "solve_mixed", "grad", "total")},
        "solve_s": {"fp64": round(solve64, 4), "mixed": round(solvem, 4), "speedup": round(solve64 / solvem, 3),
                    "fp64_iters": info64s["inner_iters"], "fp64_matvecs": info64s["fp64_matvecs"],
                    "mixed_inner_iters": infoms["inner_iters"], "mixed_outer": infoms["outer_iters"],
                    "mixed_fp64_matvecs": infoms["fp64_matvecs"], "mixed_lowp_matvecs": infoms["lowp_matvecs"],
                    "relres_fp64": info64s["relres_fp64"],
                    "relres_mixed": infoms["relres_fp64"], "gamma_w_reldiff_mixed_vs_fp64": rel_diff},
        "pair_kernel": {
            "fp64_gpairs_s": round(pairs64 / (ms64 * 1e-3) / 1e9, 2) if ms64 else None,
            "fp64_launches": n64, "fp64_avg_launch_ms": round(ms64 / n64, 4) if n64 else None,
            "mixed_gpairs_s": round(pairsm / (msm * 1e-3) / 1e9, 2) if msm else None,
            "mixed_launches": nm, "mixed_avg_launch_ms": round(msm / nm, 4) if nm else None,
            "pairs_per_step": total_pairs / a.steps,
            "flops_per_pair": fpp,
        },
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 4), "traffic": None,
                     "kernel": "pair_kernel FP64 VALUE (square + target products)"},
        "grad": {"Q": last["q"], "dQ_dlogrho": last["dq"]},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

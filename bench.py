#!/usr/bin/env python3
"""Benchmark of the tensor-product three-body eigensolver on one MI355X.

One step is one complete block Jacobi-Davidson QR solve of the workload, from a
seeded start block to the wanted eigenpairs at the FP64 residual tolerance: it
runs every stage of the hot path (Hamiltonian applies with the fused potential,
the kinetic Sylvester preconditioner, GMRES on the correction equation, FP64
block orthogonalisation and Rayleigh-Ritz).  Operator set-up (grids, potential
table, preconditioner eigen-factors) happens before the timed region; the start
block is generated on the device.

Printed: one JSON line with the solve time (value), the Hamiltonian-apply
throughput of the dominant kernel measured with HIP events inside the timed
solves against the FP64 MFMA peak (roofline), the eigenvalue error against the
CPU oracle's stored values, the same solve with FP32 inner GMRES ("mixed"), the
H apply at the precision-form grid c3 (h_apply_c3, context: n = 1024 fills the
matrix cores where c2's n = 256 is latency-bound), the 256-instance batched
workload (batched_c4), and the CPU oracle timed on this host (cpu_baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2] [--gmres-steps 3]

The GMRES step count per correction equation is a solver setting, not part of
the workload: on c2 the solve is bound by per-launch latency, and 3 steps per
outer iteration reach the same eigenvalues in less time than the library
default of 10 (more, cheaper outer iterations).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-apply GFLOP/s (% MFMA peak); JDQR s to k eigenpairs @1e-10, mixed vs FP64"
# HBM bytes per launch of the FP64 H apply at n = 256, 8 vectors (32 x 32 tile
# split over eight waves, K-chunks of 64), from rocprofv3 FETCH_SIZE /
# WRITE_SIZE scaled by a 256 MiB copy (profiles/hbm_traffic_c2_H_apply_fp64.md):
# 16508 KiB read + 4096 KiB written.  None for other workloads.
TRAFFIC_BYTES = {"c2": 16508 * 1024 + 4096 * 1024}
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
HBM_PEAK_GBS = 8000.0


def apply_flops(n):
    """Algorithmic flops of one 1D Hamiltonian apply to one vector: two dense
    mode products (2 n_x n_y (n_x + n_y)) plus the potential term (3 n_x n_y)."""
    nx, ny = n
    return 2.0 * nx * ny * (nx + ny) + 3.0 * nx * ny


def golden(name):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}_evals.txt")
    if not os.path.exists(path):
        return None, None
    iters = None
    with open(path) as f:
        for line in f:
            if "outer iterations" in line:
                for tok in line.replace(";", " ").replace(",", " ").split():
                    if tok.isdigit():
                        iters = int(tok)
                        break
    return np.loadtxt(path)[:, 0], iters


def cpu_baseline(cfg, name, sample_iters, full_iters, gmres_steps):
    """The oracle's block JDQR on the same workload and settings, timed for its
    first `sample_iters` outer iterations and scaled to a full solve of
    `full_iters` outer iterations."""
    import numpy as np
    from oracle import jdqr, problem
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    P = problem.make_problem(**cfg)
    pc = P.preconditioner()
    sig = P.two_body_shift()
    t0 = time.perf_counter()
    r = jdqr.jdqr(P.apply, P.N, cfg["nev"], cfg["block"], precond=pc.apply,
                  seed=cfg["seed_start"], target=sig, target_low=P.spectrum_lower_bound(),
                  max_outer=sample_iters, gmres_steps=gmres_steps)
    dt = time.perf_counter() - t0
    n_done = max(r.n_outer, 1)
    per_iter = dt / n_done
    full = full_iters if full_iters else n_done
    return {"value": per_iter * full, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": (f"first {n_done} outer iterations of the oracle's {name} solve with "
                       f"{gmres_steps} GMRES steps per correction ({dt:.1f} s measured), scaled to "
                       f"the {full} outer iterations of the full solve; "
                       f"NumPy/SciPy FP64, {threads} BLAS threads")}


def apply_c3_leg(reps=20):
    """Context for the H-apply metric at the precision-form grid c3 (n = 1024,
    16 vectors): for each precision every tile shape is timed (HIP events
    around `reps` launches on the stream the library uses) and the fastest is
    reported, against the MFMA peak of the precision (BF16x3: FP32-equivalent
    flops against the 2.5 PFLOP/s dense bf16 peak divided by its three bf16
    products per FP32 product)."""
    import torch

    import paper_2111_02534_amd as t3
    from workloads import config
    cfg = config("c3")
    n, b = cfg["n"], cfg["block"]
    op = t3.Operator.from_config(cfg)
    out = {"workload": f"c3: 1D, n={n} (N={op.N}), {b} vectors per apply"}
    tiles = {0: "32x32", 1: "64x64", 2: "128x128", 3: "64x128", 4: "32x32 (8 waves)"}
    for name, pk, dt, peak in (("fp64", t3.FP64, torch.float64, PEAK_TFLOPS["f64"]),
                               ("fp32", t3.FP32, torch.float32, PEAK_TFLOPS["f32"]),
                               ("bf16x3", t3.BF16X3, torch.float32, 2500.0 / 3.0)):
        X = torch.randn((b, op.N), dtype=dt, device="cuda")
        Y = torch.empty_like(X)
        best = None
        for tile in tiles:
            if pk == t3.BF16X3 and tile in (0, 4):
                continue  # runs as 64 x 64
            op.set_tile(tile)
            op.apply_H(X, Y, prec=pk)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                op.apply_H(X, Y, prec=pk)
            e1.record()
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / reps
            if best is None or us < best[0]:
                best = (us, tiles[tile])
        op.set_tile(-1)
        us, tile = best
        tf = b * apply_flops((n, n)) / (us * 1e-6) / 1e12
        out[name] = {"us_per_apply": us, "tile": tile, "tflops": tf, "peak": peak, "frac": tf / peak}
    op.close()
    return out


def batched_leg(reps, n_seq, gmres_steps):
    """The 256-instance workload c4: one batched JDQR solve (grouped persistent
    launches, GMRES iteration replayed as a HIP graph) per repetition, for each
    inner precision; eigenvalues against the oracle's stored values; and the
    first `n_seq` instances solved one by one with the single-instance solver
    (FP32 inner) for comparison."""
    import numpy as np
    import torch

    import paper_2111_02534_amd as t3
    from workloads import C4_TOL, c4_instances
    inst = c4_instances()
    path = os.path.join(ROOT, "tests", "golden", "c4_evals.txt")
    gold = np.loadtxt(path)[:, 5:9] if os.path.exists(path) else None
    t0 = time.perf_counter()
    ops = [t3.Operator.from_config(c) for c in inst]
    t_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    for pk in (t3.FP64, t3.FP32, t3.BF16X3):
        t3.autotune_batched(ops, pk, nvec=4, reps=2)
    t_tune = time.perf_counter() - t0
    res = {"instances": len(ops), "nev": 4, "block": 4, "gmres_steps": gmres_steps,
           "create_s": t_create, "autotune_s": t_tune}
    kw = dict(seed=1000, tol=C4_TOL, gmres_steps=gmres_steps)
    for name, pk in (("fp64", t3.FP64), ("fp32", t3.FP32), ("bf16x3", t3.BF16X3)):
        t3.jdqr_batched(ops, 4, 4, inner_prec=pk, **kw)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            r = t3.jdqr_batched(ops, 4, 4, inner_prec=pk, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        err = (float(np.max(np.abs(r.evals - gold) / np.maximum(np.abs(gold), 1.0)))
               if gold is not None else None)
        res[name] = {"s_per_batch": dt, "instances_per_s": len(ops) / dt,
                     "outer_iters_max": int(r.n_outer.max()),
                     "outer_iters_mean": float(r.n_outer.mean()),
                     "eig_max_err_vs_oracle_rel_to_max_abs_1": err}
    if n_seq > 0:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for op in ops[:n_seq]:
            op.jdqr(4, 4, inner_prec=t3.FP32, seed=0, want_Q=False, tol=C4_TOL,
                    gmres_steps=gmres_steps)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t1) / n_seq
        res["sequential_fp32"] = {"instances": n_seq, "s_per_instance": per,
                                  "projected_s_for_batch": per * len(ops),
                                  "batched_speedup": per * len(ops) / res["fp32"]["s_per_batch"]}
    for op in ops:
        op.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=3)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--gmres-steps", type=int, default=3,
                    help="GMRES steps per correction equation in the timed solves")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-c3-apply", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--batched-seq", type=int, default=32,
                    help="instances of the batch solved one by one for comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2111_02534_amd as t3
    from workloads import config

    torch.cuda.init()
    cfg = config(args.config)
    nev, b = cfg["nev"], cfg["block"]
    op = t3.Operator.from_config(cfg)
    n = (cfg["n"], cfg["n"])
    ref, _ = golden(args.config)

    def solve(inner, profile=False):
        return op.jdqr(nev, b, inner_prec=inner, seed=cfg["seed_start"], want_Q=False,
                       profile=profile, gmres_steps=args.gmres_steps)

    for _ in range(args.warmup):
        solve(t3.FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(solve(t3.FP64, profile=True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s_per_solve = elapsed / args.steps

    # Dominant kernel: the FP64 Hamiltonian apply (b vectors per launch).  The
    # events bracket the launches made outside the replayed GMRES graph (the
    # applies that extend the search space), which run the same kernel on the
    # same block width.
    t_k = sum(r.stats["t_kernel"][0] for r in res)
    n_k = sum(r.stats["n_kernel"][0] for r in res)
    n_vec = sum(r.stats["v_kernel"][0] for r in res)
    vec_per_launch = n_vec / max(n_k, 1)
    flops_launch = vec_per_launch * apply_flops(n)
    avg_launch_s = t_k / max(n_k, 1)
    achieved_tf = flops_launch / avg_launch_s / 1e12 if avg_launch_s > 0 else 0.0
    t_prec = sum(r.stats["t_kernel"][2] for r in res)
    err = None
    if ref is not None:
        err = float(max(np.max(np.abs(r.evals - ref) / np.abs(ref)) for r in res))

    out = {
        "metric": METRIC,
        "value": s_per_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * s_per_solve,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.config}: 1D three-body, n={cfg['n']} per Jacobi coordinate "
                                f"(N={op.N}), M/m={cfg['alpha']}, Gaussian V0={cfg['v0']}, "
                                f"w={cfg['width']}, lowest {nev} eigenpairs, block {b}, "
                                f"FP64 JDQR + Sylvester preconditioner, "
                                f"{args.gmres_steps} GMRES steps per correction"),
                   "n": cfg["n"], "nev": nev, "block": b, "gmres_steps": args.gmres_steps},
        "roofline": {"bound": "mfma", "achieved": achieved_tf, "peak": PEAK_TFLOPS["f64"],
                     "unit": "TFLOP/s", "frac": achieved_tf / PEAK_TFLOPS["f64"],
                     "traffic": TRAFFIC_BYTES.get(args.config),
                     "kernel": "k_modeprod_sk8<double, 0> (H apply, fused potential)",
                     "launch_flops": flops_launch, "avg_launch_us": 1e6 * avg_launch_s,
                     "launches": n_k},
        "h_apply_gflops": achieved_tf * 1e3,
        "jdqr": {"s_per_solve": s_per_solve, "outer_iters": res[-1].stats["n_outer"],
                 "apply_H_vectors": res[-1].stats["n_apply_H_fp64"],
                 "apply_prec_vectors": res[-1].stats["n_apply_prec"],
                 "kernel_time_frac_H": t_k / elapsed, "kernel_time_frac_prec": t_prec / elapsed,
                 "eig_max_rel_err_vs_oracle": err},
    }
    if not args.no_mixed:
        solve(t3.FP32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mres = [solve(t3.FP32) for _ in range(max(1, args.steps // 2))]
        torch.cuda.synchronize()
        m_s = (time.perf_counter() - t1) / len(mres)
        m_err = None
        if ref is not None:
            m_err = float(max(np.max(np.abs(r.evals - ref) / np.abs(ref)) for r in mres))
        out["mixed_vs_fp64"] = {"fp64_s": s_per_solve, "mixed_s": m_s, "speedup": s_per_solve / m_s,
                                "mixed_outer_iters": mres[-1].stats["n_outer"],
                                "mixed_eig_max_rel_err_vs_oracle": m_err}
    if not args.no_c3_apply:
        out["h_apply_c3"] = apply_c3_leg()
    if not args.no_batched:
        out["batched_c4"] = batched_leg(args.batched_reps, args.batched_seq, args.gmres_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.config, args.cpu_sample_iters,
                                           res[-1].stats["n_outer"], args.gmres_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

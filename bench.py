#!/usr/bin/env python3
"""Benchmark of the tensor-product three-body eigensolver on one MI355X.

One step is one complete block Jacobi-Davidson QR solve of the 2D workload c5
(four tensor modes, n = 64 per mode, N = 16,777,216 unknowns per vector; the
largest workload that one GPU holds), from a seeded start block to the 6 wanted
eigenpairs at the FP64 residual tolerance, with the 2D kinetic preconditioner:
it runs every stage of the hot path (2D Hamiltonian applies with the fused
potential, the preconditioner, GMRES on the correction equation, FP64 block
orthogonalisation and Rayleigh-Ritz).  Operator set-up happens before the
timed region; the start block is generated on the device; no step is
PCIe-inclusive (the boundary takes device buffers).

Printed: one JSON line with the seconds per FP64 solve (value); the same solve
with FP32 inner GMRES (mixed); the 2D Hamiltonian apply against the FP64 MFMA
roofline (HIP events on the library's stream, 8 vectors per apply) and the
other applies; the H-apply error of every precision at sampled entries against
the oracle's stored values; the eigenvalue error against the oracle at the
reduced 2D size c5r; the 1D workloads c2 and c3 (solve times, applies, errors
against the oracle's stored eigenvalues) and the 256-instance batch c4; and the
CPU oracle timed on this host (cpu_baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--gmres-steps S] [--m-max M]
    python bench.py --apply-sweep c3 [--prec fp64 fp32 bf16x3]   # per-tile apply times
    python bench.py --counters c5 --prec fp64 [--kind P]          # for rocprofv3 --pmc runs
    python bench.py --leg c2                                      # one extra leg alone
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-apply GFLOP/s (% MFMA peak); JDQR s to k eigenpairs @1e-10, mixed vs FP64"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
HBM_PEAK_GBS = 8000.0
# HBM bytes per 8-vector apply of the 2D Hamiltonian at c5 (FP64; the two plane
# passes, run vector by vector): rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by
# what the counter reads for a 256 MiB device copy in the same run
# (profiles/hbm_traffic_c5_plane_passes_fp64.md; 5,682,882 KiB).  Set to None
# when the plane kernels change until the counters are taken again.
TRAFFIC_BYTES = {"c5": 5682882 * 1024}


def apply_flops(ndim, n, kind="H"):
    """Algorithmic flops of one apply to one vector: 2D H 8n^5 + 3n^4 (four
    mode products of 2 n^5 each, potential 3 n^4); 1D H 4n^3 + 3n^2; 1D
    preconditioner 8n^3 + n^2; 2D preconditioner 16 n^5 + n^4."""
    if ndim == 2:
        return 8.0 * n ** 5 + 3.0 * n ** 4 if kind == "H" else 16.0 * n ** 5 + 1.0 * n ** 4
    return 4.0 * n ** 3 + 3.0 * n ** 2 if kind == "H" else 8.0 * n ** 3 + 1.0 * n ** 2


def apply_bytes(ndim, n, es, kind="H"):
    """Algorithmic HBM bytes per vector of the applies as implemented: 2D H in
    two passes, read X + write Y, then read X + read Y + write Y (the Gaussian
    potential from separable factors): 5 N es; 2D preconditioner in four passes
    of one read and one write: 8 N es; 1D: read X (+ V), write Y."""
    N = n ** (2 * ndim)
    if ndim == 2:
        return (5 if kind == "H" else 8) * N * es
    return 3 * N * es


def golden_evals(name):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}_evals.txt")
    if not os.path.exists(path):
        return None
    return np.loadtxt(path, ndmin=2)[:, 0]


def golden_samples(name):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}_apply_samples.txt")
    if not os.path.exists(path):
        return None
    return np.loadtxt(path, ndmin=2)


def rel_err(a, ref):
    import numpy as np
    a, ref = np.asarray(a, dtype=float), np.asarray(ref, dtype=float)
    return float(np.max(np.abs(a - ref) / np.abs(ref)))


def rel_err_max1(a, ref):
    """max |a - ref| / max(|ref|, 1): the scale of the residual test."""
    import numpy as np
    a, ref = np.asarray(a, dtype=float), np.asarray(ref, dtype=float)
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 1.0)))


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def time_applies(op, X, Y, prec, kind, reps):
    """Microseconds per apply: HIP events on the stream the library launches
    on (torch's current stream, passed to every call) around `reps` applies."""
    import torch
    f = op.apply_H if kind == "H" else op.apply_prec
    f(X, Y, prec=prec)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        f(X, Y, prec=prec)
    e1.record()
    torch.cuda.synchronize()
    return 1e3 * e0.elapsed_time(e1) / reps


def sampled_apply_errors(t3, op, name, cfg, reps):
    """H-apply error at the oracle's stored sample entries for every precision
    (componentwise |dY| / (|H||w|)), on the seeded input block; plus the apply
    timings on that block."""
    import numpy as np
    import torch

    from workloads import normal_block
    smp = golden_samples(name)
    b = cfg["block"]
    Xn = normal_block(op.N, b, cfg["seed_apply"])
    X64 = torch.from_numpy(Xn).cuda()
    del Xn
    out = {}
    for pname, pk, dt in (("fp64", t3.FP64, torch.float64), ("fp32", t3.FP32, torch.float32),
                          ("bf16x3", t3.BF16X3, torch.float32)):
        X = X64 if dt == torch.float64 else X64.float()
        Y = torch.empty_like(X)
        op.apply_H(X, Y, prec=pk)
        torch.cuda.synchronize()
        ent = {}
        if smp is not None:
            vs, idx = smp[:, 0].astype(int), smp[:, 1].astype(int)
            got = Y[torch.from_numpy(vs).cuda(), torch.from_numpy(idx).cuda()].double().cpu().numpy()
            ent["err_componentwise_vs_oracle"] = float(np.max(np.abs(got - smp[:, 2]) / smp[:, 3]))
            ent["err_normwise_samples_vs_oracle"] = float(np.linalg.norm(got - smp[:, 2]) /
                                                          np.linalg.norm(smp[:, 2]))
            ent["samples"] = int(smp.shape[0])
        us = time_applies(op, X, Y, pk, "H", reps)
        tf = b * apply_flops(cfg["ndim"], cfg["n"]) / (us * 1e-6) / 1e12
        ent.update({"us_per_apply": us, "vectors": b, "tflops": tf, "peak_tflops": PEAK_TFLOPS[pname],
                    "frac": tf / PEAK_TFLOPS[pname]})
        usp = time_applies(op, X, Y, pk, "P", reps)
        tfp = b * apply_flops(cfg["ndim"], cfg["n"], "P") / (usp * 1e-6) / 1e12
        ent["prec"] = {"us_per_apply": usp, "tflops": tfp, "frac": tfp / PEAK_TFLOPS[pname]}
        out[pname] = ent
        del X, Y
    del X64
    torch.cuda.empty_cache()
    return out


def solve_leg(op, cfg, inner, steps, gmres_steps, nev=None, block=None, want_Q=False, m_max=0):
    import torch
    nev = nev or cfg["nev"]
    block = block or cfg["block"]
    res = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res.append(op.jdqr(nev, block, inner_prec=inner, seed=cfg["seed_start"], want_Q=want_Q,
                           gmres_steps=gmres_steps, m_max=m_max, m_min=m_max // 2))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1), res


def stats_brief(r):
    st = r.stats
    return {"outer_iters": st["n_outer"], "restarts": st["n_restart"],
            "apply_H_vectors_fp64": st["n_apply_H_fp64"], "apply_H_vectors_low": st["n_apply_H_low"],
            "apply_prec_vectors": st["n_apply_prec"], "stall_locked_pairs": st["n_stall_lock"],
            "dependent_columns_replaced": st["n_dep_replaced"]}


def c5r_leg(t3, gmres_steps):
    """The 2D problem at n = 20 per mode against the oracle's stored eigenvalues."""
    from workloads import config
    cfg = config("c5r")
    ref = golden_evals("c5r")
    op = t3.Operator.from_config(cfg)
    out = {"workload": f"c5r: 2D, n={cfg['n']} per mode (N={op.N}), lowest {cfg['nev']}, "
                       f"block {cfg['block']}"}
    for name, pk in (("fp64", t3.FP64), ("fp32_inner", t3.FP32), ("bf16x3_inner", t3.BF16X3)):
        t0 = time.perf_counter()
        r = op.jdqr(cfg["nev"], cfg["block"], inner_prec=pk, seed=cfg["seed_start"], want_Q=False,
                    gmres_steps=gmres_steps, tol=cfg["tol"])
        ent = {"s_per_solve": time.perf_counter() - t0, "outer_iters": r.stats["n_outer"],
               "tol": cfg["tol"]}
        if ref is not None:
            ent["eig_max_rel_err_vs_oracle"] = rel_err(r.evals, ref)
        out[name] = ent
    op.close()
    return out


def c2_leg(t3, reps, gmres_steps):
    from workloads import config
    cfg = config("c2")
    ref = golden_evals("c2")
    op = t3.Operator.from_config(cfg)
    out = {"workload": f"c2: 1D, n={cfg['n']} (N={op.N}), lowest {cfg['nev']}, block {cfg['block']}, "
                       f"{gmres_steps} GMRES steps"}
    for name, pk in (("fp64", t3.FP64), ("fp32_inner", t3.FP32)):
        solve_leg(op, cfg, pk, 1, gmres_steps)
        t, res = solve_leg(op, cfg, pk, reps, gmres_steps)
        ent = {"s_per_solve": t, **stats_brief(res[-1])}
        if ref is not None:
            ent["eig_max_rel_err_vs_oracle"] = max(rel_err(r.evals, ref) for r in res)
        out[name] = ent
    out["mixed_speedup"] = out["fp64"]["s_per_solve"] / out["fp32_inner"]["s_per_solve"]
    op.close()
    return out


def c3_leg(t3, gmres_steps, reps):
    """n = 1024, 16 vectors: applies per precision with their sampled error,
    and full solves (FP64, FP32-inner, BF16x3-inner) against the oracle."""
    from workloads import config
    cfg = config("c3")
    ref = golden_evals("c3")
    op = t3.Operator.from_config(cfg)
    out = {"workload": f"c3: 1D, n={cfg['n']} (N={op.N}), {cfg['block']} vectors per apply; "
                       f"lowest {cfg['nev']}, {gmres_steps} GMRES steps"}
    out["apply"] = sampled_apply_errors(t3, op, "c3", cfg, reps)
    for name, pk in (("fp64", t3.FP64), ("fp32_inner", t3.FP32), ("bf16x3_inner", t3.BF16X3)):
        t, res = solve_leg(op, cfg, pk, 1, gmres_steps)
        ent = {"s_per_solve": t, **stats_brief(res[-1])}
        if ref is not None:
            ent["eig_max_rel_err_vs_oracle"] = rel_err(res[-1].evals, ref)
            ent["eig_max_err_vs_oracle_rel_max1"] = rel_err_max1(res[-1].evals, ref)
        out[name] = ent
    for name in ("fp32_inner", "bf16x3_inner"):
        out[name]["speedup_vs_fp64"] = out["fp64"]["s_per_solve"] / out[name]["s_per_solve"]
    op.close()
    return out


def batched_leg(t3, reps, n_seq, gmres_steps):
    """The 256-instance workload c4: one batched JDQR solve per repetition and
    inner precision; eigenvalues against the oracle's stored values (plain
    relative error |dE| / |E| per state); the first n_seq instances solved one
    by one (FP32 inner) for comparison."""
    import numpy as np
    import torch

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
    res = {"instances": len(ops), "nev": 4, "block": 4, "gmres_steps": gmres_steps,
           "create_s": t_create, "autotune_s": time.perf_counter() - t0}
    kw = dict(seed=1000, tol=C4_TOL, gmres_steps=gmres_steps)
    for name, pk in (("fp64", t3.FP64), ("fp32", t3.FP32), ("bf16x3", t3.BF16X3)):
        t3.jdqr_batched(ops, 4, 4, inner_prec=pk, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            r = t3.jdqr_batched(ops, 4, 4, inner_prec=pk, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        ent = {"s_per_batch": dt, "instances_per_s": len(ops) / dt,
               "outer_iters_max": int(r.n_outer.max()), "outer_iters_mean": float(r.n_outer.mean()),
               "stall_locked_pairs": int(r.stats["n_stall_lock"])}
        if gold is not None:
            rel = np.abs(r.evals - gold) / np.abs(gold)
            ent["eig_max_rel_err_vs_oracle"] = float(rel.max())
            ent["states_above_1e-10"] = int((rel > 1e-10).sum())
            ent["instances_above_1e-10"] = sorted({int(i) for i in np.nonzero(rel > 1e-10)[0]})
        res[name] = ent
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


def cpu_baseline(cfg, gpu_stats):
    """The CPU oracle on this host: one 2D Hamiltonian apply and one 2D
    preconditioner apply (Bartels-Stewart over four modes) of one vector of the
    c5 workload, at one BLAS thread and at all of them; the solve projected from
    the apply counts of the GPU's FP64 solve (orthogonalisation and
    Rayleigh-Ritz left out, so the projection is a lower bound)."""
    import numpy as np

    from oracle import problem
    from workloads import normal_block
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
        threadpool_info = None
    model, ncpu, avail = host_info()
    P = problem.make_problem(**cfg)
    pc = P.preconditioner()
    x = normal_block(P.N, 1, cfg["seed_apply"])[0]
    out = {}
    nthreads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1]) if threadpool_info else avail
    for label, limit in (("1_thread", 1), ("all_threads", None)):
        ctx = threadpool_limits(limits=limit) if (threadpool_limits and limit) else None
        try:
            if ctx:
                ctx.__enter__()
            t0 = time.perf_counter()
            P.apply(x)
            ta = time.perf_counter() - t0
            t0 = time.perf_counter()
            pc.apply(x)
            tp = time.perf_counter() - t0
        finally:
            if ctx:
                ctx.__exit__(None, None, None)
        out[label] = {"s_apply_H_per_vector": ta, "s_apply_prec_per_vector": tp}
    nH = gpu_stats["apply_H_vectors_fp64"] + gpu_stats["apply_H_vectors_low"]
    nP = gpu_stats["apply_prec_vectors"]
    proj = {k: v["s_apply_H_per_vector"] * nH + v["s_apply_prec_per_vector"] * nP for k, v in out.items()}
    return {"value": proj["all_threads"], "unit": "s", "cores": int(nthreads), "kind": "oracle",
            "projected": True,
            "sample": (f"oracle (NumPy/SciPy FP64) 2D H apply and 2D Bartels-Stewart preconditioner of "
                       f"one c5 vector (N={P.N}), timed once each at 1 and at {nthreads} BLAS threads; "
                       f"value = per-vector times x the {nH} H-apply and {nP} preconditioner vectors of "
                       f"the GPU's FP64 solve (projected; orthogonalisation and Rayleigh-Ritz excluded)"),
            "host_cpu": model, "host_cpus": ncpu, "host_cpus_available": avail,
            "per_vector": out, "projected_s_1_thread": proj["1_thread"]}


def apply_sweep(args):
    """Per-tile timing of the 1D applies (set_tile), then the autotuner."""
    import torch

    import paper_2111_02534_amd as t3
    from workloads import config
    tiles = {0: "32x32", 1: "64x64", 2: "128x128", 3: "64x128", 4: "32x32w8"}
    for name in args.apply_sweep:
        cfg = config(name)
        n, b = cfg["n"], cfg["block"]
        op = t3.Operator.from_config(cfg)
        print(f"== {name}: ndim={cfg['ndim']} n={n} N={op.N} block={b}", flush=True)
        for pname, pk, dt in (("fp64", t3.FP64, torch.float64), ("fp32", t3.FP32, torch.float32),
                              ("bf16x3", t3.BF16X3, torch.float32)):
            if args.prec and pname not in args.prec:
                continue
            X = torch.randn((b, op.N), dtype=dt, device="cuda")
            Y = torch.empty_like(X)
            for tile, tname in tiles.items():
                if cfg["ndim"] == 1 and tile in (1, 2, 3) and n < (64 if tile == 1 else 128):
                    continue
                if pk == t3.BF16X3 and tile in (0, 4):
                    continue
                op.set_tile(tile)
                for kind in ("H", "P"):
                    us = time_applies(op, X, Y, pk, kind, args.reps)
                    tf = b * apply_flops(cfg["ndim"], n, kind) / (us * 1e-6) / 1e12
                    print(f"  {pname} tile {tname:8s} {kind}: {us:10.1f} us {tf:8.2f} TFLOP/s "
                          f"{100 * tf / PEAK_TFLOPS[pname]:5.1f}% of peak", flush=True)
            op.set_tile(-1)
            if cfg["ndim"] == 1:
                best = op.autotune(pk, b, 5)
                print(f"  autotuned: H {1e3 * best[0]:.1f} us, P {1e3 * best[1]:.1f} us", flush=True)
        op.close()


def counters(args):
    """For hardware-counter runs: the workload's Hamiltonian apply (or, with
    --kind P, its preconditioner) in the first listed precision, repeated
    --reps times, then a device-to-device copy of --copy-mb MiB (the
    calibration kernel for byte counters)."""
    import torch

    import paper_2111_02534_amd as t3
    from workloads import config
    pname = (args.prec or ["fp64"])[0]
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[pname]
    dt = torch.float64 if pname == "fp64" else torch.float32
    for name in args.counters:
        cfg = config(name)
        op = t3.Operator.from_config(cfg)
        X = torch.randn((cfg["block"], op.N), dtype=dt, device="cuda")
        Y = torch.empty_like(X)
        f = op.apply_H if args.kind == "H" else op.apply_prec
        for _ in range(args.reps):
            f(X, Y, prec=pk)
        torch.cuda.synchronize()
        print(f"{name} {pname} {args.kind}: {args.reps} applies of {cfg['block']} vectors, N = {op.N}; "
              f"block {cfg['block'] * op.N * X.element_size()} bytes", flush=True)
        op.close()
        del X, Y
    n = args.copy_mb * (1 << 20) // 4
    A = torch.ones(n, dtype=torch.float32, device="cuda")
    B = torch.empty_like(A)
    B.copy_(A)
    torch.cuda.synchronize()
    print(f"copy: {n * 4} bytes read, {n * 4} bytes written", flush=True)


def orth_timing(args):
    """Block orthogonalisation alone (tp3b_block_orth without factors: the
    queued CGS2 + Cholesky-QR sequence JDQR runs on its expansion block) on an
    N x nq block Q and an N x nx block X, --reps calls, each on a fresh copy of
    X.  Prints the time per call (HIP events around the call; the call itself
    synchronises) and the algorithmic bytes of the sequence's kernels."""
    import torch

    import paper_2111_02534_amd as t3
    N, nq, nx = args.orth
    g = torch.Generator(device="cuda").manual_seed(7)
    Q = torch.randn((nq, N), dtype=torch.float64, device="cuda", generator=g)
    X0 = torch.randn((nx, N), dtype=torch.float64, device="cuda", generator=g)
    X = X0.clone()
    times = []
    for rep in range(args.reps + 2):
        X.copy_(X0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, rank = t3.block_orth(Q, X, want_factors=False)
        e1.record()
        torch.cuda.synchronize()
        if rep >= 2:
            times.append(e0.elapsed_time(e1) * 1e3)
    us = sum(times) / len(times)
    # Gram of the input, Q^T X, two fused update+dot passes, two triangular
    # solves and the second Gram matrix: 8 N (3 nq + 11 nx) bytes
    nbytes = 8 * N * (3 * nq + 11 * nx)
    print(json.dumps({"orth": {"N": N, "nq": nq, "nx": nx, "rank": rank, "us_per_call": us,
                               "algorithmic_bytes": nbytes, "TBps": nbytes / (us * 1e-6) / 1e12}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--gmres-steps", type=int, default=3,
                    help="GMRES steps per correction equation in the timed c5 solves")
    ap.add_argument("--m-max", type=int, default=64,
                    help="search-space size before a restart in the timed c5 solves (m_min = m_max / 2; "
                         "0: the library's default)")
    ap.add_argument("--mixed-steps", type=int, default=0, help="timed mixed solves (0: steps // 2)")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true", help="only the c5 legs and the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=2)
    ap.add_argument("--batched-seq", type=int, default=16)
    ap.add_argument("--apply-sweep", nargs="*", default=None, metavar="WORKLOAD")
    ap.add_argument("--counters", nargs="*", default=None, metavar="WORKLOAD")
    ap.add_argument("--kind", default="H", choices=["H", "P"])
    ap.add_argument("--prec", nargs="*", default=None)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mb", type=int, default=256)
    ap.add_argument("--orth", nargs=3, type=int, default=None, metavar=("N", "NQ", "NX"),
                    help="time the block orthogonalisation alone at this shape")
    ap.add_argument("--leg", default=None, choices=["c2", "c3", "c4", "c5r"],
                    help="run one of the extra legs alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.apply_sweep:
        return apply_sweep(args)
    if args.counters:
        return counters(args)
    if args.orth:
        return orth_timing(args)

    import torch

    import paper_2111_02534_amd as t3
    from workloads import config

    torch.cuda.init()
    if args.leg:
        legs = {"c2": lambda: c2_leg(t3, max(3, args.steps), 3),
                "c3": lambda: c3_leg(t3, 10, args.apply_reps),
                "c4": lambda: batched_leg(t3, args.batched_reps, args.batched_seq, 3),
                "c5r": lambda: c5r_leg(t3, args.gmres_steps)}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return
    cfg = config("c5")
    nev, b, n = cfg["nev"], cfg["block"], cfg["n"]
    op = t3.Operator.from_config(cfg)
    gs, mm = args.gmres_steps, args.m_max

    # ---- the timed FP64 solves (the step)
    if args.warmup > 0:
        solve_leg(op, cfg, t3.FP64, args.warmup, gs, m_max=mm)
    s_fp64, res = solve_leg(op, cfg, t3.FP64, args.steps, gs, m_max=mm)
    fp64_stats = stats_brief(res[-1])
    # ---- the same solve with FP32 inner GMRES
    msteps = args.mixed_steps or max(1, args.steps // 2)
    solve_leg(op, cfg, t3.FP32, 1, gs, m_max=mm)
    s_mixed, mres = solve_leg(op, cfg, t3.FP32, msteps, gs, m_max=mm)
    agree = max(rel_err(r.evals, res[-1].evals) for r in mres)

    # ---- applies: roofline of the Hamiltonian apply, sampled errors
    applies = sampled_apply_errors(t3, op, "c5", cfg, args.apply_reps)
    h64 = applies["fp64"]
    launch_flops = b * apply_flops(2, n)
    achieved = launch_flops / (h64["us_per_apply"] * 1e-6) / 1e12
    op.close()
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": s_fp64,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * s_fp64,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"c5: 2D three-body (four tensor modes), n={n} per mode "
                                f"(N={16777216} per vector), M/m={cfg['alpha']}, Gaussian V0={cfg['v0']}, "
                                f"w={cfg['width']}, lowest {nev} eigenpairs, block {b}, FP64 JDQR with "
                                f"the 2D kinetic preconditioner, {gs} GMRES steps per correction, "
                                f"restart from m_max={mm or 'default'} to m_min={mm // 2 or 'default'}"),
                   "n": n, "nev": nev, "block": b, "gmres_steps": gs, "m_max": mm or None},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["fp64"],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["fp64"],
                     "traffic": TRAFFIC_BYTES.get("c5"),
                     "traffic_note": ("HBM bytes per launch, rocprofv3 FETCH_SIZE + WRITE_SIZE scaled "
                                      "by a 256 MiB copy; the algorithmic bytes are below"),
                     "kernel": ("2D Hamiltonian apply, FP64, per vector: k_plane2d_x4<P2_SUM> (x slabs) + "
                                "k_plane2d_y1<double, P2_SUM_V_ACC> (y planes with the potential)"),
                     "launch_flops": launch_flops, "avg_launch_us": h64["us_per_apply"],
                     "algorithmic_bytes": b * apply_bytes(2, n, 8),
                     "achieved_GBs": b * apply_bytes(2, n, 8) / (h64["us_per_apply"] * 1e-6) / 1e9},
        "h_apply_gflops": achieved * 1e3,
        "jdqr": {"s_per_solve": s_fp64, **fp64_stats,
                 "eig_agreement_fp64_vs_mixed": agree},
        "mixed_vs_fp64": {"fp64_s": s_fp64, "mixed_s": s_mixed, "speedup": s_fp64 / s_mixed,
                          "mixed_outer_iters": mres[-1].stats["n_outer"],
                          "eig_max_rel_diff_vs_fp64": agree},
        "applies_c5": applies,
    }
    out["c5r_vs_oracle"] = c5r_leg(t3, gs)
    if not args.no_extras:
        out["c2"] = c2_leg(t3, max(3, args.steps), 3)
        out["c3"] = c3_leg(t3, 10, args.apply_reps)
        out["batched_c4"] = batched_leg(t3, args.batched_reps, args.batched_seq, 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, fp64_stats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

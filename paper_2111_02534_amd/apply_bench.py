"""Times the Hamiltonian and preconditioner applies of a workload on the GPU for
every mode-product tile shape (HIP events), then runs the autotuner.

    python -m paper_2111_02534_amd.apply_bench c3 [c2 ...] [--reps 20]

Reports microseconds per apply of the workload's block and the algorithmic
throughput against the MFMA peak of the precision (FP64 78.6, FP32 157.3
TFLOP/s; BF16x3 is reported as FP32-equivalent TFLOP/s and as a fraction of the
2.5 PFLOP/s dense bf16 peak counting its three bf16 products per FP32 product).
1D flops per vector: 4n^3 + 3n^2 (H), 8n^3 + n^2 (preconditioner);
2D: 8n^5 + 3n^4 (H)."""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}


def flops(ndim, n, nvec, kind):
    if ndim == 2:
        return nvec * (8.0 * n ** 5 + 3.0 * n ** 4)
    return nvec * ((4.0 * n ** 3 + 3.0 * n ** 2) if kind == "H" else (8.0 * n ** 3 + n ** 2))


def counters(args):
    import torch

    import paper_2111_02534_amd as t3
    from workloads import config
    pname = (args.prec or ["fp64"])[0]
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[pname]
    dt = torch.float64 if pname == "fp64" else torch.float32
    for name in args.names:
        cfg = config(name)
        op = t3.Operator.from_config(cfg)
        X = torch.randn((cfg["block"], op.N), dtype=dt, device="cuda")
        Y = torch.empty_like(X)
        for _ in range(args.reps):
            op.apply_H(X, Y, prec=pk)
        torch.cuda.synchronize()
        es = X.element_size()
        print(f"{name} {pname}: {args.reps} applies of {cfg['block']} vectors, N = {op.N}; "
              f"block {cfg['block'] * op.N * es} bytes", flush=True)
        op.close()
    n = args.copy_mb * (1 << 20) // 4
    A = torch.ones(n, dtype=torch.float32, device="cuda")
    B = torch.empty_like(A)
    B.copy_(A)
    torch.cuda.synchronize()
    print(f"copy: {n * 4} bytes read, {n * 4} bytes written", flush=True)


def main():
    import torch

    import paper_2111_02534_amd as t3
    from workloads import config

    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--prec", nargs="*", default=None, help="subset of fp64 fp32 bf16x3")
    ap.add_argument("--counters", action="store_true",
                    help="for hardware-counter runs: only the workload's Hamiltonian apply in the "
                         "first listed precision with the built-in tile choice, repeated --reps "
                         "times, then a device-to-device copy of --copy-mb MiB (the calibration "
                         "kernel for byte counters)")
    ap.add_argument("--copy-mb", type=int, default=256)
    args = ap.parse_args()
    if args.counters:
        return counters(args)
    for name in args.names:
        cfg = config(name)
        n, b, ndim = cfg["n"], cfg["block"], cfg["ndim"]
        t0 = time.time()
        op = t3.Operator.from_config(cfg)
        print(f"== {name}: ndim={ndim} n={n} N={op.N} block={b} (create {time.time() - t0:.1f} s)",
              flush=True)
        for dt, pk, pname in [(torch.float64, t3.FP64, "fp64"), (torch.float32, t3.FP32, "fp32"),
                              (torch.float32, t3.BF16X3, "bf16x3")]:
            if args.prec and pname not in args.prec:
                continue
            X = torch.randn((b, op.N), dtype=dt, device="cuda")
            Y = torch.empty_like(X)
            kinds = ("H", "P") if ndim == 1 else ("H",)
            for tile in range(5):
                tm, tn = [(32, 32), (64, 64), (128, 128), (64, 128), (32, 32)][tile]
                if tm > 32 and (tm > n or tn > n) and ndim == 1:
                    continue
                if pk == t3.BF16X3 and tm == 32:
                    continue
                op.set_tile(tile)
                for kind in kinds:
                    g = op.apply_H if kind == "H" else op.apply_prec

                    def f(X, Y, g=g):
                        return g(X, Y, prec=pk)
                    f(X, Y)
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(args.reps):
                        f(X, Y)
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / args.reps
                    tf = flops(ndim, n, b, kind) / ms / 1e9
                    print(f"  {pname} tile {tm}x{tn}{'w8' if tile == 4 else ''} {kind}: {1e3 * ms:10.1f} us  {tf:7.2f} TFLOP/s"
                          f"  {100 * tf / PEAK[pname]:5.1f}% of peak", flush=True)
            op.set_tile(-1)
            if ndim == 1:
                best = op.autotune(pk, b, 5)
                print(f"  autotuned best: H {1e3 * best[0]:.1f} us, P {1e3 * best[1]:.1f} us", flush=True)
        op.close()


if __name__ == "__main__":
    main()

"""Writes the stored eigenvalue references under tests/golden/ by running the
CPU oracle only (block JDQR with the Bartels-Stewart preconditioner, FP64).

    python tests/golden/make_golden.py c2
    python tests/golden/make_golden.py c3
    python tests/golden/make_golden.py c4 [--procs 8]
    python tests/golden/make_golden.py c4dense [--procs 8]
    python tests/golden/make_golden.py c5r
    python tests/golden/make_golden.py samples

Each output file holds the nev converged eigenvalues of the named workload
(ascending) and the oracle's final residual norms.  For the batched workload c4
the file holds one line per instance: index, n, M/m, V0, w and the 4 lowest
eigenvalues (instances solved independently in a process pool).  c4dense: for every instance
of the batched workload with n = 64 (N = 4096) the 4 eigenvalues of smallest real
part of the explicit Kronecker matrix (dense eigensolver, the plain definition).
c3 (n = 1024 per mode) is computed from its four parity sectors
(oracle.parity: each sector has n/2 unknowns per mode and is solved by the same
block JDQR; the spectrum of H is the union of the sectors' spectra).
c5r: the 2D workload c5 at n = 20 per mode (N = 160,000), the reduced size at
which the oracle's four-mode preconditioned JDQR finishes in minutes.
samples: for the apply inputs of c2, c3 and c5 (the seeded N(0,1) blocks of
their seed_apply, in their solve block widths), H w and |H||w| at 300 seeded
random entries of the first and the last vector, each entry computed from the
operator's definition (oracle.operator.apply_1d_at / apply_2d_at)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import jdqr, problem  # noqa: E402
from workloads import config  # noqa: E402


def run(name):
    c = config(name)
    P = problem.make_problem(**c)
    pc = P.preconditioner()
    sig = P.two_body_shift()
    t = time.time()
    t0 = time.time()

    def progress(outer, nlock, rn, theta):
        print(f"  {name} outer {outer} locked {nlock} theta0 {theta[0]:.12g} "
              f"res0 {rn[0]:.3e} ({time.time() - t0:.0f} s)", flush=True)

    tol = c.get("tol", 1e-12)
    r = jdqr.jdqr(P.apply, P.N, c["nev"], c["block"], precond=pc.apply, seed=c["seed_start"],
                  target=sig, target_low=P.spectrum_lower_bound(), max_outer=400,
                  progress=progress, tol=tol)
    dt = time.time() - t
    assert r.converged, name
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_evals.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest {c['nev']} eigenvalues of workload {name} "
                f"(n={c['n']}, L={c['L']}, M/m={c['alpha']}, V0={c['v0']}, w={c['width']}),\n")
        f.write("# computed by the CPU FP64 oracle (block JDQR, Bartels-Stewart preconditioner,\n")
        f.write(f"# residual tolerance {tol:g} max(|theta|, 1)); {r.n_outer} outer iterations, {dt:.1f} s.\n")
        f.write(f"# two-body shift sigma = {sig:.17g}\n")
        for e, rn in zip(r.evals.real, r.resnorm):
            f.write(f"{e:.17g} {rn:.3e}\n")
    print(name, r.evals.real, r.n_outer, f"{dt:.1f}s", flush=True)


def run_parity(name, per_sector, block):
    from oracle import parity
    c = config(name)
    P = problem.make_problem(**c)
    sig = P.two_body_shift()
    lo = P.spectrum_lower_bound()
    t0 = time.time()

    def progress(s, outer, nlock, rn, theta):
        print(f"  {name} sector {s} outer {outer} locked {nlock} theta0 {theta[0]:.12g} "
              f"res0 {rn[0]:.3e} ({time.time() - t0:.0f} s)", flush=True)

    ev, info = parity.lowest_by_parity(c, c["nev"], block, per_sector, sig, lo,
                                       seed=c["seed_start"], max_outer=400, progress=progress)
    dt = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_evals.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest {c['nev']} eigenvalues of workload {name} "
                f"(n={c['n']}, L={c['L']}, M/m={c['alpha']}, V0={c['v0']}, w={c['width']}),\n")
        f.write("# computed by the CPU FP64 oracle from the four parity sectors (x, y even/odd,\n")
        f.write(f"# n/2 unknowns per mode; block JDQR, block {block}, Bartels-Stewart preconditioner,\n")
        f.write(f"# residual tolerance 1e-12 max(|theta|, 1)); {dt:.1f} s.\n")
        f.write(f"# two-body shift sigma = {sig:.17g}\n")
        for sec, evs, rns, no in info:
            f.write(f"# sector {sec}: {len(evs)} eigenvalues, {no} outer iterations, "
                    f"largest {evs[-1]:.17g}\n")
        f.write("# eigenvalue sector_px sector_py resnorm\n")
        for e in ev:
            for sec, evs, rns, no in info:
                hit = np.nonzero(evs == e)[0]
                if hit.size:
                    f.write(f"{e:.17g} {sec[0]} {sec[1]} {rns[hit[0]]:.3e}\n")
                    break
    print(name, ev, f"{dt:.1f}s", flush=True)


def run_samples(names=("c2", "c3", "c5"), count=300):
    from oracle import operator
    from workloads import normal_block
    for name in names:
        c = config(name)
        P = problem.make_problem(**c)
        b = c["block"]
        X = normal_block(P.N, b, c["seed_apply"])
        rng = np.random.Generator(np.random.PCG64(4242))
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_apply_samples.txt")
        with open(out, "w") as f:
            f.write(f"# Samples of H w for workload {name}: w = vector v of normal_block(N={P.N}, "
                    f"{b}, seed={c['seed_apply']}),\n")
            f.write("# entries drawn by PCG64(4242); H w and |H||w| from the operator's "
                    "definition (CPU FP64 oracle).\n")
            f.write("# vector index Hw absH_absw\n")
            for v in (0, b - 1):
                idx = rng.integers(0, P.N, count)
                W = X[v].reshape(P.n)
                if P.ndim == 1:
                    ref, sc = operator.apply_1d_at(P.D2[0], P.D2[1], P.cx, P.cy, P.V, W, idx)
                else:
                    ref, sc = operator.apply_2d_at(P.D2, P.cx, P.cy, P.V, W, idx)
                for e, r, q in zip(idx, ref, sc):
                    f.write(f"{v} {e} {r:.17g} {q:.17g}\n")
        del X
        print("samples", name, flush=True)


def _c4_one(args):
    i, c = args
    P = problem.make_problem(**c)
    pc = P.preconditioner()
    sig = P.two_body_shift()
    r = jdqr.jdqr(P.apply, P.N, c["nev"], c["block"], precond=pc.apply, seed=c["seed_start"],
                  target=sig, target_low=P.spectrum_lower_bound(), max_outer=400, tol=c["tol"])
    if not r.converged:
        return i, np.full(c["nev"], np.nan), float("nan"), r.n_outer
    return i, r.evals.real.copy(), float(np.max(r.resnorm)), r.n_outer


def run_c4(procs):
    from multiprocessing import Pool

    from workloads import c4_instances
    inst = c4_instances()
    t = time.time()
    res = []
    # largest grids first, so that the pool drains evenly
    order = sorted(range(len(inst)), key=lambda i: -inst[i]["n"])
    with Pool(procs) as pool:
        for k, out in enumerate(pool.imap_unordered(_c4_one, [(i, inst[i]) for i in order])):
            res.append(out)
            print(f"  {k + 1}/{len(inst)} instance {out[0]} n={inst[out[0]]['n']} "
                  f"outer {out[3]}", flush=True)
    res.sort(key=lambda r: r[0])
    bad = [r[0] for r in res if not np.all(np.isfinite(r[1]))]
    if bad:
        raise SystemExit(f"instances without convergence: {bad}")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_evals.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest 4 eigenvalues of each of the {len(inst)} instances of workload c4,\n")
        f.write("# computed by the CPU FP64 oracle (block JDQR, block 4, Bartels-Stewart\n")
        f.write(f"# preconditioner, residual tolerance {inst[0]['tol']:g} max(|theta|, 1)); "
                f"{time.time() - t:.0f} s in total.\n")
        f.write("# index n alpha v0 width e0 e1 e2 e3 max_resnorm outer_iterations\n")
        for (i, ev, rn, it), c in zip(res, inst):
            f.write(f"{i} {c['n']} {c['alpha']:.17g} {c['v0']:.17g} {c['width']:.17g} "
                    + " ".join(f"{e:.17g}" for e in ev) + f" {rn:.3e} {it}\n")
    print("c4", len(res), f"{time.time() - t:.1f}s", flush=True)


def _c4_dense_one(args):
    from oracle import dense
    i, c = args
    P = problem.make_problem(**c)
    return i, dense.lowest_eigenvalues(P.kron(), c["nev"]).real.copy()


def run_c4_dense(procs):
    from multiprocessing import Pool

    from workloads import c4_instances
    inst = c4_instances()
    todo = [(i, c) for i, c in enumerate(inst) if c["n"] == 64]
    t = time.time()
    res = []
    with Pool(procs) as pool:
        for k, out in enumerate(pool.imap_unordered(_c4_dense_one, todo)):
            res.append(out)
            print(f"  {k + 1}/{len(todo)} instance {out[0]}", flush=True)
    res.sort(key=lambda r: r[0])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_dense_n64.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest 4 eigenvalues (smallest real part) of the explicit Kronecker matrix of\n")
        f.write(f"# each of the {len(todo)} instances of workload c4 with n = 64 (N = 4096),\n")
        f.write(f"# dense eigensolver of the CPU oracle; {time.time() - t:.0f} s in total.\n")
        f.write("# index e0 e1 e2 e3\n")
        for i, ev in res:
            f.write(f"{i} " + " ".join(f"{e:.17g}" for e in ev) + "\n")
    print("c4dense", len(res), f"{time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    procs = 8
    if "--procs" in args:
        k = args.index("--procs")
        procs = int(args[k + 1])
        del args[k:k + 2]
    for name in args:
        if name == "c4":
            run_c4(procs)
        elif name == "c4dense":
            run_c4_dense(procs)
        elif name == "samples":
            run_samples()
        elif name == "c3":
            run_parity("c3", {(1, 1): 10, (-1, 1): 10, (1, -1): 4, (-1, -1): 4}, 8)
        else:
            run(name)

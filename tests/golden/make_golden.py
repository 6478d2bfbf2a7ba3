"""Writes the stored eigenvalue references under tests/golden/ by running the
CPU oracle only (block JDQR with the Bartels-Stewart preconditioner, FP64).

    python tests/golden/make_golden.py c2 [c3 ...]

Each output file holds the nev converged eigenvalues of the named workload
(ascending) and the oracle's final residual norms."""
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
    r = jdqr.jdqr(P.apply, P.N, c["nev"], c["block"], precond=pc.apply, seed=c["seed_start"],
                  target=sig, max_outer=400)
    dt = time.time() - t
    assert r.converged, name
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_evals.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest {c['nev']} eigenvalues of workload {name} "
                f"(n={c['n']}, L={c['L']}, M/m={c['alpha']}, V0={c['v0']}, w={c['width']}),\n")
        f.write("# computed by the CPU FP64 oracle (block JDQR, Bartels-Stewart preconditioner,\n")
        f.write(f"# residual tolerance 1e-12); {r.n_outer} outer iterations, {dt:.1f} s.\n")
        f.write(f"# two-body shift sigma = {sig:.17g}\n")
        for e, rn in zip(r.evals.real, r.resnorm):
            f.write(f"{e:.17g} {rn:.3e}\n")
    print(name, r.evals.real, r.n_outer, f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        run(name)

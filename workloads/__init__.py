"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds problem parameters and random numbers only.  It contains none
of the method's arithmetic (no grids, operators, potentials or solvers), so that
the CPU oracle and the GPU path can both draw identical inputs from it without
sharing any numerical code.

The paper's experiments are parametric physics problems (masses, potential depth
and shape, grid size; Sec. 5, Tables 1-3); there is no dataset to stand in for.
The five workloads below are the tensor-product problems this library is
measured on:

* ``c1`` 1D, n = 32 interior points per Jacobi coordinate (N = 1024), mass ratio
  M/m = 20, Gaussian depth 1, lowest 3 eigenpairs with block size 4, FP64.
* ``c2`` 1D, n = 256 (N = 65,536), M/m = 20, depth 2, lowest 10, block 8, FP64.
* ``c3`` 1D, n = 1024 (N = 1,048,576), M/m = 50, depth 4, lowest 16, block 16;
  low-precision inner solves, FP64 outer iteration.
* ``c4`` 256 independent 1D instances, n drawn from {64, 96, 128, 192, 256},
  M/m log-uniform in [1, 100], depth uniform in [0.5, 5], width uniform in
  [0.5, 2]; lowest 4, block 4.
* ``c5`` 2D (four tensor modes), n = 64 per mode (N = 16,777,216), M/m = 20,
  depth 3, lowest 6, block 8.
* ``c5r`` the same 2D problem at n = 20 per mode (N = 160,000): the reduced size
  at which the CPU oracle's eigensolver finishes in minutes.

All use Chebyshev-Gauss-Lobatto grids on [-15, 15] with Dirichlet conditions and
the Gaussian pair potential -V0 exp(-r^2 / (2 w^2)).
"""
from __future__ import annotations

import math

import numpy as np

L_DEFAULT = 15.0

CONFIGS = {
    "c1": dict(ndim=1, n=32, L=L_DEFAULT, alpha=20.0, v0=1.0, width=1.0,
               nev=3, block=4, seed_apply=1, seed_start=0),
    "c2": dict(ndim=1, n=256, L=L_DEFAULT, alpha=20.0, v0=2.0, width=1.0,
               nev=10, block=8, seed_apply=2, seed_start=2),
    "c3": dict(ndim=1, n=1024, L=L_DEFAULT, alpha=50.0, v0=4.0, width=1.0,
               nev=16, block=16, seed_apply=3, seed_start=3),
    "c5": dict(ndim=2, n=64, L=L_DEFAULT, alpha=20.0, v0=3.0, width=1.0,
               nev=6, block=8, seed_apply=5, seed_start=5),
    # the ground state of the reduced grid lies at E = -3.2e-3: its eigenvalue is
    # compared relative to |E|, so the residual tolerance (relative to
    # max(|theta|, 1)) is 1e-14, which the small operator norm of this grid allows
    "c5r": dict(ndim=2, n=20, L=L_DEFAULT, alpha=20.0, v0=3.0, width=1.0,
                nev=6, block=8, seed_apply=5, seed_start=5, tol=1e-14),
}

C4_SIZES = (64, 96, 128, 192, 256)
# Locking tolerance of the batched workload (relative to max(|theta|, 1)), the
# same as for the single workloads; instances whose residual floor lies above it
# are locked by the stagnation rule of the eigensolver.
C4_TOL = 1e-12


def config(name: str) -> dict:
    """Return a copy of the named workload's parameters."""
    return dict(CONFIGS[name])


def c4_instances(count: int = 256, seed: int = 2111) -> list[dict]:
    """Parameters of the batched workload, drawn in the order (n, M/m, V0, w)
    per instance from one PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(C4_SIZES[int(rng.integers(0, len(C4_SIZES)))])
        alpha = float(math.exp(rng.uniform(math.log(1.0), math.log(100.0))))
        v0 = float(rng.uniform(0.5, 5.0))
        w = float(rng.uniform(0.5, 2.0))
        out.append(dict(ndim=1, n=n, L=L_DEFAULT, alpha=alpha, v0=v0, width=w,
                        nev=4, block=4, seed_start=1000 + i, tol=C4_TOL))
    return out


def normal_block(N: int, b: int, seed: int, dtype=np.float64) -> np.ndarray:
    """A block of b standard-normal vectors of length N, shape (b, N).

    Row v is vector v; in memory this is the column-major N x b block with
    leading dimension N that the library takes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((b, N)).astype(dtype, copy=False)


def uniform_block(N: int, b: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(b, N))


def gaussian_bumps_1d(xs: np.ndarray, ys: np.ndarray, b: int, seed: int) -> np.ndarray:
    """Smooth test vectors: b random Gaussian bumps evaluated on a tensor grid,
    shape (b, len(xs) * len(ys)), x index slow.  Centres, widths and amplitudes
    are seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((b, xs.size * ys.size))
    for v in range(b):
        cx, cy = rng.uniform(-3, 3, size=2)
        sx, sy = rng.uniform(1.0, 3.0, size=2)
        amp = rng.uniform(0.5, 2.0)
        g = amp * np.exp(-((xs[:, None] - cx) / sx) ** 2 - ((ys[None, :] - cy) / sy) ** 2)
        out[v] = g.ravel()
    return out

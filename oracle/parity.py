"""The lowest eigenvalues of a 1D problem from its four parity sectors (the
parity selection rule of Sec. 5.1).

The potential V(x, y) = u(|y - x/2|) + u(|y + x/2|) is even in x (heavy
exchange) and even in y, and on a grid symmetric about 0 the second-derivative
matrices commute with the reflections, so H commutes with both reflections.
Its spectrum is therefore the union of the spectra of the four restrictions to
functions of parity (p_x, p_y) in {+1, -1}^2, each posed on the positive half
of both grids (n/2 unknowns per mode).  The k eigenvalues of smallest real part
of H are the k smallest of that union.

Each sector is solved with the oracle's block JDQR.  The union is trusted only
when every sector's largest computed eigenvalue lies at or above the k-th value
of the union (so no sector can hold a further eigenvalue below the cut);
otherwise that sector is solved again for more eigenvalues.
"""
from __future__ import annotations

import numpy as np

from . import jdqr, problem

SECTORS = ((+1, +1), (-1, +1), (+1, -1), (-1, -1))


def sector_problem(cfg, px, py):
    """The problem of workload parameters `cfg` (1D, even n per mode, CGL grid)
    restricted to x-parity px and y-parity py."""
    c = dict(cfg)
    n = c["n"]
    if c.get("ndim", 1) != 1 or np.ndim(n) or n % 2:
        raise ValueError("parity sectors need a 1D problem with an even n per mode")
    c["n"] = n // 2
    c["parity"] = (px, py)
    c["grid"] = "cgl"
    return problem.make_problem(**c)


def lowest_by_parity(cfg, nev, block, per_sector, sigma, target_low, seed=0, progress=None,
                     **kw):
    """The nev eigenvalues of smallest real part of the full problem `cfg`.

    per_sector: dict (px, py) -> number of eigenvalues first computed in that
    sector.  sigma: preconditioner shift and correction target (the full
    problem's two-body shift); target_low: the early target below the spectrum.
    Returns (evals ascending, list of (sector, evals, resnorm, n_outer))."""
    k = dict(per_sector)
    found = {}
    while True:
        for s in SECTORS:
            if s in found and len(found[s][0]) >= k[s]:
                continue
            P = sector_problem(cfg, *s)
            pc = P.preconditioner(sigma=sigma)
            r = jdqr.jdqr(P.apply, P.N, k[s], block, precond=pc.apply, target=sigma,
                          target_low=target_low, seed=seed, progress=(
                              (lambda o, nl, rn, th, s=s: progress(s, o, nl, rn, th))
                              if progress else None), **kw)
            if not r.converged:
                raise RuntimeError(f"sector {s} did not converge")
            found[s] = (r.evals.real.copy(), r.resnorm.copy(), r.n_outer)
        union = np.sort(np.concatenate([found[s][0] for s in SECTORS]))
        cut = union[nev - 1]
        short = [s for s in SECTORS if found[s][0][-1] < cut]
        if not short:
            return union[:nev], [(s,) + found[s] for s in SECTORS]
        for s in short:
            k[s] += block

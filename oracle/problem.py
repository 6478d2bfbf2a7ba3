"""Assemble a discretised three-body problem from its physical parameters.

Grid (reading: n counts interior unknowns; n + 2 Gauss-Lobatto points including
the two Dirichlet end points), coefficients in units with heavy mass 1, the
Gaussian pair potential -V0 exp(-r^2/(2 w^2)), and the default preconditioner
shift (the two-body ground energy on the y grid with the heavy-light reduced
mass).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cheb, operator, physics, precond, twobody


@dataclass
class Problem:
    ndim: int
    n: tuple
    L: tuple
    cx: float
    cy: float
    mu_hl: float
    shape: str
    v0: float
    width: float
    D2: tuple
    grids: tuple
    V: np.ndarray

    @property
    def N(self):
        return int(np.prod(self.n))

    def apply(self, X):
        if self.ndim == 1:
            return operator.apply_1d(self.D2[0], self.D2[1], self.cx, self.cy, self.V, X)
        return operator.apply_2d(self.D2, self.cx, self.cy, self.V, X)

    def kron(self):
        if self.ndim == 1:
            return operator.kron_1d(self.D2[0], self.D2[1], self.cx, self.cy, self.V)
        return operator.kron_2d(self.D2, self.cx, self.cy, self.V)

    def two_body_shift(self):
        """Ground energy of -(1/(2 mu_hl)) d^2/dr^2 + u(|r|) on the y grid (the
        first y mode's grid and second-derivative matrix)."""
        k = 1 if self.ndim == 1 else 2
        A = (-(1.0 / (2.0 * self.mu_hl)) * self.D2[k]
             + np.diag(physics.PAIR[self.shape](np.abs(self.grids[k]), self.v0, self.width)))
        return float(np.min(np.linalg.eigvals(A).real))

    def spectrum_lower_bound(self):
        """min V plus the smallest eigenvalue of each kinetic mode operator
        -c D2_k: a lower bound of the spectrum of the continuous problem
        (Weyl), used as the eigensolver's starting target."""
        coef = (self.cx, self.cy) if self.ndim == 1 else (self.cx, self.cx, self.cy, self.cy)
        lam = sum(np.min(np.linalg.eigvals(-c * d).real) for c, d in zip(coef, self.D2))
        return float(np.min(self.V) + lam)

    def preconditioner(self, sigma=None):
        if sigma is None:
            sigma = self.two_body_shift()
        if self.ndim != 1:
            return precond.KineticKronecker2D(self.D2, self.cx, self.cy, sigma)
        return precond.KineticSylvester(self.D2[0], self.D2[1], self.cx, self.cy, sigma)


def make_problem(ndim, n, L, alpha=None, v0=1.0, width=1.0, shape="gauss",
                 units="unit_heavy", cx=None, cy=None, mu_hl=None, grid="cgl", parity=None,
                 **_ignored):
    """grid: "cgl" (n interior Gauss-Lobatto points of [-L, L], Dirichlet) or
    "mapped" (Chebyshev roots mapped to the real line with parameter L).
    parity: per mode 0 (full grid of n points), +1 or -1 (even / odd functions;
    n unknowns at the positive nodes of a 2n-point grid of the same kind)."""
    nn = (n,) * (2 * ndim) if np.isscalar(n) else tuple(n)
    LL = (L,) * (2 * ndim) if np.isscalar(L) else tuple(L)
    if cx is None:
        if units == "unit_heavy":
            cx, cy, mu_hl = physics.coeffs_unit_heavy(alpha)
        else:
            cx, cy, mu_hl = physics.coeffs_paper_units(alpha)
    if grid == "cgl":
        par = (0,) * len(nn) if parity is None else tuple(parity)
        D2, grids = [], []
        for k, l, p in zip(nn, LL, par):
            if p == 0:
                D2.append(cheb.second_derivative_dirichlet(k, l))
                grids.append(cheb.nodes(k, l))
            else:
                xh, Dh = cheb.parity_half(cheb.nodes(2 * k, l),
                                          cheb.second_derivative_dirichlet(2 * k, l), p)
                D2.append(Dh)
                grids.append(xh)
        D2, grids = tuple(D2), tuple(grids)
    elif grid == "mapped":
        par = (0,) * len(nn) if parity is None else tuple(parity)
        D2, grids = [], []
        for k, l, p in zip(nn, LL, par):
            if p == 0:
                D2.append(cheb.mapped_second_derivative(k, l))
                grids.append(cheb.mapped_nodes(k, l))
            else:
                xh, Dh = cheb.parity_half(cheb.mapped_nodes(2 * k, l),
                                          cheb.mapped_second_derivative(2 * k, l), p)
                D2.append(Dh)
                grids.append(xh)
        D2, grids = tuple(D2), tuple(grids)
    else:
        raise ValueError(f"unknown grid {grid!r}")
    if ndim == 1:
        V = physics.potential_1d(grids[0], grids[1], shape, v0, width)
    else:
        V = physics.potential_2d(*grids, shape, v0, width)
    return Problem(ndim, nn, LL, cx, cy, mu_hl if mu_hl is not None else 1.0,
                   shape, v0, width, D2, grids, V)

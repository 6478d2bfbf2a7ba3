"""Heavy-light two-body problem (Sec. 2, eq. (1); Sec. 5.1).

Two uses: the ground energy of the discretised two-body Hamiltonian is the
preconditioner's default shift (Sec. 4.2: the preconditioner targets the
two-body threshold, which lies close to the wanted three-body energies; reading:
sigma = the two-body ground energy eps_2, i.e. minus the binding energy), and the
depth v0 that produces a prescribed binding energy E0 (the paper's workflow,
Sec. 2: first E0 is chosen, then v0 follows from the generalized eigenproblem
of eq. (1); Table 1 lists v0 in 1D, Table 3 in 2D), which pins the
second-derivative matrices against the paper's printed depths.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import cheb, physics


def ground_energy(n, L, mu, shape, v0, width=1.0):
    """Smallest real eigenvalue of -(1/(2 mu)) D2 + diag(u(|r|)) on the n
    interior Gauss-Lobatto nodes of [-L, L]."""
    r = cheb.nodes(n, L)
    D2 = cheb.second_derivative_dirichlet(n, L)
    A = -(1.0 / (2.0 * mu)) * D2 + np.diag(physics.PAIR[shape](np.abs(r), v0, width))
    ev = np.linalg.eigvals(A)
    return float(np.min(ev.real))


def depth_for_binding(n, L, E0, f=lambda r: np.exp(-r * r)):
    """Depth v0 for which [-1/2 d^2/dr^2 - v0 f(r)] has the eigenvalue -E0.

    Rearranged as the generalized eigenproblem (-1/2 D2 + E0 I) psi = v0 F psi
    with F = diag(f(r)); the ground state corresponds to the smallest positive
    real v0."""
    r = cheb.nodes(n, L)
    D2 = cheb.second_derivative_dirichlet(n, L)
    A = -0.5 * D2 + E0 * np.eye(n)
    B = np.diag(f(r))
    ev = scipy.linalg.eigvals(A, B)
    ev = ev[np.isfinite(ev)]
    real = ev[np.abs(ev.imag) < 1e-9 * np.maximum(1.0, np.abs(ev.real))].real
    return float(np.min(real[real > 0]))


def depth_for_binding_grid(r, D2, E0, f=lambda r: np.exp(-r * r), mu=1.0):
    """depth_for_binding on a given grid (nodes r, second-derivative matrix D2),
    e.g. the even half of the mapped grid; mu: heavy-light reduced mass in the
    kinetic term -(1/(2 mu)) d^2/dr^2 (1 in the paper's units)."""
    A = -(0.5 / mu) * D2 + E0 * np.eye(D2.shape[0])
    B = np.diag(f(r))
    ev = scipy.linalg.eigvals(A, B)
    ev = ev[np.isfinite(ev)]
    real = ev[np.abs(ev.imag) < 1e-9 * np.maximum(1.0, np.abs(ev.real))].real
    return float(np.min(real[real > 0]))


def _smallest_positive_real(ev):
    ev = ev[np.isfinite(ev)]
    real = ev[np.abs(ev.imag) < 1e-9 * np.maximum(1.0, np.abs(ev.real))].real
    return float(np.min(real[real > 0]))


def depth_for_binding_2d(r, D2, E0, f=lambda r: np.exp(-r * r), mu=1.0):
    """Depth v0 for the two-body problem in two dimensions (eq. (1) with a 2D
    Laplacian; Sec. 5.2), on the Cartesian product of the 1D grid (nodes r,
    second-derivative matrix D2) with itself:
        (-(1/(2 mu)) (D2 x I + I x D2) + E0 I) psi = v0 diag(f(|xi|)) psi,
    |xi| = sqrt(r_i^2 + r_j^2); the smallest positive real eigenvalue."""
    n = r.size
    I = np.eye(n)
    A = -(0.5 / mu) * (np.kron(D2, I) + np.kron(I, D2)) + E0 * np.eye(n * n)
    rad = np.sqrt(r[:, None] ** 2 + r[None, :] ** 2).ravel()
    return _smallest_positive_real(scipy.linalg.eigvals(A, np.diag(f(rad))))


def radial_laplacian_even_2d(N, L):
    """The s-wave part of the 2D Laplacian, d^2/dr^2 + (1/r) d/dr, on the
    even half of the N-point mapped grid (N even).  A rotation-invariant
    function of the plane is an even function of r on the whole line, so it is
    represented by the full mapped grid (which never contains r = 0) folded
    with even parity; no condition at r = 0 is needed.  An independent route
    to the 2D two-body problem: the Cartesian form above couples two 1D grids,
    this one uses a single radial grid."""
    x = cheb.mapped_nodes(N, L)
    R = cheb.mapped_second_derivative(N, L) + np.diag(1.0 / x) @ cheb.mapped_first_derivative(N, L)
    return cheb.parity_half(x, R, +1)


def depth_for_binding_radial_2d(N, L, E0, f=lambda r: np.exp(-r * r), mu=1.0):
    """Depth v0 for the 2D two-body ground state (an s state) from the radial
    equation: (-(1/(2 mu)) (d^2/dr^2 + (1/r) d/dr) + E0) psi = v0 f(r) psi."""
    r, R = radial_laplacian_even_2d(N, L)
    A = -(0.5 / mu) * R + E0 * np.eye(r.size)
    return _smallest_positive_real(scipy.linalg.eigvals(A, np.diag(f(r))))

"""Heavy-light two-body problem (Sec. 2, eq. (1); Sec. 5.1).

Two uses: the ground energy of the discretised two-body Hamiltonian is the
preconditioner's default shift (Sec. 4.2: the preconditioner targets the
two-body threshold, which lies close to the wanted three-body energies; reading:
sigma = the two-body ground energy eps_2, i.e. minus the binding energy), and the
depth v0 that produces a prescribed binding energy E0 (the paper's workflow,
Sec. 2 and Table 1), which pins the second-derivative matrix against the paper's
printed v0.
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


def depth_for_binding_grid(r, D2, E0, f=lambda r: np.exp(-r * r)):
    """depth_for_binding on a given grid (nodes r, second-derivative matrix D2),
    e.g. the even half of the mapped grid."""
    A = -0.5 * D2 + E0 * np.eye(D2.shape[0])
    B = np.diag(f(r))
    ev = scipy.linalg.eigvals(A, B)
    ev = ev[np.isfinite(ev)]
    real = ev[np.abs(ev.imag) < 1e-9 * np.maximum(1.0, np.abs(ev.real))].real
    return float(np.min(real[real > 0]))

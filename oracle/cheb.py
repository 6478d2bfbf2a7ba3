"""Chebyshev-Gauss-Lobatto collocation on [-L, L] (Sec. 3.1, eq. (7)).

The paper discretises each Jacobi coordinate with Chebyshev points and dense
differentiation matrices.  This oracle uses n interior unknowns: the grid has
K + 1 = n + 2 Gauss-Lobatto points t_j = cos(pi j / K), j = 0..K, including the
two end points, which carry the homogeneous Dirichlet condition and are removed.
Physical nodes are x = -L t, so they ascend with the index.

Pins: polynomial exactness (a degree <= K polynomial vanishing at +-L is
differentiated exactly), the particle-in-a-box spectrum (k pi / 2L)^2, and
symmetry of the second derivative under Clenshaw-Curtis quadrature for
polynomial arguments.
"""
from __future__ import annotations

import numpy as np


def gauss_lobatto(K: int) -> np.ndarray:
    """t_j = cos(pi j / K), j = 0..K (from +1 down to -1)."""
    j = np.arange(K + 1)
    return np.cos(np.pi * j / K)


def first_derivative(t: np.ndarray) -> np.ndarray:
    """Derivative matrix of the polynomial interpolant on Gauss-Lobatto nodes.

    Off the diagonal, entry (i, j) is the derivative at t_i of the j-th Lagrange
    basis polynomial, (w_j / w_i) / (t_i - t_j), with the Gauss-Lobatto
    barycentric weights w_j = (-1)^j, halved at both ends.  The diagonal is the
    negative row sum, because the derivative of the constant 1 is zero.
    """
    K = t.size - 1
    w = (-1.0) ** np.arange(K + 1)
    w[0] *= 0.5
    w[K] *= 0.5
    dt = t[:, None] - t[None, :]
    np.fill_diagonal(dt, 1.0)
    D = (w[None, :] / w[:, None]) / dt
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def nodes(n: int, L: float) -> np.ndarray:
    """The n interior nodes x_i = -L t_i, i = 1..n (ascending)."""
    t = gauss_lobatto(n + 1)
    return -L * t[1:-1]


def second_derivative_dirichlet(n: int, L: float) -> np.ndarray:
    """n x n second-derivative collocation matrix on the interior nodes of
    [-L, L] for functions vanishing at both ends.

    d/dx = -(1/L) d/dt, so d^2/dx^2 = (1/L^2) d^2/dt^2; the Dirichlet condition
    removes the boundary rows (no equation there) and columns (the value there is
    zero)."""
    t = gauss_lobatto(n + 1)
    D = first_derivative(t)
    D2 = D @ D
    return D2[1:-1, 1:-1] / (L * L)


def clenshaw_curtis_weights(n: int, L: float) -> np.ndarray:
    """Quadrature weights on the n interior nodes of [-L, L], exact for
    polynomials of degree <= K = n + 1 that vanish at the ends.

    Obtained by solving the moment equations sum_j w_j T_m(t_j) = int T_m dt
    over all K + 1 Gauss-Lobatto nodes (int_{-1}^{1} T_m = 2 / (1 - m^2) for
    even m, 0 for odd m) and scaling by L for x = -L t."""
    K = n + 1
    t = gauss_lobatto(K)
    m = np.arange(K + 1)
    Tm = np.cos(np.outer(m, np.arccos(np.clip(t, -1.0, 1.0))))
    mom = np.where(m % 2 == 0, 2.0 / (1.0 - m.astype(float) ** 2 + (m == 1)), 0.0)
    w = np.linalg.solve(Tm, mom)
    return L * w[1:-1]


# ------------------------------------------------- mapped grid on the real line
# The paper's grid (Sec. 3.1): Chebyshev points on a finite interval carried to
# the whole real line by an algebraic map (Boyd's rational Chebyshev basis).
# Here the collocation points are the N roots of T_N, t_j = cos(pi (2j+1)/(2N)),
# and x = L t / sqrt(1 - t^2) (map parameter L).  A grid function is
# interpolated by a polynomial in t of degree N - 1; derivatives follow from
# the chain rule with t'(x) = (1 - t^2)^{3/2} / L and
# t''(x) = -3 t (1 - t^2)^2 / L^2:  d^2/dx^2 = t'^2 d^2/dt^2 + t'' d/dt.
# No boundary condition is imposed: the basis is defined on all of R.

def gauss_roots(N: int) -> np.ndarray:
    """Roots of T_N in ascending order."""
    j = np.arange(N)
    return np.cos(np.pi * (2 * j + 1) / (2 * N))[::-1]


def first_derivative_roots(t: np.ndarray) -> np.ndarray:
    """Derivative matrix of the polynomial interpolant on the roots of T_N:
    barycentric weights of the first-kind Chebyshev points are proportional to
    (-1)^j sin((2j+1) pi / (2N)) (in the descending order of the roots); the
    diagonal is the negative row sum."""
    N = t.size
    # weights in the order of t (ascending = reversed descending index)
    j = np.arange(N)[::-1]
    w = (-1.0) ** j * np.sin((2 * j + 1) * np.pi / (2 * N))
    dt = t[:, None] - t[None, :]
    np.fill_diagonal(dt, 1.0)
    D = (w[None, :] / w[:, None]) / dt
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def mapped_nodes(N: int, L: float) -> np.ndarray:
    t = gauss_roots(N)
    return L * t / np.sqrt(1.0 - t * t)


def mapped_first_derivative(N: int, L: float) -> np.ndarray:
    """N x N first-derivative collocation matrix on the mapped grid:
    d/dx = t'(x) d/dt."""
    t = gauss_roots(N)
    return ((1.0 - t * t) ** 1.5 / L)[:, None] * first_derivative_roots(t)


def mapped_second_derivative(N: int, L: float) -> np.ndarray:
    """N x N second-derivative collocation matrix on the mapped grid."""
    t = gauss_roots(N)
    Dt = first_derivative_roots(t)
    s = 1.0 - t * t
    tp = s ** 1.5 / L
    tpp = -3.0 * t * s * s / (L * L)
    return (tp ** 2)[:, None] * (Dt @ Dt) + tpp[:, None] * Dt


def parity_half(x: np.ndarray, D2: np.ndarray, sign: int):
    """Restriction to functions of definite parity (sign +1 even, -1 odd) on a
    grid symmetric about 0 with an even number of points: the unknowns are the
    values at the positive nodes, and a value at -x equals sign times the value
    at x, so column j of the half-grid operator is D2[:, j] + sign D2[:, mirror(j)]
    restricted to the positive rows (the parity selection rule of Sec. 5.1)."""
    N = x.size
    if N % 2:
        raise ValueError("parity restriction needs an even number of points")
    p = np.arange(N // 2, N)
    m = N - 1 - p
    return x[p], D2[np.ix_(p, p)] + sign * D2[np.ix_(p, m)]

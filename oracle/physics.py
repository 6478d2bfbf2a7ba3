"""Jacobi-coordinate kinetic coefficients and the pair potential (Sec. 2).

The three-body Hamiltonian (eq. (2)) is H = -c_x Lap_x - c_y Lap_y + V with x the
heavy-heavy separation and y the light particle relative to the heavy pair's
centre of mass.  Reading taken where the text is inconsistent: eq. (3) writes
the light-heavy distances as |x +- y/2|, but with the paper's coefficients
(alpha_x = 2/(1+alpha) belongs to the heavy-heavy coordinate) the light-heavy
distances are |y -+ x/2|; this oracle uses V = u(|y - x/2|) + u(|y + x/2|).
The separable harmonic pin (closed-form spectrum) fixes this reading.
"""
from __future__ import annotations

import numpy as np


def coeffs_unit_heavy(alpha: float):
    """(c_x, c_y, mu_hl) for heavy mass M = 1, light mass m = 1/alpha, hbar = 1.

    c_x = 1/(2 mu_x) with mu_x = M/2; c_y = 1/(2 mu_y) with
    mu_y = 2 M m / (2 M + m); mu_hl = M m / (M + m) is the heavy-light reduced
    mass of the two-body problem."""
    M = 1.0
    m = 1.0 / alpha
    mu_x = M / 2.0
    mu_y = 2.0 * M * m / (2.0 * M + m)
    mu_hl = M * m / (M + m)
    return 1.0 / (2.0 * mu_x), 1.0 / (2.0 * mu_y), mu_hl


def coeffs_paper_units(alpha: float):
    """(c_x, c_y, mu_hl) in the paper's dimensionless units, eq. (2):
    c_x = alpha_x / 2 with alpha_x = 2 / (1 + alpha), c_y = alpha_y / 2 with
    alpha_y = (1 + 2 alpha) / (2 + 2 alpha); the two-body equation (1) has
    kinetic term -1/2 Lap, i.e. mu_hl = 1."""
    ax = 2.0 / (1.0 + alpha)
    ay = (1.0 + 2.0 * alpha) / (2.0 + 2.0 * alpha)
    return ax / 2.0, ay / 2.0, 1.0


# Pair potentials u(r) between the light particle and one heavy particle.
def pair_gauss(r, v0, width):
    """-v0 exp(-r^2 / (2 w^2)) (Gaussian of width w)."""
    return -v0 * np.exp(-(r * r) / (2.0 * width * width))


def pair_gauss_paper(r, v0, width=None):
    """-v0 f_G(r) with f_G = exp(-r^2) (eq. (4))."""
    return -v0 * np.exp(-(r * r))


def pair_lorentz3(r, v0, width=None):
    """-v0 f_L(r) with f_L = 1 / (1 + r^2)^3 (eq. (5))."""
    return -v0 / (1.0 + r * r) ** 3


def pair_harmonic(r, v0, width=None):
    """+v0 r^2 / 2 (confining; used only for its closed-form spectrum)."""
    return 0.5 * v0 * r * r


PAIR = {
    "gauss": pair_gauss,
    "gauss_paper": pair_gauss_paper,
    "lorentz3": pair_lorentz3,
    "harmonic": pair_harmonic,
}


def potential_1d(x, y, shape, v0, width=1.0):
    """V[i, j] = u(|y_j - x_i/2|) + u(|y_j + x_i/2|), shape (n_x, n_y)."""
    u = PAIR[shape]
    X = x[:, None]
    Y = y[None, :]
    return u(np.abs(Y - X / 2.0), v0, width) + u(np.abs(Y + X / 2.0), v0, width)


def potential_2d(x1, x2, y1, y2, shape, v0, width=1.0):
    """V[i1, i2, j1, j2] = u(|y - x/2|) + u(|y + x/2|) for 2-vectors x = (x1, x2),
    y = (y1, y2); shape (n_x1, n_x2, n_y1, n_y2)."""
    u = PAIR[shape]
    X1 = x1[:, None, None, None]
    X2 = x2[None, :, None, None]
    Y1 = y1[None, None, :, None]
    Y2 = y2[None, None, None, :]
    rm = np.sqrt((Y1 - X1 / 2.0) ** 2 + (Y2 - X2 / 2.0) ** 2)
    rp = np.sqrt((Y1 + X1 / 2.0) ** 2 + (Y2 + X2 / 2.0) ** 2)
    return u(rm, v0, width) + u(rp, v0, width)

"""GPU checks of the paper's procedure over binding energies (Sec. 2; Sec. 5.1,
5.2) and of the Lorentzian-cube shape f_L (eq. (5)).

* tp3b_homotopy_solve fixes v0 for each E0 from the two-body problem, then
  solves the three-body problem, each solve started from the previous Schur
  vectors.  The depths must match Table 1; the three-body ratios E/E0 must
  match Table 1 (to the 5e-8 to which this grid, with its choice of map,
  reproduces the printed values) and the same solves started from a random block
  (1e-10): the start block changes the path of the iteration, not the
  converged eigenvalues.
* f_L: the Hamiltonian apply and the eigensolver against the oracle."""
import os

import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import dense, physics, problem
from workloads import normal_block

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_homotopy_table1_bosons():
    t3 = need_gpu()
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_paper.txt"))[:2]
    E0s = rows[:, 0]
    cx, cy, mu = physics.coeffs_paper_units(20.0)
    grid = dict(ndim=1, n=[256, 128], L=[40.0, 20.0], c_x=cx, c_y=cy, pot="gauss_paper",
                mu_hl=mu, grid="mapped", parity=[1, 1])
    two_body = dict(ndim=1, n=[8, 256], L=[12.0, 12.0], pot="gauss_paper", grid="mapped",
                    parity=[0, 1])
    say("homotopy E0", E0s)
    h = t3.homotopy(E0s, 3, 4, two_body=two_body, seed=1, max_outer=600, **grid)
    say("  v0", h["v0"], "outer", h["n_outer"])
    assert np.all(np.abs(h["v0"] - rows[:, 1]) <= 6e-9)
    for i, E0 in enumerate(E0s):
        ratio = h["evals"][i] / E0
        op = t3.Operator(grid["ndim"], grid["n"], grid["L"], cx, cy, pot="gauss_paper",
                         v0=h["v0"][i], mu_hl=mu, sigma=-E0, grid="mapped", parity=[1, 1])
        cold = op.jdqr(3, 4, seed=1, max_outer=600, want_Q=False)
        op.close()
        say("  E0", E0, "ratios", ratio, "table", rows[i, 2:5], "cold outer", cold.stats["n_outer"],
            "warm outer", h["n_outer"][i])
        assert np.max(np.abs(h["evals"][i] - cold.evals) / np.maximum(np.abs(cold.evals), 1.0)) <= 1e-10
        assert np.max(np.abs(ratio - rows[i, 2:5])) <= 5e-8


def test_lorentz3_matches_oracle():
    """f_L on a CGL grid: the apply against the oracle (1e-12 normwise) and the
    eigensolver against the dense eigenvalues (1e-10)."""
    import torch
    t3 = need_gpu()
    cx, cy, mu = physics.coeffs_unit_heavy(20.0)
    n, L, v0 = (36, 28), (8.0, 6.0), 1.6
    P = problem.make_problem(ndim=1, n=n, L=L, alpha=20.0, v0=v0, shape="lorentz3")
    op = t3.Operator(1, list(n), list(L), cx, cy, pot="lorentz3", v0=v0, mu_hl=mu)
    assert np.max(np.abs(op.V() - P.V.ravel())) <= 1e-14
    Xn = normal_block(P.N, 3, 61)
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    op.apply_H(X, Y)
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy() - Yr) / np.linalg.norm(Yr)
    ref = dense.lowest_eigenvalues(P.kron(), 3).real
    r = op.jdqr(3, 4, seed=2)
    eerr = np.max(np.abs(r.evals - ref) / np.maximum(np.abs(ref), 1.0))
    say("lorentz3 apply", err, "evals", r.evals, ref, eerr)
    assert err <= 1e-12
    assert eerr <= 1e-10


def test_homotopy_2d_small_grid_matches_dense():
    """The procedure in 2D (M/m = 1, paper units, f_G) on a 6^4 Gauss-Lobatto
    grid: the depth of each E0 from the 2D two-body problem on the Cartesian
    product of the two light-particle modes (against the oracle's generalized
    eigenproblem on the same grid), and the lowest three-body eigenvalue of
    each step against the dense eigenvalues of the explicit Kronecker matrix
    at that depth."""
    t3 = need_gpu()
    from oracle import cheb, twobody
    n, L = 6, 6.0
    E0s = np.array([0.4, 0.2])
    cx, cy, mu = physics.coeffs_paper_units(1.0)
    grid = dict(ndim=2, n=[n] * 4, L=L, c_x=cx, c_y=cy, pot="gauss_paper", mu_hl=mu)
    h = t3.homotopy(E0s, 1, 2, seed=2, max_outer=800, **grid)
    x = cheb.nodes(n, L)
    D2 = cheb.second_derivative_dirichlet(n, L)
    for i, E0 in enumerate(E0s):
        v0 = twobody.depth_for_binding_2d(x, D2, E0, lambda r: np.exp(-r * r))
        P = problem.make_problem(ndim=2, n=n, L=L, alpha=1.0, v0=h["v0"][i], shape="gauss_paper",
                                 units="paper")
        ref = dense.lowest_eigenvalues(P.kron(), 1).real
        say("2d homotopy E0", E0, "v0", h["v0"][i], v0, "E", h["evals"][i], ref,
            "outer", h["n_outer"][i])
        assert abs(h["v0"][i] - v0) <= 1e-10 * v0
        assert abs(h["evals"][i][0] - ref[0]) <= 1e-10 * max(abs(ref[0]), 1.0)

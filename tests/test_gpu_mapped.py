"""GPU parity on the paper's grid: Chebyshev roots mapped to the real line with
parity half grids (Sec. 3.1, Sec. 5.1), against the oracle and against the
paper's Table 1."""
import os

import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import cheb, physics, problem, twobody
from workloads import normal_block

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pair(t3, n, L, alpha, v0, parity, shape="gauss_paper", units="paper"):
    P = problem.make_problem(ndim=1, n=n, L=L, alpha=alpha, v0=v0, shape=shape, units=units,
                             grid="mapped", parity=parity)
    op = t3.Operator(1, list(n), list(L), P.cx, P.cy, pot=shape, v0=v0, mu_hl=P.mu_hl,
                     grid="mapped", parity=parity)
    return op, P


@pytest.mark.parametrize("parity", [(0, 0), (1, 1), (-1, 1), (1, -1)])
def test_mapped_setup_and_apply_match_oracle(parity):
    import torch
    t3 = need_gpu()
    n = (40, 24) if parity == (0, 0) else (20, 12)
    op, P = _pair(t3, n, (6.0, 3.0), 20.0, 0.35, parity)
    for k in range(2):
        D = op.D2(k)
        assert np.max(np.abs(D - P.D2[k])) <= 1e-12 * np.max(np.abs(P.D2[k]))
    assert np.max(np.abs(op.V() - P.V.ravel())) <= 1e-14
    assert abs(op.sigma - P.two_body_shift()) <= 1e-10 * abs(op.sigma)
    Xn = normal_block(P.N, 3, 61)
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    op.apply_H(X, Y)
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy() - Yr) / np.linalg.norm(Yr)
    say("mapped", parity, "apply rel err", err)
    assert err <= 1e-12


def test_table1_lowest_states_on_gpu():
    """Table 1, E0 = 0.1, M/m = 20, f_G, paper units: the two lowest bosonic and
    fermionic ratios E/E0 from the GPU eigensolver on the mapped parity grids
    (128 x 64 points) -- to the printed 8 digits, and to 1e-10 of the oracle's
    dense eigenvalues on the same grid."""
    t3 = need_gpu()
    row = np.loadtxt(os.path.join(GOLDEN, "table1_paper.txt"))[0]
    E0 = row[0]
    xs, Ds = cheb.parity_half(cheb.mapped_nodes(256, 8.0), cheb.mapped_second_derivative(256, 8.0), +1)
    v0 = twobody.depth_for_binding_grid(xs, Ds, E0)
    for name, px, cols in (("bosons", +1, [2, 3]), ("fermions", -1, [5, 6])):
        op, P = _pair(t3, (64, 32), (8.0, 4.0), 20.0, v0, (px, +1))
        dense_ev = np.sort(np.linalg.eigvals(P.kron()).real)[:2]
        r = op.jdqr(2, 2, seed=7, max_outer=400)
        ratio = r.evals / E0
        say(name, "gpu", ratio, "table", row[cols], "dense", dense_ev / E0, r.stats["n_outer"])
        assert np.max(np.abs(r.evals - dense_ev) / np.maximum(np.abs(dense_ev), 1.0)) <= 1e-10
        assert np.max(np.abs(ratio - row[cols])) <= 1.5e-8


@pytest.mark.parametrize("E0_row,grid,cols_b,cols_f,bar", [
    (0, (128, 64, 12.0, 6.0), [2, 3, 4], [5, 6], 1.5e-8),
    (1, (256, 128, 40.0, 20.0), [2, 3, 4], [5, 6], 5e-8),
])
def test_table1_rows_on_larger_grids(E0_row, grid, cols_b, cols_f, bar):
    """Larger mapped parity grids (the oracle's dense solve does not reach them;
    the paper's printed values are the reference): E0 = 0.1 -- all three bosonic
    and the two lowest fermionic ratios to the printed 8 digits; E0 = 0.01 -- the
    same states to 5e-8 (the converged values differ from the printed digits by
    up to 4e-8)."""
    t3 = need_gpu()
    row = np.loadtxt(os.path.join(GOLDEN, "table1_paper.txt"))[E0_row]
    E0 = row[0]
    xs, Ds = cheb.parity_half(cheb.mapped_nodes(512, 12.0), cheb.mapped_second_derivative(512, 12.0), +1)
    v0 = twobody.depth_for_binding_grid(xs, Ds, E0)
    assert abs(v0 - row[1]) <= 6e-9
    cx, cy, mu = physics.coeffs_paper_units(20.0)
    nx, ny, Lx, Ly = grid
    for px, cols in ((+1, cols_b), (-1, cols_f)):
        op = t3.Operator(1, [nx, ny], [Lx, Ly], cx, cy, pot="gauss_paper", v0=v0, mu_hl=mu,
                         grid="mapped", parity=[px, 1])
        r = op.jdqr(3, 4, seed=1, max_outer=600, want_Q=False)
        ratio = (r.evals / E0)[:len(cols)]
        say("E0", E0, "parity", px, ratio, row[cols])
        assert np.max(np.abs(ratio - row[cols])) <= bar

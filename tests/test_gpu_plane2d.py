"""GPU parity of the 2D applies on LDS-resident planes (operators whose four
mode sizes are all at most 64): the Hamiltonian in two passes (x slabs, then
y planes with the potential) and the kinetic preconditioner in four passes.

Grids cover full 64 x 64 matrices, ragged ones (sizes that are not multiples
of the 16 x 16 MFMA blocks), equal full x modes (the FP64 x passes then take
items of four matrices with one shared factor) and unequal ones, group counts
that do not divide by the matrices a workgroup holds (odd n_y^2 for FP64, n_y^2
not a multiple of 4 for FP32),
every potential form (separable Gaussian factors, point-by-point table,
Lorentzian cube), shifted applies, strided blocks, and the fallback of larger
modes to the three single-mode passes.  Bars: FP64 1e-12 normwise against the
oracle's tensor apply (1e-10 for the preconditioner, which the GPU applies in
the eigenbases of the mode operators, against the oracle's Bartels-Stewart
solve), FP32 1e-5 / 2e-5."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import physics, problem
from workloads import normal_block

pytestmark = pytest.mark.gpu

GRIDS = [
    ((20, 20, 13, 13), (15.0, 15.0, 15.0, 15.0)),   # ragged blocks, odd Ny
    ((64, 64, 9, 9), (12.0, 12.0, 6.0, 6.0)),      # full x slabs, ragged y planes
    ((7, 7, 5, 5), (6.0, 6.0, 5.0, 5.0)),          # tiny
    ((16, 16, 64, 64), (6.0, 6.0, 9.0, 9.0)),      # full y planes, Ny a multiple of 4
    ((64, 64, 8, 8), (12.0, 12.0, 6.0, 6.0)),      # equal full x modes: FP64 four-matrix x items
    ((64, 64, 6, 6), (12.0, 11.0, 6.0, 6.0)),      # full x slabs, unequal x modes
    ((16, 16, 64, 64), (6.0, 6.0, 9.0, 8.5)),      # full y planes, unequal y modes
]


def _pair(t3, n, L, alpha=20.0, v0=3.0, width=1.0, shape="gauss", table=False):
    cx, cy, mu = physics.coeffs_unit_heavy(alpha)
    P = problem.make_problem(ndim=2, n=n, L=L, alpha=alpha, v0=v0, width=width, shape=shape)
    if table:
        op = t3.Operator(2, list(n), list(L), cx, cy, pot="table", V_table=P.V.ravel(),
                         sigma=P.two_body_shift(), mu_hl=mu)
    else:
        op = t3.Operator(2, list(n), list(L), cx, cy, pot=shape, v0=v0, width=width, mu_hl=mu)
    return op, P


@pytest.mark.parametrize("grid", range(len(GRIDS)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_2d_planes(grid, prec):
    import torch
    t3 = need_gpu()
    n, L = GRIDS[grid]
    op, P = _pair(t3, n, L)
    pk, dt, bar = (t3.FP64, torch.float64, 1e-12) if prec == "fp64" else (t3.FP32, torch.float32, 1e-5)
    for nvec in (3, 8):
        Xn = normal_block(P.N, nvec, 61 + grid)
        X = to_dev(Xn, dt)
        Y = torch.empty_like(X)
        say("2d planes apply", n, prec, nvec)
        op.apply_H(X, Y, prec=pk)
        torch.cuda.synchronize()
        Yr = P.apply(X.double().cpu().numpy().T).T
        err = np.linalg.norm(Y.double().cpu().numpy() - Yr) / np.linalg.norm(Yr)
        say("  normwise rel err", err)
        assert err <= bar


@pytest.mark.parametrize("n", [(20, 20, 13, 13), (8, 8, 64, 64)])
@pytest.mark.parametrize("shape,table", [("gauss", True), ("lorentz3", False), ("gauss_paper", False)])
def test_apply_2d_planes_potential_forms(shape, table, n):
    """The point-by-point table and the non-separable Lorentzian read V from the
    table in the epilogue; the Gaussians use their separable factors (ragged
    planes, and full planes with equal y modes: one plane per work item)."""
    import torch
    t3 = need_gpu()
    L = (8.0, 8.0, 6.0, 6.0)
    op, P = _pair(t3, n, L, v0=2.5, width=0.8, shape=shape, table=table)
    Xn = normal_block(P.N, 4, 71)
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    op.apply_H(X, Y)
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy() - Yr) / np.linalg.norm(Yr)
    say("2d planes potential", shape, "table" if table else "", err)
    assert err <= 1e-12


@pytest.mark.parametrize("n,pad", [((20, 20, 13, 13), 3), ((8, 8, 64, 64), 2)])
def test_apply_2d_planes_shifted_and_strided(n, pad):
    """(H - s_v) X on a block whose leading dimension is N + pad (N + 3:
    unaligned vectors; N + 2 on full equal-mode planes: aligned, the one-plane
    y pass), against the oracle's apply minus the shift."""
    import torch
    t3 = need_gpu()
    L = (15.0, 15.0, 15.0, 15.0)
    op, P = _pair(t3, n, L)
    nvec, ld = 3, P.N + pad
    Xn = normal_block(P.N, nvec, 72)
    Xb = torch.zeros((nvec, ld), dtype=torch.float64, device="cuda")
    Xb[:, :P.N] = to_dev(Xn)
    Yb = torch.full((nvec, ld), 7.0, dtype=torch.float64, device="cuda")
    s = np.array([0.3, -1.1, 2.5])
    op.apply_H(Xb[:, :P.N], Yb[:, :P.N], shifts=to_dev(s))
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T).T - s[:, None] * Xn
    Y = Yb.cpu().numpy()
    err = np.linalg.norm(Y[:, :P.N] - Yr) / np.linalg.norm(Yr)
    say("2d planes shifted strided", err)
    assert err <= 1e-12
    assert np.all(Y[:, P.N:] == 7.0)


@pytest.mark.parametrize("grid", range(len(GRIDS)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prec_2d_planes(grid, prec):
    import torch
    t3 = need_gpu()
    n, L = GRIDS[grid]
    op, P = _pair(t3, n, L)
    pc = P.preconditioner(sigma=op.sigma)
    pk, dt, bar = (t3.FP64, torch.float64, 1e-10) if prec == "fp64" else (t3.FP32, torch.float32, 2e-5)
    Xn = normal_block(P.N, 3, 81 + grid)
    X = to_dev(Xn, dt)
    Y = torch.empty_like(X)
    say("2d planes prec", n, prec)
    op.apply_prec(X, Y, prec=pk)
    torch.cuda.synchronize()
    Zr = pc.apply(X.double().cpu().numpy().T).T
    err = np.linalg.norm(Y.double().cpu().numpy() - Zr) / np.linalg.norm(Zr)
    say("  rel err", err)
    assert err <= bar


def test_apply_2d_large_modes_fallback():
    """Mode sizes above 64 run the three single-mode passes."""
    import torch
    t3 = need_gpu()
    n, L = (66, 66, 5, 5), (10.0, 10.0, 5.0, 5.0)
    op, P = _pair(t3, n, L)
    Xn = normal_block(P.N, 2, 91)
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    op.apply_H(X, Y)
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy() - Yr) / np.linalg.norm(Yr)
    say("2d fallback apply", err)
    assert err <= 1e-12
    pc = P.preconditioner(sigma=op.sigma)
    op.apply_prec(X, Y)
    torch.cuda.synchronize()
    Zr = pc.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy() - Zr) / np.linalg.norm(Zr)
    say("2d fallback prec", err)
    assert err <= 1e-10

"""GPU parity of the BF16x3 mode products against the oracle.

BF16x3 splits every FP32 operand f into bf16 hi = rn(f) and lo = rn(f - hi) and
forms a*b as hi_a hi_b + hi_a lo_b + lo_a hi_b with FP32 accumulation.  With 8
significant bits per bf16 value, |lo| <= 2^-8 |f| and the remainder
f - hi - lo is at most 2^-16 |f|, so each product is off by at most about
3 * 2^-16 |a b|.  Summed over a row, the componentwise error of Y = H W is then
bounded by (3 * 2^-16 + FP32 accumulation) * (|H||W|), which is the bar written
in each test: the dropped-term budget plus the same FP32 allowance as the FP32
tests.  A kernel that kept only hi*hi (error ~2^-8) fails it by two orders of
magnitude.  Inputs are rounded to FP32 first and the oracle evaluates on those
rounded values in FP64."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import physics, problem
from workloads import config, gaussian_bumps_1d, normal_block

pytestmark = pytest.mark.gpu

SPLIT = 3 * 2.0 ** -16


def fp32_budget(n):
    return 4 * (2 * n + 2) * 6e-8


def _absH_absW(P, Xn):
    """|H||W| per entry (componentwise error scale), 1D; Xn is (N, b)."""
    Kx, Ky = np.abs(P.cx * P.D2[0]), np.abs(P.cy * P.D2[1])
    out = np.empty_like(Xn)
    for v in range(Xn.shape[1]):
        W = np.abs(Xn[:, v]).reshape(P.n[0], P.n[1])
        out[:, v] = (Kx @ W + W @ Ky.T + np.abs(P.V) * W).ravel()
    return out


@pytest.mark.parametrize("name,nvec", [("c1", 4), ("c2", 8), ("c2", 3)])
def test_apply_bf16x3_random(name, nvec):
    import torch
    t3 = need_gpu()
    cfg = config(name)
    P = problem.make_problem(**cfg)
    op = t3.Operator.from_config(cfg)
    Xn = normal_block(P.N, nvec, cfg["seed_apply"] + 7).astype(np.float32).astype(np.float64)
    X = to_dev(Xn, torch.float32)
    Y = torch.empty_like(X)
    say("apply bf16x3", name, nvec)
    op.apply_H(X, Y, prec=t3.BF16X3)
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T)
    scale = _absH_absW(P, Xn.T)
    Yg = Y.cpu().numpy().astype(np.float64).T
    err = np.max(np.abs(Yg - Yr) / scale)
    nerr = np.linalg.norm(Yg - Yr) / np.linalg.norm(Yr)
    say("  componentwise", err, "normwise", nerr)
    assert err <= SPLIT + fp32_budget(max(P.n))
    # BF16x3 must be well beyond plain bf16 accuracy (2^-8 per product)
    assert err <= 2.0 ** -12


@pytest.mark.parametrize("nx,ny,nvec", [(37, 50, 3), (130, 70, 2), (64, 200, 2), (2, 2, 1)])
def test_apply_bf16x3_ragged_smooth(nx, ny, nvec):
    import torch
    t3 = need_gpu()
    cx, cy, mu = physics.coeffs_unit_heavy(7.0)
    P = problem.make_problem(ndim=1, n=(nx, ny), L=(9.0, 6.0), alpha=7.0, v0=1.5, width=0.8)
    op = t3.Operator(1, [nx, ny], [9.0, 6.0], cx, cy, v0=1.5, width=0.8, mu_hl=mu)
    Xn = gaussian_bumps_1d(P.grids[0], P.grids[1], nvec, seed=nx * 131 + ny + 1).T
    Xn = Xn.astype(np.float32).astype(np.float64)
    say("apply bf16x3 ragged", nx, ny, nvec)
    X = to_dev(np.ascontiguousarray(Xn.T), torch.float32)
    Y = torch.empty_like(X)
    op.apply_H(X, Y, prec=t3.BF16X3)
    torch.cuda.synchronize()
    Yr = P.apply(Xn)
    scale = _absH_absW(P, Xn)
    err = np.max(np.abs(Y.cpu().numpy().astype(np.float64).T - Yr) / np.maximum(scale, 1e-300))
    say("  componentwise", err)
    assert err <= SPLIT + fp32_budget(max(nx, ny))


def test_apply_bf16x3_shifted_and_strided():
    """Per-vector shifts and leading dimensions larger than N."""
    import torch
    t3 = need_gpu()
    cfg = config("c1")
    P = problem.make_problem(**cfg)
    op = t3.Operator.from_config(cfg)
    Xn = normal_block(P.N, 3, 12).astype(np.float32).astype(np.float64)
    sh = np.array([0.5, -1.25, 3.0])
    buf = torch.zeros((3, P.N + 13), dtype=torch.float32, device="cuda")
    buf[:, :P.N] = to_dev(Xn, torch.float32)
    out = torch.full((3, P.N + 7), 7.0, dtype=torch.float32, device="cuda")
    op.apply_H(buf[:, :P.N], out[:, :P.N], prec=t3.BF16X3, shifts=to_dev(sh))
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T) - Xn.T * sh[None, :]
    scale = _absH_absW(P, Xn.T) + np.abs(Xn.T * sh[None, :])
    o = out.cpu().numpy().astype(np.float64)
    err = np.max(np.abs(o[:, :P.N].T - Yr) / scale)
    say("bf16x3 shifted/strided", err)
    assert err <= SPLIT + fp32_budget(max(P.n))
    assert np.all(o[:, P.N:] == 7.0)


def test_prec_bf16x3():
    """Preconditioner: four BF16x3 mode products and the FP32 divide; the
    eigenvector matrices have condition numbers below 5 (n <= 1024), so the
    normwise error stays within a small multiple of the per-product 3 * 2^-16."""
    import torch
    t3 = need_gpu()
    cfg = config("c2")
    P = problem.make_problem(**cfg)
    op = t3.Operator.from_config(cfg)
    pc = P.preconditioner()
    Xn = normal_block(P.N, 4, 33).astype(np.float32)
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    op.apply_prec(X, Y, prec=t3.BF16X3)
    torch.cuda.synchronize()
    Zr = pc.apply(Xn.T.astype(np.float64)).T
    err = np.linalg.norm(Y.cpu().numpy() - Zr) / np.linalg.norm(Zr)
    say("prec bf16x3 rel err", err)
    assert err <= 1e-3


def test_apply_bf16x3_2d_small():
    import torch
    t3 = need_gpu()
    cx, cy, mu = physics.coeffs_unit_heavy(20.0)
    n = (9, 9, 7, 7)
    P = problem.make_problem(ndim=2, n=n, L=(6.0, 6.0, 5.0, 5.0), alpha=20.0, v0=3.0)
    op = t3.Operator(2, list(n), [6.0, 6.0, 5.0, 5.0], cx, cy, v0=3.0, mu_hl=mu)
    Xn = normal_block(P.N, 3, 41).astype(np.float32).astype(np.float64)
    X = to_dev(Xn, torch.float32)
    Y = torch.empty_like(X)
    op.apply_H(X, Y, prec=t3.BF16X3)
    torch.cuda.synchronize()
    Yr = P.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy().astype(np.float64) - Yr) / np.linalg.norm(Yr)
    say("2d small bf16x3 rel err", err)
    assert err <= 4 * SPLIT


def test_apply_bf16x3_c3_full_size_sampled():
    """n = 1024, 16 vectors, the tile shape the heuristic picks at full size;
    sampled outputs computed one by one from the operator's definition."""
    import torch
    t3 = need_gpu()
    cfg = config("c3")
    P = problem.make_problem(**cfg)
    op = t3.Operator.from_config(cfg)
    b = cfg["block"]
    X = to_dev(normal_block(P.N, b, cfg["seed_apply"]), torch.float32)
    Y = torch.empty_like(X)
    say("c3 bf16x3 full-size apply")
    op.apply_H(X, Y, prec=t3.BF16X3)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy().astype(np.float64)
    Xh = X.cpu().numpy().astype(np.float64)
    nx, ny = P.n
    Kx, Ky = P.cx * P.D2[0], P.cy * P.D2[1]
    rng = np.random.default_rng(1)
    for v in range(0, b, 5):
        W = Xh[v].reshape(nx, ny)
        idx = rng.integers(0, P.N, 300)
        i, j = np.divmod(idx, ny)
        ref = -np.einsum("sk,ks->s", Kx[i, :], W[:, j]) - np.einsum("sk,sk->s", W[i, :], Ky[j, :]) \
            + P.V[i, j] * W[i, j]
        scale = np.einsum("sk,ks->s", np.abs(Kx[i, :]), np.abs(W[:, j])) \
            + np.einsum("sk,sk->s", np.abs(W[i, :]), np.abs(Ky[j, :])) + np.abs(P.V[i, j] * W[i, j])
        err = np.max(np.abs(Yh[v, idx] - ref) / scale)
        say("  vec", v, "componentwise", err)
        assert err <= SPLIT + fp32_budget(max(nx, ny))


def test_jdqr_c2_bf16x3_inner():
    """JDQR with BF16x3 inner GMRES and FP64 outer iteration reaches the FP64
    oracle's eigenvalues within 1e-10."""
    import os
    t3 = need_gpu()
    cfg = config("c2")
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_evals.txt")
    ref = np.loadtxt(path)[:, 0]
    op = t3.Operator.from_config(cfg)
    say("jdqr c2 bf16x3")
    r = op.jdqr(cfg["nev"], cfg["block"], inner_prec=t3.BF16X3, seed=cfg["seed_start"])
    err = np.max(np.abs(r.evals - ref) / np.abs(ref))
    say("  err", err, r.stats)
    assert err <= 1e-10

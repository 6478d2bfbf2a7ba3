"""GPU parity of the 2D (four-mode) kinetic preconditioner and of the
preconditioned 2D eigensolver.

The oracle solves the shifted four-mode Kronecker sum by Bartels-Stewart
(Schur factors and back substitution); the library inverts it in the
eigenbases of the mode operators.  Both are exact, so they agree to the
conditioning of the eigenvector matrices (below 5 for these grids) times the
working precision: 1e-10 in FP64.  FP32 and BF16x3 bars follow from the
per-product error (2^-24 n, 3 * 2^-16) through eight mode products."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import dense, operator, physics, problem
from workloads import config, normal_block

pytestmark = pytest.mark.gpu


def _pair(t3, n, L, alpha, v0, width=1.0):
    cx, cy, mu = physics.coeffs_unit_heavy(alpha)
    op = t3.Operator(2, list(n), list(L) if not np.isscalar(L) else L, cx, cy, v0=v0, width=width,
                     mu_hl=mu)
    P = problem.make_problem(ndim=2, n=n, L=L, alpha=alpha, v0=v0, width=width)
    return op, P


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 2e-3)])
def test_prec_2d_small(prec, bar):
    import torch
    t3 = need_gpu()
    op, P = _pair(t3, (9, 9, 7, 7), (6.0, 6.0, 5.0, 5.0), 20.0, 3.0)
    assert abs(op.sigma - P.two_body_shift()) <= 1e-11 * abs(op.sigma)
    pc = P.preconditioner(sigma=op.sigma)
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xn = normal_block(P.N, 3, 51)
    X = to_dev(Xn, dt)
    Y = torch.empty_like(X)
    op.apply_prec(X, Y, prec=pk)
    torch.cuda.synchronize()
    Zr = pc.apply(X.double().cpu().numpy().T).T
    err = np.linalg.norm(Y.double().cpu().numpy() - Zr) / np.linalg.norm(Zr)
    say("prec 2d small", prec, err)
    assert err <= bar


def test_prec_2d_ragged_modes():
    """Distinct sizes per mode pair and distinct half-widths (tiles ragged in
    every pass)."""
    import torch
    t3 = need_gpu()
    op, P = _pair(t3, (11, 11, 13, 13), (7.0, 7.0, 4.0, 4.0), 5.0, 2.0, 0.8)
    pc = P.preconditioner(sigma=op.sigma)
    Xn = normal_block(P.N, 2, 52)
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    op.apply_prec(X, Y)
    torch.cuda.synchronize()
    Zr = pc.apply(Xn.T).T
    err = np.linalg.norm(Y.cpu().numpy() - Zr) / np.linalg.norm(Zr)
    say("prec 2d ragged", err)
    assert err <= 1e-10


def test_prec_2d_c5_full_size_one_vector():
    """n = 64 per mode (N = 16.8 M), one vector, against the oracle's
    Bartels-Stewart solve of the full vector."""
    import torch
    t3 = need_gpu()
    cfg = config("c5")
    op = t3.Operator.from_config(cfg)
    P = problem.make_problem(**cfg)
    Xn = normal_block(P.N, 1, cfg["seed_apply"])
    X = to_dev(Xn)
    Y = torch.empty_like(X)
    say("c5 prec apply")
    op.apply_prec(X, Y)
    torch.cuda.synchronize()
    pc = P.preconditioner(sigma=op.sigma)
    Zr = pc.apply(Xn[0])
    err = np.linalg.norm(Y.cpu().numpy()[0] - Zr) / np.linalg.norm(Zr)
    say("  rel err", err)
    assert err <= 1e-10


def _sampled_2d(P, W, idx):
    """(H w) and (|H||w|) at the flat indices idx, entry by entry from the
    operator's definition (eq. (8)): the four mode products and the potential."""
    n = P.n
    i1, r = np.divmod(idx, n[1] * n[2] * n[3])
    i2, r = np.divmod(r, n[2] * n[3])
    j1, j2 = np.divmod(r, n[3])
    K = [P.cx * P.D2[0], P.cx * P.D2[1], P.cy * P.D2[2], P.cy * P.D2[3]]
    pairs = [(K[0][i1, :], W[:, i2, j1, j2].T), (K[1][i2, :], W[i1, :, j1, j2]),
             (K[2][j1, :], W[i1, i2, :, j2]), (K[3][j2, :], W[i1, i2, j1, :])]
    vw = P.V[i1, i2, j1, j2] * W[i1, i2, j1, j2]
    ref = -sum(np.einsum("sk,sk->s", a, w) for a, w in pairs) + vw
    scale = sum(np.einsum("sk,sk->s", np.abs(a), np.abs(w)) for a, w in pairs) + np.abs(vw)
    return ref, scale


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_apply_2d_c5_full_size_sampled(prec):
    """c5 at full size (n = 64 per mode, N = 16.8 M) in the launch shape of its
    solves (8 vectors): 300 sampled outputs of the first and the last vector,
    each computed from the definition, within a componentwise bound of the
    form used for the 1D applies: 4 (4n + 1) units of the precision times
    |H||w| (BF16x3: plus 3 * 2^-16 for the dropped split terms).  In FP64 the
    error measured when written (1.35e-13 against 2.26e-13) is mostly the
    difference between the library's and the oracle's own constructions of
    D2 (the set-up test allows 1e-13 of max |D2|), not the apply's rounding."""
    import torch
    t3 = need_gpu()
    cfg = config("c5")
    P = problem.make_problem(**cfg)
    op = t3.Operator.from_config(cfg)
    b, n = cfg["block"], P.n[0]
    pk, dt, u = {"fp64": (t3.FP64, torch.float64, 2.2e-16), "fp32": (t3.FP32, torch.float32, 6e-8),
                 "bf16x3": (t3.BF16X3, torch.float32, 6e-8)}[prec]
    bar = 4 * (4 * n + 1) * u + (3 * 2.0 ** -16 if prec == "bf16x3" else 0.0)
    X = to_dev(normal_block(P.N, b, cfg["seed_apply"]), dt)
    Y = torch.empty_like(X)
    say("c5 full-size apply", prec)
    op.apply_H(X, Y, prec=pk)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    for v in (0, b - 1):
        W = X[v].cpu().double().numpy().reshape(P.n)
        Yv = Y[v].cpu().double().numpy()
        idx = rng.integers(0, P.N, 300)
        ref, scale = _sampled_2d(P, W, idx)
        err = np.max(np.abs(Yv[idx] - ref) / scale)
        say("  vec", v, "componentwise", err, "bar", bar)
        assert err <= bar


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c5_blocks_equal_vector_by_vector(prec):
    """c5 at full size: the shifted H apply and the preconditioner of a
    3-vector block equal, bit for bit, the same applies to each vector alone
    (the large FP64 vectors go through the plane passes one vector at a time,
    the FP32 block in one pass each; either way every vector's arithmetic is
    its own), and the preconditioner of vector 1 matches the oracle's
    four-mode Bartels-Stewart solve to 1e-10 (FP64; FP32 4e-5)."""
    import torch
    t3 = need_gpu()
    cfg = config("c5")
    op = t3.Operator.from_config(cfg)
    pk, dt = (t3.FP64, torch.float64) if prec == "fp64" else (t3.FP32, torch.float32)
    Xn = normal_block(op.N, 3, 7)
    X = to_dev(Xn, dt)
    del Xn
    s = to_dev(np.array([0.25, -1.5, 3.0]))
    Y = torch.empty_like(X)
    say("c5 block shifted apply", prec)
    op.apply_H(X, Y, prec=pk, shifts=s)
    Z = torch.empty_like(X)
    op.apply_prec(X, Z, prec=pk)
    for v in range(3):
        y1 = torch.empty_like(X[v:v + 1])
        op.apply_H(X[v:v + 1], y1, prec=pk, shifts=s[v:v + 1])
        z1 = torch.empty_like(X[v:v + 1])
        op.apply_prec(X[v:v + 1], z1, prec=pk)
        torch.cuda.synchronize()
        assert torch.equal(y1[0], Y[v]), v
        assert torch.equal(z1[0], Z[v]), v
    P = problem.make_problem(**cfg)
    pc = P.preconditioner(sigma=op.sigma)
    zr = pc.apply(X[1].double().cpu().numpy())
    err = np.linalg.norm(Z[1].double().cpu().numpy() - zr) / np.linalg.norm(zr)
    say("  prec vector 1 vs oracle", err)
    assert err <= (1e-10 if prec == "fp64" else 4e-5)
    op.close()


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_jdqr_2d_preconditioned_vs_dense(inner):
    t3 = need_gpu()
    op, P = _pair(t3, (7, 7, 6, 6), 6.0, 20.0, 3.0)
    ref = dense.lowest_eigenvalues(P.kron(), 3).real
    pk = t3.FP64 if inner == "fp64" else t3.FP32
    r = op.jdqr(3, 4, precond=True, inner_prec=pk, seed=4, max_outer=400)
    r0 = op.jdqr(3, 4, precond=False, seed=4, max_outer=2000)
    err = np.max(np.abs(r.evals - ref) / np.abs(ref))
    say("2d jdqr prec", inner, r.evals, err, "outer", r.stats["n_outer"], "without prec",
        r0.stats["n_outer"])
    assert err <= 1e-10
    assert r.stats["n_outer"] < r0.stats["n_outer"]


def test_jdqr_2d_c5_full_size():
    """c5 at full size (2D, n = 64 per mode, N = 16.8 M; 6 eigenpairs, block 8)
    with the 2D preconditioner, FP64 and FP32 inner solves: the eigenvalues of
    the two agree to 1e-10 (|dE| / max(|E|, 1)); the Schur vectors are
    orthonormal to 1e-12; for the first and the last Schur vector the oracle's
    own apply gives ||H q_j - Q R[:, j]|| within the loosest locking bar
    1e-8 max(|R_jj|, 1) plus the FP64 floor of forming H q_j,
    4 (sum of the mode sizes + 1) eps || |H| |q_j| ||."""
    t3 = need_gpu()
    cfg = config("c5")
    P = problem.make_problem(**cfg)
    op = t3.Operator.from_config(cfg)
    say("jdqr c5 fp64")
    r64 = op.jdqr(cfg["nev"], cfg["block"], inner_prec=t3.FP64, seed=cfg["seed_start"])
    say("  outer", r64.stats["n_outer"])
    say("jdqr c5 fp32 inner")
    r32 = op.jdqr(cfg["nev"], cfg["block"], inner_prec=t3.FP32, seed=cfg["seed_start"],
                  want_Q=False)
    say("  outer", r32.stats["n_outer"])
    dE = np.max(np.abs(r64.evals - r32.evals) / np.maximum(np.abs(r64.evals), 1.0))
    Q = r64.Q.cpu().numpy()
    R = np.asarray(r64.R)
    orth = np.max(np.abs(Q @ Q.T - np.eye(Q.shape[0])))
    say("  fp64 vs fp32-inner", dE, "orthonormality", orth)
    assert dE <= 1e-10
    assert orth <= 1e-12
    nev = Q.shape[0]
    for j in (0, nev - 1):
        hq = P.apply(Q[j])
        res = np.linalg.norm(hq - Q.T @ R[:, j])
        absHq = operator.apply_2d([-np.abs(d) for d in P.D2], P.cx, P.cy, np.abs(P.V), np.abs(Q[j]))
        bar = 1e-8 * max(abs(R[j, j]), 1.0) + 4 * (sum(P.n) + 1) * 2.2e-16 * np.linalg.norm(absHq)
        say("  column", j, "residual", res, "bar", bar)
        assert res <= bar

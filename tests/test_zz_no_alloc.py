"""The allocation-free block orthogonalisation (tp3b_block_orth_noalloc,
scratch in the library's static device array) against tp3b_block_orth without
factors: the same kernels in the same order, so the outputs are identical
while no column is dependent; two calls in a row, the second smaller (the
array keeps the first call's contents); a rank-deficient block keeps the
span of its independent columns; a request above the array's size is
rejected before any launch."""
import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _case(rng, N, nq, nx):
    Q = np.linalg.qr(rng.standard_normal((N, nq)))[0] if nq else np.zeros((N, 0))
    X = rng.standard_normal((N, nx)) + (Q @ rng.standard_normal((nq, nx)) if nq else 0)
    return Q, X


def test_noalloc_matches_block_orth_twice():
    import torch
    t3 = need_gpu()
    rng = np.random.default_rng(77)
    for N, nq, nx in ((1_048_576, 48, 16), (70_000, 20, 8)):
        Q, X = _case(rng, N, nq, nx)
        Qd = to_dev(Q.T)
        Xa = to_dev(X.T)
        Xb = to_dev(X.T)
        say("noalloc orth", N, nq, nx)
        _, _, rk_a = t3.block_orth(Qd, Xa, want_factors=False)
        rk_b = t3.block_orth_noalloc(Qd, Xb)
        torch.cuda.synchronize()
        assert rk_a == rk_b == nx
        A, B = Xa.cpu().numpy(), Xb.cpu().numpy()
        say("  max |diff|", np.max(np.abs(A - B)))
        assert np.array_equal(A, B)
        assert np.max(np.abs(B @ B.T - np.eye(nx))) <= 1e-12
        assert np.max(np.abs(B @ Q)) <= 1e-12


def test_noalloc_rank_deficient_keeps_span():
    import torch
    t3 = need_gpu()
    rng = np.random.default_rng(78)
    N = 6000
    Q = np.linalg.qr(rng.standard_normal((N, 6)))[0]
    X = rng.standard_normal((N, 5))
    X[:, 1] = 3 * X[:, 0] - Q @ np.arange(6.0)
    Xd = to_dev(X.T)
    rk = t3.block_orth_noalloc(to_dev(Q.T), Xd)
    torch.cuda.synchronize()
    Xo = Xd.cpu().numpy().T
    assert rk == 4
    assert np.max(np.abs(Xo.T @ Xo - np.eye(5))) <= 1e-12
    assert np.max(np.abs(Q.T @ Xo)) <= 1e-12
    for j in (0, 2, 3, 4):
        r = X[:, j] - Q @ (Q.T @ X[:, j])
        r -= Xo @ (Xo.T @ r)
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(X[:, j])


def test_noalloc_rejects_oversize():
    t3 = need_gpu()
    import torch
    N, nq, nx = 1_048_576, 200, 32
    Q = torch.zeros((nq, N), dtype=torch.float64, device="cuda")
    X = torch.zeros((nx, N), dtype=torch.float64, device="cuda")
    with pytest.raises(t3.Tp3bError) as e:
        t3.block_orth_noalloc(Q, X)
    assert e.value.code == -2  # TP3B_ENOMEM

"""The discretised three-body Hamiltonian (Sec. 3).

``apply_1d`` / ``apply_2d`` follow the tensor form: for each vector w, with W the
vector viewed as a tensor (x index slowest, eq. (6)), H w is the sum of one dense
matrix product per tensor mode plus the pointwise potential (eqs. (9)-(11)).
``kron_1d`` / ``kron_2d`` build the same operator as an explicit matrix from
Kronecker products (eqs. (7), (8)); they are used only on tiny grids, as the
brute-force check of the tensor form.
"""
from __future__ import annotations

import numpy as np


def apply_1d(D2x, D2y, cx, cy, V, X):
    """Y = H X for a block X of shape (N, b), N = n_x n_y.

    Per vector: Y = -c_x D2x W - c_y W D2y^T + V o W with W of shape (n_x, n_y)
    (row i = x_i).  This is eq. (10) with a_1 = -c_x, a_2 = -c_y written for a
    row-major W (the paper's column-major n_y x n_x reshape is its transpose)."""
    nx, ny = D2x.shape[0], D2y.shape[0]
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    Y = np.empty_like(X)
    for v in range(X.shape[1]):
        W = np.ascontiguousarray(X[:, v]).reshape(nx, ny)
        Yv = -cx * (D2x @ W) - cy * (W @ D2y.T) + V * W
        Y[:, v] = Yv.ravel()
    return Y[:, 0] if squeeze else Y


def apply_2d(D2, cx, cy, V, X):
    """Y = H X for the four-mode tensor [x1][x2][y1][y2] (eq. (11)).

    D2 = (D2_x1, D2_x2, D2_y1, D2_y2); each mode's second-derivative matrix acts
    on its own index."""
    n = tuple(d.shape[0] for d in D2)
    X = np.asarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    Y = np.empty_like(X)
    for v in range(X.shape[1]):
        W = np.ascontiguousarray(X[:, v]).reshape(n)
        T = -cx * (np.einsum("ia,ajkl->ijkl", D2[0], W)
                   + np.einsum("ja,iakl->ijkl", D2[1], W))
        T += -cy * (np.einsum("ka,ijal->ijkl", D2[2], W)
                    + np.einsum("la,ijka->ijkl", D2[3], W))
        T += V * W
        Y[:, v] = T.ravel()
    return Y[:, 0] if squeeze else Y


def kron_1d(D2x, D2y, cx, cy, V):
    """Explicit H = -c_x (D2x (x) I) - c_y (I (x) D2y) + diag(vec V), eq. (7)."""
    nx, ny = D2x.shape[0], D2y.shape[0]
    return (-cx * np.kron(D2x, np.eye(ny)) - cy * np.kron(np.eye(nx), D2y)
            + np.diag(V.ravel()))


def kron_2d(D2, cx, cy, V):
    """Explicit 2D H, eq. (8): Kronecker sum over four modes plus diag(vec V)."""
    n = [d.shape[0] for d in D2]
    I = [np.eye(k) for k in n]

    def embed(k, A):
        mats = [I[0], I[1], I[2], I[3]]
        mats[k] = A
        out = mats[0]
        for M in mats[1:]:
            out = np.kron(out, M)
        return out

    H = -cx * (embed(0, D2[0]) + embed(1, D2[1])) - cy * (embed(2, D2[2]) + embed(3, D2[3]))
    return H + np.diag(V.ravel())


def apply_1d_at(D2x, D2y, cx, cy, V, W, idx):
    """(H w) and (|H| |w|) at the flat indices idx of one vector W (n_x, n_y),
    entry by entry from eq. (10): row i of D2x against column j of W, row i of W
    against row j of D2y, and the potential term."""
    ny = D2y.shape[0]
    i, j = np.divmod(np.asarray(idx), ny)
    a = cx * np.einsum("sk,sk->s", D2x[i, :], W[:, j].T)
    b = cy * np.einsum("sk,sk->s", W[i, :], D2y[j, :])
    vw = V[i, j] * W[i, j]
    ref = -a - b + vw
    scale = (cx * np.einsum("sk,sk->s", np.abs(D2x[i, :]), np.abs(W[:, j].T))
             + cy * np.einsum("sk,sk->s", np.abs(W[i, :]), np.abs(D2y[j, :])) + np.abs(vw))
    return ref, scale


def apply_2d_at(D2, cx, cy, V, W, idx):
    """(H w) and (|H| |w|) at the flat indices idx of one vector W (n1, n2, n3,
    n4), entry by entry from eq. (8): each mode's row against the fibre of W
    through the entry along that mode, plus the potential term."""
    n = W.shape
    i1, r = np.divmod(np.asarray(idx), n[1] * n[2] * n[3])
    i2, r = np.divmod(r, n[2] * n[3])
    j1, j2 = np.divmod(r, n[3])
    coef = (cx, cx, cy, cy)
    rows = (D2[0][i1, :], D2[1][i2, :], D2[2][j1, :], D2[3][j2, :])
    fibres = (W[:, i2, j1, j2].T, W[i1, :, j1, j2], W[i1, i2, :, j2], W[i1, i2, j1, :])
    vw = V[i1, i2, j1, j2] * W[i1, i2, j1, j2]
    ref = vw - sum(c * np.einsum("sk,sk->s", a, f) for c, a, f in zip(coef, rows, fibres))
    scale = np.abs(vw) + sum(c * np.einsum("sk,sk->s", np.abs(a), np.abs(f))
                             for c, a, f in zip(coef, rows, fibres))
    return ref, scale

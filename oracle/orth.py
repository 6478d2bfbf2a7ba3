"""Block orthogonalisation (the basis-extension step of the eigensolver).

Reading (the paper delegates this step to its eigensolver library): classical
Gram-Schmidt against Q applied twice, followed by a Householder QR of the
projected block, with R normalised to a positive diagonal so that the result is
unique.  A column whose norm after projection falls below ``drop_tol`` (1e-7)
times its norm before projection is linearly dependent on the rest (1e-7 is
about the square root of the FP64 unit roundoff, the smallest ratio a
Gram-matrix based orthogonalisation can resolve); it is replaced by a
seeded random vector, which is orthogonalised in its place, and the returned
rank counts only the independent columns.
"""
from __future__ import annotations

import numpy as np


def _project(Q, X):
    C = np.zeros((Q.shape[1], X.shape[1]))
    if Q.shape[1] == 0:
        return X, C
    for _ in range(2):
        c = Q.T @ X
        X = X - Q @ c
        C += c
    return X, C


def block_orth(Q, X, seed=0, drop_tol=1e-7):
    """Orthonormalise X (N, nx) against the orthonormal Q (N, nq) and itself.

    Returns (Xo, C, R, rank) with Xo^T Xo = I, Q^T Xo = 0 and, when rank == nx,
    X = Q C + Xo R with R upper triangular, positive diagonal."""
    Q = np.asarray(Q, dtype=np.float64)
    X = np.array(X, dtype=np.float64, copy=True)
    N, nx = X.shape
    norm0 = np.linalg.norm(X, axis=0)
    Xp, C = _project(Q, X)
    rng = np.random.Generator(np.random.PCG64(seed))
    rank = nx
    deficient = np.zeros(nx, dtype=bool)
    for _attempt in range(4):
        Qx, R = np.linalg.qr(Xp)
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        Qx = Qx * s
        R = R * s[:, None]
        bad = (np.abs(np.diag(R)) < drop_tol * np.maximum(norm0, np.finfo(float).tiny)) & ~deficient
        if not bad.any():
            break
        for j in np.nonzero(bad)[0]:
            deficient[j] = True
            rank -= 1
            r = rng.standard_normal(N)
            base = np.hstack([Q, Qx[:, :j]])
            r, _ = _project(base, r[:, None])
            Xp[:, j] = r[:, 0] / np.linalg.norm(r)
            norm0[j] = 1.0
    R[:, deficient] = 0.0
    R[deficient, :] = 0.0
    return Qx, C, R, rank

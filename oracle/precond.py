"""Kinetic-only shifted preconditioner solved by Bartels-Stewart (Sec. 4.2).

The preconditioner drops the potential and solves (K - sigma I) z = b with
K = K_x (x) I + I (x) K_y the kinetic Kronecker sum, K_x = -c_x D2x,
K_y = -c_y D2y.  With Z the (n_x, n_y) view of z this is the Sylvester equation
(eq. (14))

    (K_x - s_x I) Z + Z (K_y - s_y I)^T = B,     s_x + s_y = sigma,

with the shift split in proportion to the kinetic coefficients,
s_x = c_x sigma / (c_x + c_y), s_y = c_y sigma / (c_x + c_y) (Sec. 4.2).
(Reading: the paper labels the two factors the other way round between eq. (9)
and eq. (14); here each factor acts on its own mode.)

Bartels-Stewart: real Schur forms A_x = U_x T_x U_x^T and A_y = U_y T_y U_y^T
of the two shifted factors are computed once; each solve is F = U_x^T B U_y,
a substitution with the triangular factors for G in T_x G + G T_y^T = F, and
Z = U_x G U_y^T.  The second-derivative matrices have real spectra, so both
Schur factors are triangular (no 2 x 2 blocks); a matrix with complex
eigenvalues is rejected.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def shift_split(cx, cy, sigma):
    return cx * sigma / (cx + cy), cy * sigma / (cx + cy)


class KineticSylvester:
    def __init__(self, D2x, D2y, cx, cy, sigma):
        nx, ny = D2x.shape[0], D2y.shape[0]
        sx, sy = shift_split(cx, cy, sigma)
        self.nx, self.ny = nx, ny
        self.Ax = -cx * D2x - sx * np.eye(nx)
        self.Ay = -cy * D2y - sy * np.eye(ny)
        self.Tx, self.Ux = scipy.linalg.schur(self.Ax, output="real")
        self.Ty, self.Uy = scipy.linalg.schur(self.Ay, output="real")
        for T in (self.Tx, self.Ty):
            if np.any(np.abs(np.diag(T, -1)) > 0.0):
                raise NotImplementedError("shifted factor has complex eigenvalues")

    def solve_matrix(self, B):
        """Z with A_x Z + Z A_y^T = B; B has shape (n_x, n_y) or (b, n_x, n_y)."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        single = B.ndim == 2
        if single:
            B = B[None]
        F = self.Ux.T @ B @ self.Uy
        # Work with G^T (columns of G as contiguous rows) for the sweep.
        Ft = np.ascontiguousarray(np.swapaxes(F, 1, 2))      # (b, n_y, n_x)
        Gt = np.zeros_like(Ft)
        Ty = self.Ty
        # T_y^T is lower triangular: column j of G T_y^T involves G[:, l] for
        # l >= j, so the columns are found from the last one backwards.
        for j in range(self.ny - 1, -1, -1):
            rhs = Ft[:, j, :] - (Ty[j, j + 1:] @ Gt[:, j + 1:, :])
            M = self.Tx + Ty[j, j] * np.eye(self.nx)
            Gt[:, j, :] = scipy.linalg.solve_triangular(M, rhs.T, lower=False,
                                                        check_finite=False).T
        G = np.swapaxes(Gt, 1, 2)
        Z = self.Ux @ G @ self.Uy.T
        return Z[0] if single else Z

    def apply(self, X):
        """P^{-1} X for a block X of shape (N, b) (or a single vector)."""
        X = np.asarray(X, dtype=np.float64)
        squeeze = X.ndim == 1
        if squeeze:
            X = X[:, None]
        B = np.ascontiguousarray(X.T).reshape(X.shape[1], self.nx, self.ny)
        Z = self.solve_matrix(B)
        out = Z.reshape(X.shape[1], -1).T.copy()
        return out[:, 0] if squeeze else out

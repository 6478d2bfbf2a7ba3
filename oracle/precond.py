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
        nb = B.shape[0]
        F = self.Ux.T @ B @ self.Uy
        # Columns of G are found from the last one backwards (T_y^T is lower
        # triangular, so column j of G T_y^T involves the columns l >= j).  The
        # columns are stored as contiguous slabs Gt[j] of shape (n_x, b) so that
        # the sum over l > j is one matrix-vector product.
        Ft = np.ascontiguousarray(np.transpose(F, (2, 1, 0)))   # (n_y, n_x, b)
        Gt = np.zeros_like(Ft)
        Ty = self.Ty
        M = np.array(self.Tx, order="F")
        diag = np.diag_indices(self.nx)
        for j in range(self.ny - 1, -1, -1):
            rest = self.ny - j - 1
            rhs = Ft[j] - (Ty[j, j + 1:] @ Gt[j + 1:].reshape(rest, self.nx * nb)).reshape(self.nx, nb)
            M[diag] = self.Tx[diag] + Ty[j, j]
            Gt[j] = scipy.linalg.solve_triangular(M, rhs, lower=False, check_finite=False)
        G = np.ascontiguousarray(np.transpose(Gt, (2, 1, 0)))   # (b, n_x, n_y)
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


class KineticKronecker2D:
    """Kinetic preconditioner for the 2D (four-mode) operator: Z with
    (K - sigma I) Z = B, K = sum over the modes x1, x2, y1, y2 of -c D2_k acting
    on its own index (the kinetic part of eq. (8)).

    The paper builds this preconditioner for 1D only (Sec. 4.2); here its
    Bartels-Stewart approach is carried to four modes.  With real Schur forms
    A_k = U_k T_k U_k^T (T_k upper triangular: the spectra are real), the
    transformed right-hand side F = B x_1 U_1^T x_2 U_2^T x_3 U_3^T x_4 U_4^T
    satisfies the triangular system (T_1 + T_2 + T_3 + T_4 - sigma) G = F (each
    T_k on its own mode), solved by back substitution over the x1 index, then
    over the x2 index, each remaining (y1, y2) problem being a triangular
    Sylvester equation (T_3 - s I) G + G T_4^T = R; finally Z = G x_k U_k.
    """

    def __init__(self, D2, cx, cy, sigma):
        self.n = tuple(d.shape[0] for d in D2)
        coef = (cx, cx, cy, cy)
        self.A = [-c * d for c, d in zip(coef, D2)]
        self.sigma = float(sigma)
        self.T, self.U = [], []
        for A in self.A:
            T, U = scipy.linalg.schur(A, output="real")
            if np.any(np.abs(np.diag(T, -1)) > 0.0):
                raise NotImplementedError("a mode factor has complex eigenvalues")
            self.T.append(T)
            self.U.append(U)

    @staticmethod
    def _modes(W, M):
        """W x_k M_k for k = 0..3 (M_k acting on index k)."""
        W = np.einsum("ia,ajkl->ijkl", M[0], W)
        W = np.einsum("ja,iakl->ijkl", M[1], W)
        W = np.einsum("ka,ijal->ijkl", M[2], W)
        return np.einsum("la,ijka->ijkl", M[3], W)

    def _solve_triangular(self, F):
        T1, T2, T3, T4 = self.T
        n1, n2 = self.n[0], self.n[1]
        G = np.zeros_like(F)
        for i1 in range(n1 - 1, -1, -1):
            R1 = F[i1] - np.tensordot(T1[i1, i1 + 1:], G[i1 + 1:], axes=(0, 0))
            H = np.zeros_like(R1)
            for i2 in range(n2 - 1, -1, -1):
                R2 = R1[i2] - np.tensordot(T2[i2, i2 + 1:], H[i2 + 1:], axes=(0, 0))
                s = self.sigma - T1[i1, i1] - T2[i2, i2]
                H[i2] = scipy.linalg.solve_sylvester(T3 - s * np.eye(T3.shape[0]), T4.T, R2)
            G[i1] = H
        return G

    def solve_tensor(self, B):
        F = self._modes(B, [U.T for U in self.U])
        G = self._solve_triangular(F)
        return self._modes(G, self.U)

    def apply(self, X):
        """P^{-1} X for a block X of shape (N, b) (or a single vector)."""
        X = np.asarray(X, dtype=np.float64)
        squeeze = X.ndim == 1
        if squeeze:
            X = X[:, None]
        out = np.empty_like(X)
        for v in range(X.shape[1]):
            out[:, v] = self.solve_tensor(np.ascontiguousarray(X[:, v]).reshape(self.n)).ravel()
        return out[:, 0] if squeeze else out

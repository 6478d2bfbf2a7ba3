"""Block Jacobi-Davidson QR for the eigenvalues of smallest real part
(Sec. 4.1, eqs. (12)-(13)), with preconditioned GMRES on the correction
equation (Sec. 4.1-4.2).

JDQR builds a partial Schur form A Q = Q R (eq. (12)) of the non-symmetric
operator.  One outer iteration, as taken here (readings for the points the paper
leaves to its eigensolver library are marked R):

1. Rayleigh-Ritz: M = V^T A V on the orthonormal search basis V (V is kept
   orthogonal to the locked vectors Q).
2. Ordered real Schur form M = S T S^T, ascending real part.  (R) Computed from
   the eigenvectors of M: sorted, complex pairs replaced by their real and
   imaginary parts, then orthonormalised by QR; the nested spans make S a Schur
   basis.
3. The leading b Schur vectors u_j = V s_j with values theta_j = T_jj have the
   partial-Schur residuals r_j = (I - Q Q^T)(A u_j - sum_{i<=j} u_i T_ij), which
   equal the part of A u_j outside span[Q, V].
4. (R) Locking: leading u_j, in order, with ||r_j|| <= tol max(|theta_j|, 1)
   are moved from V to Q and R is extended by [Q^T A u_j; T_{1..j, j}].  (The
   criterion is absolute below unit magnitude: the FP64 rounding floor of the
   residual of these stiff operators lies near 1e-13 in absolute terms, so a
   purely relative 1e-12 is unreachable for eigenvalues of size ~0.1.)  The
   floor grows with ||A|| (it reaches ~5e-10 on some 128 x 128 grids with small
   mass ratios), so a leading pair whose residual stagnates below stall_tol is
   locked as well (see the jdqr docstring).
5. (R) Restart: when the basis would grow beyond m_max it is compressed to its
   m_min leading Schur vectors (the paper's "truncated" compression of the
   search space).
6. Correction equation (eq. (13)) for every j of the block, with
   Q~ = [Q, u_1..u_b] (R: the whole current block is deflated):
   (I - Q~Q~^T)(A - theta_j I)(I - Q~Q~^T) t_j = -r_j.
   It is solved approximately by left-preconditioned GMRES with the skew
   projection of Jacobi-Davidson (R: preconditioner P applied as
   (I - Y H^{-1} Q~^T) P^{-1}, Y = P^{-1} Q~, H = Q~^T Y, which keeps every
   Krylov vector orthogonal to Q~), a fixed number of steps from t = 0.
   Without a preconditioner this is the plain orthogonal projection.
   (R) While a residual is still large (||r_j|| > switch_tol |theta_j|) the
   fixed target (the preconditioner's shift, near the wanted eigenvalues) is
   used in place of theta_j, as Jacobi-Davidson does far from convergence.
7. The corrections are orthonormalised against [Q, V] and appended; their
   products with A are appended to A V.

Defaults (R, the paper gives none): m_max = max(4b, 2(nev + b)) rounded up to a
multiple of b, m_min = m_max / 2, 10 GMRES steps, residual tolerance 1e-12.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .orth import block_orth


def default_sizes(nev, b):
    m_max = max(4 * b, 2 * (nev + b))
    m_max = ((m_max + b - 1) // b) * b
    return m_max // 2, m_max


def ordered_schur(M):
    """Real orthogonal S and quasi-triangular T = S^T M S with eigenvalues in
    ascending order of real part.  Also returns a boolean array marking the
    first position of each 2 x 2 block (a complex-conjugate pair)."""
    w, Y = np.linalg.eig(M)
    order = np.argsort(w.real, kind="stable")
    cols = []
    pair = []
    for idx in order:
        if w[idx].imag == 0.0:
            cols.append(Y[:, idx].real)
            pair.append(False)
        elif w[idx].imag > 0.0:
            cols.append(Y[:, idx].real)
            cols.append(Y[:, idx].imag)
            pair.extend([True, False])
    B = np.column_stack(cols)
    S, _ = np.linalg.qr(B)
    T = S.T @ M @ S
    return S, T, np.array(pair, dtype=bool)


def gmres_fixed(op, rhs, steps):
    """GMRES(steps) from a zero start for each column of rhs (N, b).

    ``op(Z)`` applies the (column-dependent) operator to all columns at once.
    Arnoldi uses classical Gram-Schmidt applied twice.  A column whose Arnoldi
    vector vanishes (exact solution reached) stops early."""
    N, b = rhs.shape
    beta = np.linalg.norm(rhs, axis=0)
    Vk = np.zeros((b, steps + 1, N))
    H = np.zeros((b, steps + 1, steps))
    active = beta > 0
    for j in np.nonzero(active)[0]:
        Vk[j, 0] = rhs[:, j] / beta[j]
    kdone = np.zeros(b, dtype=int)
    for k in range(steps):
        W = op(np.ascontiguousarray(Vk[:, k, :].T))
        for j in range(b):
            if not active[j]:
                continue
            w = np.ascontiguousarray(W[:, j])
            basis = Vk[j, : k + 1]             # (k+1, N)
            h = np.zeros(k + 1)
            for _ in range(2):
                c = basis @ w
                w = w - basis.T @ c
                h += c
            H[j, : k + 1, k] = h
            hn = np.linalg.norm(w)
            H[j, k + 1, k] = hn
            kdone[j] = k + 1
            if hn <= 1e-14 * max(beta[j], 1e-300):
                active[j] = False
            else:
                Vk[j, k + 1] = w / hn
        if not active.any():
            break
    T = np.zeros((N, b))
    for j in range(b):
        k = kdone[j]
        if k == 0 or beta[j] == 0:
            continue
        e1 = np.zeros(k + 1)
        e1[0] = beta[j]
        y, *_ = np.linalg.lstsq(H[j, : k + 1, :k], e1, rcond=None)
        T[:, j] = Vk[j, :k].T @ y
    return T


@dataclass
class JDQRResult:
    evals: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    resnorm: np.ndarray
    n_outer: int = 0
    n_apply: int = 0
    n_apply_inner: int = 0
    n_prec: int = 0
    converged: bool = False
    history: list = field(default_factory=list)


def jdqr(apply_A, N, nev, block, *, tol=1e-12, m_min=None, m_max=None,
         gmres_steps=10, precond=None, apply_inner=None, X0=None, seed=0,
         max_outer=1000, target=None, switch_tol=1e-2, stall_tol=1e-8, target_low=None,
         low_iters=3, progress=None):
    """Partial Schur form for the nev eigenvalues of smallest real part.

    apply_A(X) -> A X for X of shape (N, k), in FP64.  apply_inner, if given,
    is used inside GMRES instead of apply_A (the low-precision form).
    precond(X) -> P^{-1} X or None (no preconditioner).
    target: shift used in the correction equation instead of theta_j while
    ||r_j|| > switch_tol |theta_j| (None: always theta_j).
    target_low, low_iters: (R) in the first low_iters outer iterations, while
    no pair has locked, target_low is used instead of target: a shift below the
    whole spectrum steers the early corrections to the lowest states (as
    inverse iteration from below does), so that a ground state far below target
    enters the search space before other states lock (None: target throughout).
    stall_tol: (R) when nothing locks, the leading pair is locked anyway once
    its residual is <= stall_tol max(|theta|, 1) and has stayed within 10 % of
    its previous value in three consecutive outer iterations -- the residual has
    reached the FP64 rounding floor of the stored images A V, which grows with
    ||A|| (<= 0 disables).
    progress: optional callable(outer, n_locked, rn, theta) called once per
    outer iteration (reporting only)."""
    b = block
    dmin, dmax = default_sizes(nev, b)
    m_min = dmin if m_min is None else m_min
    m_max = dmax if m_max is None else m_max
    apply_inner = apply_A if apply_inner is None else apply_inner
    res = JDQRResult(evals=np.zeros(0), Q=np.zeros((N, 0)), R=np.zeros((0, 0)),
                     resnorm=np.zeros(0))
    Q = np.zeros((N, 0))
    Rl = np.zeros((0, 0))
    lock_res = []
    if X0 is None:
        rng = np.random.Generator(np.random.PCG64(seed))
        X0 = rng.standard_normal((b, N)).T
    V, _, _, _ = block_orth(Q, X0, seed=seed + 1)
    AV = apply_A(V)
    res.n_apply += V.shape[1]
    outer = 0
    prev_rn0, stall = np.inf, 0
    while Q.shape[1] < nev and outer < max_outer:
        M = V.T @ AV
        S, T, pair = ordered_schur(M)
        m = V.shape[1]
        nb = min(b, m)
        U = V @ S[:, :nb]
        AU = AV @ S[:, :nb]
        Rres = AU - V @ (M @ S[:, :nb])
        if Q.shape[1]:
            Rres -= Q @ (Q.T @ Rres)
        theta = np.diag(T)[:nb].copy()
        rn = np.linalg.norm(Rres, axis=0)
        # lock the converged prefix (2 x 2 blocks move as a unit)
        p = 0
        while p < nb and Q.shape[1] + p < nev:
            blk = 2 if pair[p] else 1
            if p + blk > nb or not np.all(rn[p:p + blk] <= tol * np.maximum(np.abs(theta[p:p + blk]), 1.0)):
                break
            p += blk
        if p == 0 and stall_tol > 0:
            # stagnation at the rounding floor (see stall_tol)
            if (rn[0] <= stall_tol * max(abs(theta[0]), 1.0)
                    and 0.9 * prev_rn0 <= rn[0] <= 1.1 * prev_rn0):
                stall += 1
            else:
                stall = 0
            prev_rn0 = rn[0]
            blk = 2 if pair[0] else 1
            if stall >= 3 and blk <= nb:
                p = blk
                res.history.append(("stall-lock", outer, float(rn[0])))
        if p > 0:
            prev_rn0, stall = np.inf, 0
            QtAU = Q.T @ AU[:, :p]
            k = Rl.shape[0]
            Rn = np.zeros((k + p, k + p))
            Rn[:k, :k] = Rl
            Rn[:k, k:] = QtAU
            Rn[k:, k:] = T[:p, :p]
            Rl = Rn
            Q = np.hstack([Q, U[:, :p]])
            lock_res.extend(rn[:p].tolist())
            V = V @ S[:, p:]
            AV = AV @ S[:, p:]
            res.history.append(("lock", outer, p))
            if Q.shape[1] >= nev or V.shape[1] == 0:
                break
            continue
        outer += 1
        if m + nb > m_max:
            keep = max(m_min, nb)
            V = V @ S[:, :keep]
            AV = AV @ S[:, :keep]
            res.history.append(("restart", outer, keep))
        Qt = np.hstack([Q, U])
        if precond is not None:
            Yh = precond(Qt)
            res.n_prec += Qt.shape[1]
        else:
            Yh = Qt
        Hinv = np.linalg.inv(Qt.T @ Yh)

        def proj(Z):
            return Z - Yh @ (Hinv @ (Qt.T @ Z))

        def pinv(Z):
            if precond is None:
                return Z
            res.n_prec += Z.shape[1]
            return precond(Z)

        shift = theta.copy()
        if target is not None:
            far = rn > switch_tol * np.abs(theta)
            # (R) in the first low_iters outer iterations, while nothing is
            # locked, a target below the spectrum
            low = target_low is not None and Q.shape[1] == 0 and outer <= low_iters
            shift[far] = target_low if low else target

        def op(Z):
            res.n_apply_inner += Z.shape[1]
            return proj(pinv(apply_inner(Z) - Z * shift[None, :]))

        rhs = proj(pinv(-Rres))
        Tc = gmres_fixed(op, rhs, gmres_steps)
        Vn, _, _, rank = block_orth(np.hstack([Q, V]), Tc, seed=seed + 7 * outer + 3)
        V = np.hstack([V, Vn])
        AV = np.hstack([AV, apply_A(Vn)])
        res.n_apply += Vn.shape[1]
        res.history.append(("iter", outer, float(rn[0]), float(theta[0])))
        if progress is not None:
            progress(outer, Q.shape[1], rn, theta)
    ev = np.linalg.eigvals(Rl) if Rl.size else np.zeros(0)
    order = np.argsort(ev.real, kind="stable")
    res.evals = ev[order]
    res.Q = Q
    res.R = Rl
    res.resnorm = np.array(lock_res)
    res.n_outer = outer
    res.converged = Q.shape[1] >= nev
    return res

"""Python binding of libtp3b, the MI355X tensor-product three-body eigensolver.

Argument marshalling only: every step of the computation runs in the native
library (HIP kernels for gfx950 and its host driver).  PyTorch provides device
memory and streams.  Blocks of vectors are torch tensors of shape (nvec, N),
row v being vector v, i.e. the column-major N x nvec block the C ABI takes.

The library must have been built (``python -m paper_2111_02534_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtp3b.so")

TP3B_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV", -5: "ENOTSUP",
          -6: "ENONFINITE"}
FP64, FP32, BF16X3 = 0, 1, 2
POT = {"gauss": 0, "gauss_paper": 1, "lorentz3": 2, "harmonic": 3, "table": 4}
GRID = {"cgl": 0, "mapped": 1}


class Tp3bError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tp3b {STATUS.get(code, code)}: {msg}")
        self.code = code


class ProblemDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 4), ("L", ctypes.c_double * 4),
                ("c_x", ctypes.c_double), ("c_y", ctypes.c_double), ("pot", ctypes.c_int32),
                ("v0", ctypes.c_double), ("width", ctypes.c_double),
                ("V_table", ctypes.POINTER(ctypes.c_double)),
                ("D2", ctypes.POINTER(ctypes.c_double) * 4), ("sigma", ctypes.c_double),
                ("mu_hl", ctypes.c_double), ("grid", ctypes.c_int32),
                ("parity", ctypes.c_int32 * 4)]


class JdqrOpts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("block", ctypes.c_int32), ("m_min", ctypes.c_int32),
                ("m_max", ctypes.c_int32), ("gmres_steps", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("tol", ctypes.c_double),
                ("switch_tol", ctypes.c_double), ("target", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("check_finite", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("stall_tol", ctypes.c_double),
                ("low_start", ctypes.c_int32), ("test_dup_column", ctypes.c_int32)]


class JdqrStats(ctypes.Structure):
    _fields_ = [("n_conv", ctypes.c_int32), ("n_outer", ctypes.c_int32),
                ("n_restart", ctypes.c_int32), ("n_lock_events", ctypes.c_int32),
                ("n_apply_H_fp64", ctypes.c_int64), ("n_apply_H_low", ctypes.c_int64),
                ("n_apply_prec", ctypes.c_int64), ("t_apply", ctypes.c_double),
                ("t_prec", ctypes.c_double), ("t_orth", ctypes.c_double), ("t_rr", ctypes.c_double),
                ("t_gmres", ctypes.c_double), ("t_total", ctypes.c_double),
                ("t_kernel", ctypes.c_double * 4), ("n_kernel", ctypes.c_int64 * 4),
                ("v_kernel", ctypes.c_int64 * 4), ("n_stall_lock", ctypes.c_int32),
                ("n_dep_replaced", ctypes.c_int32)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name in ("t_kernel", "n_kernel", "v_kernel") else v
        return out


EXPORTS = ["tp3b_create", "tp3b_destroy", "tp3b_op_info", "tp3b_get_D2", "tp3b_get_V",
           "tp3b_apply_H", "tp3b_apply_H_shifted", "tp3b_apply_prec", "tp3b_block_orth",
           "tp3b_jdqr_default_opts", "tp3b_jdqr_solve", "tp3b_host_schur", "tp3b_last_error",
           "tp3b_set_tile", "tp3b_autotune", "tp3b_apply_H_batched", "tp3b_apply_prec_batched",
           "tp3b_autotune_batched", "tp3b_jdqr_solve_batched", "tp3b_two_body_depth",
           "tp3b_homotopy_solve", "tp3b_block_orth_noalloc"]

_lib = None


def lib():
    """The loaded native library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libtp3b.so not built at {LIB_PATH}; run __graft_entry__.build()")
        # torch first: it brings its own HIP runtime, and the library must bind
        # to that one (loaded the other way round, torch finds no device).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        L.tp3b_create.argtypes = [ctypes.POINTER(ProblemDesc), vp, ctypes.POINTER(vp)]
        L.tp3b_destroy.argtypes = [vp]
        L.tp3b_op_info.argtypes = [vp, ctypes.POINTER(i64), dp, dp]
        L.tp3b_get_D2.argtypes = [vp, i32, dp]
        L.tp3b_get_V.argtypes = [vp, dp]
        L.tp3b_apply_H.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
        L.tp3b_apply_H_shifted.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp, vp]
        L.tp3b_apply_prec.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
        L.tp3b_block_orth.argtypes = [i64, i32, vp, i64, i32, vp, i64, vp, vp,
                                      ctypes.POINTER(i32), ctypes.c_uint64, vp]
        L.tp3b_block_orth_noalloc.argtypes = [i64, i32, vp, i64, i32, vp, i64,
                                              ctypes.POINTER(i32), ctypes.c_uint64, vp]
        L.tp3b_jdqr_default_opts.argtypes = [ctypes.POINTER(JdqrOpts)]
        L.tp3b_jdqr_solve.argtypes = [vp, ctypes.POINTER(JdqrOpts), vp, i32, dp, vp, dp, dp,
                                      ctypes.POINTER(JdqrStats)]
        L.tp3b_host_schur.argtypes = [i32, dp, dp, dp, dp]
        L.tp3b_set_tile.argtypes = [vp, i32]
        L.tp3b_autotune.argtypes = [vp, i32, i32, i32, dp]
        pp = ctypes.POINTER(vp)
        i64p = ctypes.POINTER(i64)
        L.tp3b_apply_H_batched.argtypes = [pp, i32, i32, i32, pp, i64p, pp, i64p, pp, vp]
        L.tp3b_apply_prec_batched.argtypes = [pp, i32, i32, i32, pp, i64p, pp, i64p, vp]
        L.tp3b_autotune_batched.argtypes = [pp, i32, i32, i32, i32]
        L.tp3b_jdqr_solve_batched.argtypes = [pp, i32, ctypes.POINTER(JdqrOpts), dp, dp,
                                              ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32), pp,
                                              ctypes.POINTER(JdqrStats)]
        L.tp3b_two_body_depth.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_double, dp]
        L.tp3b_homotopy_solve.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(ProblemDesc),
                                          ctypes.POINTER(JdqrOpts), i32, dp, dp, dp, dp,
                                          ctypes.POINTER(ctypes.c_int32)]
        L.tp3b_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "tp3b_last_error":
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(code):
    if code != TP3B_OK:
        raise Tp3bError(code, lib().tp3b_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dbl_ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def jacobi_coefficients(alpha):
    """(c_x, c_y, mu_hl) for heavy mass 1 and light mass 1/alpha (hbar = 1):
    c_x = 1/(2 mu_x), mu_x = 1/2; c_y = 1/(2 mu_y), mu_y = 2m/(2 + m);
    mu_hl = m/(1 + m)."""
    m = 1.0 / alpha
    return 1.0, (2.0 + m) / (4.0 * m), m / (1.0 + m)


def paper_coefficients(alpha):
    """(c_x, c_y, mu_hl) in the paper's units (eq. (2)): alpha_x/2, alpha_y/2, 1."""
    return 1.0 / (1.0 + alpha), (1.0 + 2.0 * alpha) / (4.0 * (1.0 + alpha)), 1.0


def make_desc(ndim, n, L, c_x=1.0, c_y=1.0, pot="gauss", v0=1.0, width=1.0, sigma=None,
              mu_hl=1.0, V_table=None, D2=None, grid="cgl", parity=None):
    """A tp3b_problem_desc and the host arrays it points to (keep them alive
    while the descriptor is used)."""
    import numpy as np
    nm = 2 * ndim
    n = [n] * nm if isinstance(n, int) else list(n)
    L = [L] * nm if isinstance(L, (int, float)) else list(L)
    d = ProblemDesc()
    d.ndim = ndim
    for k in range(nm):
        d.n[k] = int(n[k])
        d.L[k] = float(L[k])
    d.c_x, d.c_y = float(c_x), float(c_y)
    d.pot = POT[pot] if isinstance(pot, str) else int(pot)
    d.v0, d.width = float(v0), float(width)
    d.sigma = float("nan") if sigma is None else float(sigma)
    d.mu_hl = float(mu_hl)
    d.grid = GRID[grid] if isinstance(grid, str) else int(grid)
    if parity is not None:
        for k, p in enumerate(parity):
            d.parity[k] = int(p)
    keep = []
    if V_table is not None:
        arr = np.ascontiguousarray(V_table, dtype=np.float64).ravel()
        keep.append(arr)
        d.V_table = _dbl_ptr(arr)
        d.pot = POT["table"]
    if D2 is not None:
        for k, m in enumerate(D2):
            if m is not None:
                arr = np.ascontiguousarray(m, dtype=np.float64)
                keep.append(arr)
                d.D2[k] = _dbl_ptr(arr)
    return d, keep


def two_body_depth(E0, ndim, n, L, pot="gauss", width=1.0, mu_hl=1.0, grid="cgl", parity=None,
                   D2=None):
    """Depth v0 giving the two-body binding energy E0 on the light-particle
    modes of the described grid (tp3b_two_body_depth; host computation)."""
    d, keep = make_desc(ndim, n, L, pot=pot, width=width, mu_hl=mu_hl, grid=grid, parity=parity,
                        D2=D2)
    v = ctypes.c_double()
    _check(lib().tp3b_two_body_depth(ctypes.byref(d), float(E0), ctypes.byref(v)))
    del keep
    return v.value


def homotopy(E0s, nev, block, ndim, n, L, c_x, c_y, pot="gauss", width=1.0, mu_hl=1.0,
             grid="cgl", parity=None, sigma=None, two_body=None, inner_prec=FP64, tol=1e-12,
             seed=0, max_outer=1000, gmres_steps=10, graph=True):
    """The paper's procedure over binding energies (tp3b_homotopy_solve):
    depth per E0, three-body solve, each solve started from the previous
    one.  two_body: optional dict of make_desc arguments for the two-body grid.
    Returns dict(v0, evals, resnorm, n_outer) with one row per E0."""
    import numpy as np
    d, keep = make_desc(ndim, n, L, c_x, c_y, pot=pot, width=width, sigma=sigma, mu_hl=mu_hl,
                        grid=grid, parity=parity)
    tb = None
    if two_body is not None:
        tb, keep2 = make_desc(**two_body)
        keep += keep2
    o = JdqrOpts()
    _check(lib().tp3b_jdqr_default_opts(ctypes.byref(o)))
    o.nev, o.block, o.gmres_steps, o.max_outer = nev, block, gmres_steps, max_outer
    o.inner_prec, o.tol, o.seed, o.graph = inner_prec, tol, seed, int(bool(graph))
    E = np.ascontiguousarray(E0s, dtype=np.float64)
    cnt = E.size
    v0 = np.full(cnt, np.nan)
    ev = np.full((cnt, nev), np.nan)
    rn = np.full((cnt, nev), np.nan)
    no = (ctypes.c_int32 * cnt)()
    code = lib().tp3b_homotopy_solve(ctypes.byref(d), ctypes.byref(tb) if tb is not None else None,
                                     ctypes.byref(o), cnt, _dbl_ptr(E), _dbl_ptr(v0), _dbl_ptr(ev),
                                     _dbl_ptr(rn), no)
    del keep
    out = {"v0": v0, "evals": ev, "resnorm": rn, "n_outer": np.array(list(no))}
    if code != TP3B_OK:
        err = Tp3bError(code, lib().tp3b_last_error().decode())
        err.result = out
        raise err
    return out


class Operator:
    """A discretised three-body Hamiltonian and its preconditioner on the
    current HIP device (a tp3b_op handle)."""

    def __init__(self, ndim, n, L, c_x, c_y, pot="gauss", v0=1.0, width=1.0, sigma=None,
                 mu_hl=1.0, V_table=None, D2=None, grid="cgl", parity=None):
        d, self._keep = make_desc(ndim, n, L, c_x, c_y, pot=pot, v0=v0, width=width, sigma=sigma,
                                  mu_hl=mu_hl, V_table=V_table, D2=D2, grid=grid, parity=parity)
        nm = 2 * ndim
        n = [n] * nm if isinstance(n, int) else list(n)
        L = [L] * nm if isinstance(L, (int, float)) else list(L)
        h = ctypes.c_void_p()
        _check(lib().tp3b_create(ctypes.byref(d), None, ctypes.byref(h)))
        self.handle = h
        self.ndim, self.n, self.L = ndim, n, L
        N = ctypes.c_int64()
        sig = ctypes.c_double()
        lm = ctypes.c_double()
        _check(lib().tp3b_op_info(h, ctypes.byref(N), ctypes.byref(sig), ctypes.byref(lm)))
        self.N, self.sigma = N.value, sig.value

    @classmethod
    def from_config(cls, cfg, units="unit_heavy", **kw):
        if units == "unit_heavy":
            cx, cy, mu = jacobi_coefficients(cfg["alpha"])
        else:
            cx, cy, mu = paper_coefficients(cfg["alpha"])
        return cls(cfg["ndim"], cfg["n"], cfg["L"], cx, cy, pot=kw.pop("pot", cfg.get("shape", "gauss")),
                   v0=cfg["v0"], width=cfg.get("width", 1.0), mu_hl=mu,
                   grid=cfg.get("grid", "cgl"), parity=cfg.get("parity"), **kw)

    def close(self):
        if getattr(self, "handle", None):
            lib().tp3b_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, tile):
        """Force a mode-product tile shape (0: 32x32, 1: 64x64, 2: 128x128,
        3: 64x128, 4: 32x32 over eight wavefronts; -1: automatic)."""
        _check(lib().tp3b_set_tile(self.handle, int(tile)))

    def autotune(self, prec=FP64, nvec=1, reps=5):
        """Time every tile shape for this operator's applies and keep the fastest.
        Returns the best (H apply, preconditioner) times in ms."""
        import numpy as np
        best = np.full(2, np.nan)
        _check(lib().tp3b_autotune(self.handle, prec, nvec, reps, _dbl_ptr(best)))
        return best

    def D2(self, mode):
        import numpy as np
        out = np.empty((self.n[mode], self.n[mode]))
        _check(lib().tp3b_get_D2(self.handle, mode, _dbl_ptr(out)))
        return out

    def V(self):
        import numpy as np
        out = np.empty(self.N)
        _check(lib().tp3b_get_V(self.handle, _dbl_ptr(out)))
        return out

    @staticmethod
    def _prec_of(t):
        import torch
        if t.dtype == torch.float64:
            return FP64
        if t.dtype == torch.float32:
            return FP32
        raise TypeError("blocks must be float64 or float32 tensors")

    def _blk(self, X, Y):
        if X.dim() != 2 or X.shape[1] != self.N or X.stride(1) != 1:
            raise ValueError("blocks are (nvec, N) tensors with unit stride along N")
        if Y.shape != X.shape or Y.stride(1) != 1 or Y.dtype != X.dtype:
            raise ValueError("Y must match X")
        if X.shape[0] == 1:  # a single vector: the row stride is irrelevant
            return 1, self.N, self.N
        return X.shape[0], X.stride(0), Y.stride(0)

    def _prec(self, X, prec):
        p = self._prec_of(X)
        if prec is None:
            return p
        if (prec == FP64) != (p == FP64):
            raise TypeError("FP64 applies take float64 blocks, FP32/BF16X3 applies float32 blocks")
        return int(prec)

    def apply_H(self, X, Y, prec=None, shifts=None, stream=None):
        nvec, ldx, ldy = self._blk(X, Y)
        p = self._prec(X, prec)
        if shifts is None:
            _check(lib().tp3b_apply_H(self.handle, p, nvec, _ptr(X), ldx, _ptr(Y), ldy,
                                      _stream(stream)))
        else:
            _check(lib().tp3b_apply_H_shifted(self.handle, p, nvec, _ptr(X), ldx, _ptr(Y), ldy,
                                              _ptr(shifts), _stream(stream)))
        return Y

    def apply_prec(self, X, Y, prec=None, stream=None):
        nvec, ldx, ldy = self._blk(X, Y)
        p = self._prec(X, prec)
        _check(lib().tp3b_apply_prec(self.handle, p, nvec, _ptr(X), ldx, _ptr(Y), ldy,
                                     _stream(stream)))
        return Y

    def jdqr(self, nev, block, *, X0=None, inner_prec=FP64, precond=True, tol=1e-12,
             gmres_steps=10, m_min=0, m_max=0, max_outer=1000, seed=0, switch_tol=1e-2,
             target=None, verbose=False, want_Q=True, profile=False, stall_tol=1e-8,
             low_start=3, graph=True, test_dup_column=0):
        import numpy as np
        import torch
        o = JdqrOpts()
        _check(lib().tp3b_jdqr_default_opts(ctypes.byref(o)))
        o.nev, o.block, o.m_min, o.m_max = nev, block, m_min, m_max
        o.gmres_steps, o.max_outer, o.precond = gmres_steps, max_outer, int(bool(precond))
        o.inner_prec, o.tol, o.switch_tol = inner_prec, tol, switch_tol
        o.target = float("nan") if target is None else float(target)
        o.seed, o.verbose, o.profile = seed, int(verbose), int(profile)
        o.stall_tol, o.low_start, o.graph = float(stall_tol), int(low_start), int(bool(graph))
        o.test_dup_column = int(test_dup_column)
        evals = np.empty(nev)
        R = np.empty((nev, nev), order="F")
        res = np.empty(nev)
        Q = torch.empty((nev, self.N), dtype=torch.float64, device="cuda") if want_Q else None
        st = JdqrStats()
        b0 = 0 if X0 is None else X0.shape[0]
        code = lib().tp3b_jdqr_solve(self.handle, ctypes.byref(o), _ptr(X0), b0, _dbl_ptr(evals),
                                     _ptr(Q), R.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     _dbl_ptr(res), ctypes.byref(st))
        result = JdqrResult(evals, Q, R, res, st.as_dict(), code)
        if code != TP3B_OK:
            err = Tp3bError(code, lib().tp3b_last_error().decode())
            err.result = result
            raise err
        return result


@dataclass
class JdqrResult:
    evals: object
    Q: object
    R: object
    resnorm: object
    stats: dict
    status: int


def block_orth(Q, X, seed=0, want_factors=True, stream=None):
    """Orthonormalise the block X (nx, N) in place against Q (nq, N) (FP64).
    Returns (C, R, rank) with C (nq x nx) and R (nx x nx) as torch tensors in
    column-major order (C[:, j] = coefficients of column j)."""
    import torch
    nx, N = X.shape
    nq = 0 if Q is None else Q.shape[0]
    C = torch.empty((nx, max(nq, 1)), dtype=torch.float64, device=X.device) if want_factors else None
    R = torch.empty((nx, nx), dtype=torch.float64, device=X.device) if want_factors else None
    rank = ctypes.c_int32()
    _check(lib().tp3b_block_orth(N, nq, _ptr(Q), Q.stride(0) if nq else N, nx, _ptr(X),
                                 X.stride(0), _ptr(C) if nq else ctypes.c_void_p(0), _ptr(R),
                                 ctypes.byref(rank), seed, _stream(stream)))
    Cm = C.T[:nq] if (want_factors and nq) else None
    Rm = R.T if want_factors else None
    return Cm, Rm, rank.value


def block_orth_noalloc(Q, X, seed=0, stream=None):
    """tp3b_block_orth_noalloc: orthonormalise X (nx, N) in place against Q
    (nq, N) without factors, the library allocating nothing.  Returns the rank."""
    nx, N = X.shape
    nq = 0 if Q is None else Q.shape[0]
    rank = ctypes.c_int32()
    _check(lib().tp3b_block_orth_noalloc(N, nq, _ptr(Q), Q.stride(0) if nq else N, nx, _ptr(X),
                                         X.stride(0), ctypes.byref(rank), seed, _stream(stream)))
    return rank.value


def _ptr_array(items):
    arr = (ctypes.c_void_p * len(items))()
    for i, t in enumerate(items):
        arr[i] = None if t is None else (t if isinstance(t, int) else t.data_ptr())
    return arr


def _batch_blocks(ops, Xs, Ys):
    if not (len(ops) == len(Xs) == len(Ys)) or not ops:
        raise ValueError("one X and one Y block per operator")
    nvec = Xs[0].shape[0]
    ldx = (ctypes.c_int64 * len(ops))()
    ldy = (ctypes.c_int64 * len(ops))()
    for i, (op, X, Y) in enumerate(zip(ops, Xs, Ys)):
        if X.shape[0] != nvec:
            raise ValueError("every block has the same number of vectors")
        _, ldx[i], ldy[i] = op._blk(X, Y)
    return nvec, ldx, ldy


def _batch_prec(Xs, prec):
    p = Operator._prec_of(Xs[0])
    if any(Operator._prec_of(X) != p for X in Xs):
        raise TypeError("all blocks of a batched call have one dtype")
    if prec is None:
        return p
    if (prec == FP64) != (p == FP64):
        raise TypeError("FP64 applies take float64 blocks, FP32/BF16X3 applies float32 blocks")
    return int(prec)


def apply_H_batched(ops, Xs, Ys, prec=None, shifts=None, stream=None):
    """Y_i = H_i X_i for every operator of a batch in grouped launches
    (tp3b_apply_H_batched).  Xs, Ys: lists of (nvec, N_i) tensors."""
    nvec, ldx, ldy = _batch_blocks(ops, Xs, Ys)
    p = _batch_prec(Xs, prec)
    h = _ptr_array([op.handle.value for op in ops])
    sh = _ptr_array(shifts) if shifts is not None else None
    _check(lib().tp3b_apply_H_batched(h, len(ops), p, nvec, _ptr_array(Xs), ldx, _ptr_array(Ys),
                                      ldy, sh, _stream(stream)))
    return Ys


def apply_prec_batched(ops, Xs, Ys, prec=None, stream=None):
    """Y_i = (K_i - sigma_i)^{-1} X_i for every operator of a batch."""
    nvec, ldx, ldy = _batch_blocks(ops, Xs, Ys)
    p = _batch_prec(Xs, prec)
    h = _ptr_array([op.handle.value for op in ops])
    _check(lib().tp3b_apply_prec_batched(h, len(ops), p, nvec, _ptr_array(Xs), ldx,
                                         _ptr_array(Ys), ldy, _stream(stream)))
    return Ys


def autotune_batched(ops, prec=FP64, nvec=1, reps=3):
    """Choose the mode-product tile shape per grid-size group of a batch."""
    h = _ptr_array([op.handle.value for op in ops])
    _check(lib().tp3b_autotune_batched(h, len(ops), int(prec), int(nvec), int(reps)))


@dataclass
class BatchedResult:
    evals: object      # (count, nev)
    resnorm: object    # (count, nev)
    n_conv: object     # (count,)
    n_outer: object    # (count,)
    Q: object          # list of (nev, N_i) tensors or None
    stats: dict
    status: int


def jdqr_batched(ops, nev, block, *, inner_prec=FP64, precond=True, tol=1e-12, gmres_steps=10,
                 m_min=0, m_max=0, max_outer=1000, seed=0, switch_tol=1e-2, target=None,
                 graph=True, want_Q=False, verbose=False, stall_tol=1e-8, low_start=3):
    """Block JDQR on every operator of a batch at once (tp3b_jdqr_solve_batched)."""
    import numpy as np
    import torch
    o = JdqrOpts()
    _check(lib().tp3b_jdqr_default_opts(ctypes.byref(o)))
    o.nev, o.block, o.m_min, o.m_max = nev, block, m_min, m_max
    o.gmres_steps, o.max_outer, o.precond = gmres_steps, max_outer, int(bool(precond))
    o.inner_prec, o.tol, o.switch_tol = inner_prec, tol, switch_tol
    o.target = float("nan") if target is None else float(target)
    o.seed, o.verbose, o.graph = seed, int(verbose), int(bool(graph))
    o.stall_tol, o.low_start = float(stall_tol), int(low_start)
    n = len(ops)
    evals = np.empty((n, nev))
    res = np.empty((n, nev))
    nconv = (ctypes.c_int32 * n)()
    nouter = (ctypes.c_int32 * n)()
    Q = [torch.empty((nev, op.N), dtype=torch.float64, device="cuda") for op in ops] if want_Q else None
    qarr = _ptr_array(Q) if want_Q else None
    st = JdqrStats()
    h = _ptr_array([op.handle.value for op in ops])
    code = lib().tp3b_jdqr_solve_batched(h, n, ctypes.byref(o), _dbl_ptr(evals), _dbl_ptr(res),
                                         nconv, nouter, qarr, ctypes.byref(st))
    result = BatchedResult(evals, res, np.array(nconv[:]), np.array(nouter[:]), Q, st.as_dict(),
                           code)
    if code != TP3B_OK:
        err = Tp3bError(code, lib().tp3b_last_error().decode())
        err.result = result
        raise err
    return result


def host_schur(A):
    """Real Schur form of a small matrix with the library's host QR iteration
    (for host-side tests).  Returns (T, Z, eigenvalues)."""
    import numpy as np
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    Z = np.empty_like(A)
    wr = np.empty(n)
    wi = np.empty(n)
    _check(lib().tp3b_host_schur(n, _dbl_ptr(A), _dbl_ptr(Z), _dbl_ptr(wr), _dbl_ptr(wi)))
    return A, Z, wr + 1j * wi

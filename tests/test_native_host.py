"""Host-side checks of the native library (no GPU needed): it loads, exports
every symbol its header declares, validates arguments before touching the
device, and its host QR iteration computes correct real Schur forms."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2111_02534_amd as t3
    return t3, t3.lib()


def test_exports_every_declared_symbol():
    t3, L = _lib()
    hdr = open(os.path.join(ROOT, "include", "tp3b.h")).read()
    names = set(re.findall(r"\b(tp3b_[a-z0-9_]+)\s*\(", hdr))
    assert names, "no declarations found"
    for n in sorted(names):
        assert hasattr(L, n), n


def test_argument_errors_before_launch():
    t3, L = _lib()
    d = t3.ProblemDesc()
    d.ndim = 3
    h = ctypes.c_void_p()
    assert L.tp3b_create(ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert b"ndim" in L.tp3b_last_error()
    d.ndim = 1
    d.n[0], d.n[1] = 1, 8
    assert L.tp3b_create(ctypes.byref(d), None, ctypes.byref(h)) == -1
    assert L.tp3b_create(None, None, ctypes.byref(h)) == -1
    assert L.tp3b_apply_H(None, 0, 1, None, 1, None, 1, None) == -1
    assert L.tp3b_apply_prec(None, 0, 1, None, 1, None, 1, None) == -1
    r = ctypes.c_int32()
    assert L.tp3b_block_orth(100, 0, None, 100, 40, None, 100, None, None, ctypes.byref(r), 0, None) == -1
    assert L.tp3b_block_orth(100, 0, None, 100, 2, None, 100, None, None, ctypes.byref(r), 0, None) == -1
    o = t3.JdqrOpts()
    assert L.tp3b_jdqr_default_opts(ctypes.byref(o)) == 0
    assert o.tol == 1e-12 and o.gmres_steps == 10
    assert L.tp3b_jdqr_solve(None, ctypes.byref(o), None, 0, None, None, None, None, None) == -1
    assert L.tp3b_destroy(None) == 0


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (30, 3), (64, 4)])
def test_host_schur_random(n, seed):
    t3, _ = _lib()
    A = np.random.default_rng(seed).standard_normal((n, n))
    T, Z, ev = t3.host_schur(A)
    assert np.allclose(Z.T @ Z, np.eye(n), atol=1e-13)
    assert np.max(np.abs(A @ Z - Z @ T)) <= 1e-13 * n * max(1.0, np.max(np.abs(A)))
    assert np.allclose(np.tril(T, -2), 0)
    ref = np.linalg.eigvals(A)
    assert np.allclose(np.sort_complex(ev), np.sort_complex(ref), atol=1e-11)


def test_host_schur_second_derivative():
    from oracle import cheb
    t3, _ = _lib()
    A = -cheb.second_derivative_dirichlet(128, 15.0)
    T, Z, ev = t3.host_schur(A)
    ref = np.sort(np.linalg.eigvals(A).real)
    assert np.max(np.abs(ev.imag)) == 0
    assert np.max(np.abs(np.sort(ev.real) - ref) / ref) <= 1e-11


# ---- two-body depth (host computation in the library)
def _table(name):
    return np.loadtxt(os.path.join(ROOT, "tests", "golden", name))


def test_two_body_depth_1d_matches_oracle_and_table1():
    """Library depth on the even half of a 256-point mapped grid (the
    light-particle mode of a 1D descriptor) against the oracle's generalized
    eigenproblem on the same grid and Table 1's printed depths."""
    from oracle import cheb, twobody
    t3, _ = _lib()
    x, D2 = cheb.parity_half(cheb.mapped_nodes(256, 8.0), cheb.mapped_second_derivative(256, 8.0), +1)
    for E0, v0_paper in _table("table1_paper.txt")[:, :2]:
        got = t3.two_body_depth(E0, 1, [8, 128], [8.0, 8.0], pot="gauss_paper", grid="mapped",
                                parity=[0, 1])
        ref = twobody.depth_for_binding_grid(x, D2, E0)
        assert abs(got - ref) <= 1e-10 * ref, (E0, got, ref)
        assert abs(got - v0_paper) <= 6e-9


@pytest.mark.parametrize("E0,shape,N", [(0.1, "gauss_paper", 48), (0.1, "lorentz3", 56),
                                        (0.01, "gauss_paper", 48)])
def test_two_body_depth_2d_matches_oracle(E0, shape, N):
    """2D: the Cartesian product of the two light-particle modes (even half
    grids), against the oracle's dense generalized eigenproblem."""
    from oracle import cheb, twobody
    t3, _ = _lib()
    f = (lambda r: np.exp(-r * r)) if shape == "gauss_paper" else (lambda r: 1.0 / (1.0 + r * r) ** 3)
    x, D2 = cheb.parity_half(cheb.mapped_nodes(N, 4.0), cheb.mapped_second_derivative(N, 4.0), +1)
    got = t3.two_body_depth(E0, 2, [4, 4, N // 2, N // 2], 4.0, pot=shape, grid="mapped",
                            parity=[0, 0, 1, 1])
    ref = twobody.depth_for_binding_2d(x, D2, E0, f)
    assert abs(got - ref) <= 1e-11 * ref, (got, ref)


def test_two_body_depth_cgl_reduced_mass():
    """CGL grid, Gaussian of width 1.3, heavy-light reduced mass of M/m = 20 in
    heavy-mass units, against the oracle with the mass in its kinetic term."""
    from oracle import cheb, physics, twobody
    t3, _ = _lib()
    _, _, mu = physics.coeffs_unit_heavy(20.0)
    w = 1.3
    got = t3.two_body_depth(0.05, 1, [16, 64], [15.0, 15.0], pot="gauss", width=w, mu_hl=mu)
    x = cheb.nodes(64, 15.0)
    D2 = cheb.second_derivative_dirichlet(64, 15.0)
    ref = twobody.depth_for_binding_grid(x, D2, 0.05, lambda r: np.exp(-r * r / (2 * w * w)), mu=mu)
    assert abs(got - ref) <= 1e-11 * ref, (got, ref)


def test_two_body_depth_argument_errors():
    t3, L = _lib()
    d, keep = t3.make_desc(1, [8, 16], 5.0, pot="harmonic")
    v = ctypes.c_double()
    assert L.tp3b_two_body_depth(ctypes.byref(d), 0.1, ctypes.byref(v)) == -5
    d, keep = t3.make_desc(1, [8, 16], 5.0, pot="gauss_paper")
    assert L.tp3b_two_body_depth(ctypes.byref(d), 0.0, ctypes.byref(v)) == -1
    assert L.tp3b_two_body_depth(ctypes.byref(d), -1.0, ctypes.byref(v)) == -1
    assert L.tp3b_two_body_depth(None, 0.1, ctypes.byref(v)) == -1
    d.n[1] = 4096
    assert L.tp3b_two_body_depth(ctypes.byref(d), 0.1, ctypes.byref(v)) == -1
    o = t3.JdqrOpts()
    L.tp3b_jdqr_default_opts(ctypes.byref(o))
    E = (ctypes.c_double * 1)(0.1)
    assert L.tp3b_homotopy_solve(None, None, ctypes.byref(o), 1, E, None, None, None, None) == -1
    d.n[1] = 16
    assert L.tp3b_homotopy_solve(ctypes.byref(d), None, ctypes.byref(o), 0, E, None, None, None,
                                 None) == -1

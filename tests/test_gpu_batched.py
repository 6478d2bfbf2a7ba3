"""GPU parity of the batched forms: grouped applies over many instances and
the batched block JDQR.

* A grouped apply runs the same tile bodies as the single-operator launch, so
  for the same tile shape its output must equal the single apply bit for bit;
  both are also checked against the oracle.
* The batched eigensolver must reach the dense eigenvalues of each instance
  (oracle's explicit Kronecker matrix) within 1e-10 on small mixed batches, and
  the oracle's stored eigenvalues of all 256 instances of the batched workload.
* Capturing the GMRES iteration as a HIP graph must not change any result: the
  graph is replayed once per outer iteration with eager work and host
  synchronisations in between, and every replay feeds the next iteration, so a
  wrong replay changes the final eigenvalues or iteration counts."""
import os

import numpy as np
import pytest

from gpu_util import need_gpu, say, to_dev
from oracle import dense, physics, problem
from workloads import C4_TOL, c4_instances, normal_block

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (nx, ny, L, alpha, v0, width): ragged, square, several tile shapes
MIX = [(32, 32, 15.0, 20.0, 1.0, 1.0), (37, 50, 9.0, 7.0, 1.5, 0.8), (64, 64, 12.0, 3.0, 2.0, 1.2),
       (96, 96, 15.0, 50.0, 4.0, 0.7), (130, 70, 10.0, 1.5, 0.8, 1.9), (20, 24, 8.0, 10.0, 2.5, 1.0)]


def _make(t3, nx, ny, L, alpha, v0, w):
    cx, cy, mu = physics.coeffs_unit_heavy(alpha)
    op = t3.Operator(1, [nx, ny], [L, L], cx, cy, v0=v0, width=w, mu_hl=mu)
    P = problem.make_problem(ndim=1, n=(nx, ny), L=L, alpha=alpha, v0=v0, width=w)
    return op, P


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_apply_batched_matches_single(prec):
    import torch
    t3 = need_gpu()
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    pairs = [_make(t3, *m) for m in MIX]
    ops = [p[0] for p in pairs]
    nvec = 3
    Xs = [to_dev(normal_block(op.N, nvec, 100 + i), dt) for i, op in enumerate(ops)]
    shifts = [to_dev(np.array([0.3, -1.0, 2.5]) * (i + 1)) for i in range(len(ops))]
    for use_shift in (False, True):
        Yb = [torch.empty_like(X) for X in Xs]
        say("apply batched", prec, "shifted" if use_shift else "")
        t3.apply_H_batched(ops, Xs, Yb, prec=pk, shifts=shifts if use_shift else None)
        torch.cuda.synchronize()
        for i, (op, P) in enumerate(pairs):
            Ys = torch.empty_like(Xs[i])
            op.apply_H(Xs[i], Ys, prec=pk, shifts=shifts[i] if use_shift else None)
            torch.cuda.synchronize()
            assert torch.equal(Ys, Yb[i]), (prec, i)
            if prec == "fp64":
                Xn = Xs[i].cpu().numpy()
                Yr = P.apply(Xn.T).T
                if use_shift:
                    Yr = Yr - shifts[i].cpu().numpy()[:, None] * Xn
                err = np.linalg.norm(Yb[i].cpu().numpy() - Yr) / np.linalg.norm(Yr)
                assert err <= 1e-12, (i, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_apply_prec_batched_matches_single(prec):
    import torch
    t3 = need_gpu()
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[prec]
    dt = torch.float64 if prec == "fp64" else torch.float32
    pairs = [_make(t3, *m) for m in MIX]
    ops = [p[0] for p in pairs]
    nvec = 4
    Xs = [to_dev(normal_block(op.N, nvec, 200 + i), dt) for i, op in enumerate(ops)]
    Yb = [torch.empty_like(X) for X in Xs]
    say("prec batched", prec)
    t3.apply_prec_batched(ops, Xs, Yb, prec=pk)
    torch.cuda.synchronize()
    for i, (op, P) in enumerate(pairs):
        Ys = torch.empty_like(Xs[i])
        op.apply_prec(Xs[i], Ys, prec=pk)
        torch.cuda.synchronize()
        assert torch.equal(Ys, Yb[i]), (prec, i)
        if prec == "fp64":
            pc = P.preconditioner(sigma=op.sigma)
            Zr = pc.apply(Xs[i].cpu().numpy().T).T
            err = np.linalg.norm(Yb[i].cpu().numpy() - Zr) / np.linalg.norm(Zr)
            assert err <= 1e-10, (i, err)


def test_autotune_batched_keeps_results():
    """After the batch autotuner has chosen tiles, the grouped apply still
    matches the oracle (any tile shape computes the same product)."""
    import torch
    t3 = need_gpu()
    pairs = [_make(t3, *m) for m in MIX[:4]]
    ops = [p[0] for p in pairs]
    t3.autotune_batched(ops, t3.FP64, nvec=2, reps=2)
    Xs = [to_dev(normal_block(op.N, 2, 300 + i)) for i, op in enumerate(ops)]
    Yb = [torch.empty_like(X) for X in Xs]
    t3.apply_H_batched(ops, Xs, Yb)
    torch.cuda.synchronize()
    for i, (op, P) in enumerate(pairs):
        Yr = P.apply(Xs[i].cpu().numpy().T).T
        assert np.linalg.norm(Yb[i].cpu().numpy() - Yr) <= 1e-12 * np.linalg.norm(Yr)


SMALL = [(20, 24, 8.0, 10.0, 2.5, 1.0), (24, 24, 10.0, 20.0, 1.0, 1.0), (28, 22, 9.0, 3.0, 3.0, 0.7),
         (32, 32, 15.0, 20.0, 1.0, 1.0), (26, 30, 12.0, 60.0, 4.0, 1.5)]


def _dense_refs(pairs, nev):
    return [dense.lowest_eigenvalues(P.kron(), nev).real for _, P in pairs]


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16x3"])
def test_jdqr_batched_small_vs_dense(inner):
    t3 = need_gpu()
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[inner]
    pairs = [_make(t3, *m) for m in SMALL]
    ops = [p[0] for p in pairs]
    refs = _dense_refs(pairs, 3)
    say("jdqr batched small", inner)
    r = t3.jdqr_batched(ops, 3, 4, inner_prec=pk, seed=5, want_Q=True)
    say("  n_outer", r.n_outer, r.stats)
    for i, (op, P) in enumerate(pairs):
        err = np.max(np.abs(r.evals[i] - refs[i]) / np.abs(refs[i]))
        say("  inst", i, r.evals[i], "err", err)
        assert err <= 1e-10
        Q = r.Q[i].cpu().numpy().T
        assert np.max(np.abs(Q.T @ Q - np.eye(3))) <= 1e-12
        assert np.all(r.resnorm[i] <= 1e-12 * np.maximum(np.abs(r.evals[i]), 1.0) * 1.0001)


def test_jdqr_batched_graph_matches_eager():
    t3 = need_gpu()
    pairs = [_make(t3, *m) for m in SMALL]
    ops = [p[0] for p in pairs]
    for inner in (t3.FP64, t3.FP32):
        say("graph vs eager, inner", inner)
        rg = t3.jdqr_batched(ops, 3, 4, inner_prec=inner, seed=9, graph=True)
        re = t3.jdqr_batched(ops, 3, 4, inner_prec=inner, seed=9, graph=False)
        assert np.array_equal(rg.n_outer, re.n_outer)
        assert np.array_equal(rg.evals, re.evals)
        assert np.array_equal(rg.resnorm, re.resnorm)


def test_jdqr_batched_without_preconditioner():
    t3 = need_gpu()
    pairs = [_make(t3, *m) for m in SMALL[:3]]
    ops = [p[0] for p in pairs]
    refs = _dense_refs(pairs, 2)
    r = t3.jdqr_batched(ops, 2, 2, precond=False, seed=3, max_outer=3000)
    for i in range(len(ops)):
        assert np.max(np.abs(r.evals[i] - refs[i]) / np.abs(refs[i])) <= 1e-10


def test_jdqr_batched_single_instance_matches_solver():
    """A batch of one runs the single-instance iteration (same start block)."""
    t3 = need_gpu()
    op, P = _make(t3, *SMALL[3])
    rb = t3.jdqr_batched([op], 3, 4, seed=2)
    rs = op.jdqr(3, 4, seed=2)
    say("batch of one", rb.evals[0], rs.evals, rb.n_outer, rs.stats["n_outer"])
    assert np.max(np.abs(rb.evals[0] - rs.evals) / np.abs(rs.evals)) <= 1e-12


def _c4_golden():
    path = os.path.join(GOLDEN, "c4_evals.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return np.loadtxt(path)


@pytest.mark.parametrize("inner,steps", [("fp32", 10), ("bf16x3", 10), ("fp64", 3), ("fp32", 3),
                                         ("bf16x3", 3)])
def test_jdqr_c4_full_batch(inner, steps):
    """All 256 instances of the batched workload, inner solves in each
    precision with FP64 outer iteration, against the oracle's stored
    eigenvalues; with the default GMRES step count and with the 3 steps the
    benchmark times."""
    import time

    import torch
    t3 = need_gpu()
    gold = _c4_golden()
    inst = c4_instances()
    assert gold.shape[0] == len(inst)
    ops = [t3.Operator.from_config(c) for c in inst]
    for c, g in zip(inst, gold):
        assert int(g[1]) == c["n"] and abs(g[2] - c["alpha"]) <= 1e-12 * c["alpha"]
    pk = {"fp64": t3.FP64, "fp32": t3.FP32, "bf16x3": t3.BF16X3}[inner]
    torch.cuda.synchronize()
    t0 = time.time()
    r = t3.jdqr_batched(ops, 4, 4, inner_prec=pk, seed=1000, tol=C4_TOL, gmres_steps=steps)
    dt = time.time() - t0
    ref = gold[:, 5:9]
    diff = np.abs(r.evals - ref)
    scale = np.maximum(np.abs(ref), 1.0)
    # Bars:
    # * eigenvalues are compared relative to max(|E|, 1), as residuals are (a
    #   state at the continuum threshold has |E| = 6e-4);
    # * an instance whose pairs all locked at the residual tolerance (both
    #   solvers) agrees to 1e-10;
    # * a pair locked at the FP64 floor of H u (up to ~3e-9 on some of these
    #   grids) carries a first-order eigenvalue error kappa ||r|| in each solver,
    #   kappa ~ 1 (left eigenvectors are the quadrature-weighted right ones), so
    #   the bar is 2 (||r_gpu|| + ||r_oracle||).
    rg = np.nanmax(r.resnorm, axis=1)
    ro = gold[:, 9]
    lim = 1e-12 * np.max(scale, axis=1) * 1.0001
    tight = (rg <= lim) & (ro <= lim)
    err = np.max(diff / scale, axis=1)
    bound = np.maximum(1e-10 * np.max(scale, axis=1), 2.0 * (rg + ro)) / np.max(scale, axis=1)
    say("c4", inner, steps, f"{dt:.2f} s", "outer max", r.n_outer.max(), "mean", r.n_outer.mean())
    say("  instances within 1e-10:", int(np.sum(err <= 1e-10)), "of", len(err),
        "; locked at the tolerance by both:", int(np.sum(tight)),
        "; max err there", float(np.max(err[tight])) if np.any(tight) else None,
        "; max err overall", float(np.max(err)),
        "; worst instance", int(np.argmax(err)), "res gpu/oracle", float(rg[np.argmax(err)]),
        float(ro[np.argmax(err)]))
    assert np.all(r.n_conv == 4)
    assert np.all(err[tight] <= 1e-10)
    assert np.all(err <= bound)

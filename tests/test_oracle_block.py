"""Pins of the block TRPL+K oracle (oracle/block.py; the paper leaves the
block form to future work, Sec. 5.5, so each pin is a property the readings
B1-B5 must keep): s = 1 is TRPL+K step for step; closed-form and dense-LAPACK
spectra for s > 1 with soft and hard locking, B = I and B != I; the
defining invariants of every cycle (T = U^T A U, B-orthonormal basis); the
product-count law; and, with M = c I and B = I, a block-tridiagonal Krylov
part of T (block Lanczos)."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import block as BL
from oracle import trplk as O
from workloads import make, start_block

CASES = [("lap2d", dict(N=24)), ("fem3d", dict(Ne=8, p=6, m=20, k=10)),
         ("aniso3d", dict(N=10, p=12, m=16, k=8, tol=1e-9))]


def _prob(name, kw):
    P = make(name, "small", **kw)
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    return P, A, B, start_block(P.A.n, P.k, 12)


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_block_size_one_is_trplk(name, kw):
    P, A, B, X0 = _prob(name, kw)
    r0 = O.solve(A, B, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=O.jacobi(A))
    r1 = BL.solve(A, B, P.p, P.m, P.k, P.l, 1, P.tol, X0, apply_M=O.jacobi(A))
    assert (r0.cycles, r0.matvecs, r0.precs) == (r1.cycles, r1.matvecs, r1.precs)
    assert np.array_equal(r0.theta, r1.theta) and np.array_equal(r0.X, r1.X)


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("s", [2, 4])
def test_block_spectra_against_dense(name, kw, s):
    P, A, B, X0 = _prob(name, kw)
    r = BL.solve(A, B, P.p, P.m, P.k, P.l, s, P.tol, X0, apply_M=O.jacobi(A))
    ev = sl.eigh(A.toarray(), None if B is None else B.toarray(), eigvals_only=True)[:P.p]
    assert r.converged.all()
    assert np.all(r.true_res <= P.tol * r.normA * 1.001)
    floor = 16 * 2.2e-16 * (r.normA if B is None else np.max(np.abs(ev)))
    assert np.all(np.abs(r.theta - ev) <= np.maximum(1e-9 * np.abs(ev), floor))
    if name == "lap2d":
        i = np.arange(1, 25)
        sv = 4 * np.sin(i * np.pi / 50) ** 2
        closed = np.sort((sv[:, None] + sv[None, :]).ravel())[:P.p]
        assert np.all(np.abs(r.theta - closed) <= 1e-10 * closed)
    if B is None and P.p <= P.k:
        assert r.matvecs == P.k + (P.m - P.k) * r.cycles


def _block_trace(A, B, out, s):
    def tr(cycle, U, AU, BU, T, kact, Q, info):
        nb = U.shape[1]
        out["T"] = max(out.get("T", 0.0), float(np.max(np.abs(T - U.T @ (A @ U)))))
        BUt = U if B is None else B @ U
        out["orth"] = max(out.get("orth", 0.0), float(np.max(np.abs(U.T @ BUt - np.eye(nb)))))
        out["BU"] = max(out.get("BU", 0.0), float(np.max(np.abs(BU - BUt))))
        # block index of every Krylov column; the +K columns come after
        blk = []
        for b, sz in enumerate(info["blocks"]):
            blk += [b] * sz
        kry = slice(kact, kact + len(blk))
        Tk = T[kry, kry]
        far = 0.0
        for i in range(len(blk)):
            for j in range(len(blk)):
                if abs(blk[i] - blk[j]) >= 2:
                    far = max(far, abs(Tk[i, j]))
        out["far"] = max(out.get("far", 0.0), far)
        out["nblk"] = max(out.get("nblk", 0), len(info["blocks"]))
        out["sizes"] = out.get("sizes", set()) | set(info["blocks"])
    return tr


@pytest.mark.parametrize("s", [2, 3])
def test_block_lanczos_structure_for_scalar_preconditioner(s):
    """M = c I, B = I: the inner blocks span a block Krylov space of A, so
    the Krylov part of T is block tridiagonal (entries between blocks two or
    more apart vanish), whatever the per-column shifts."""
    P = make("lap2d", "small", N=20, p=4, m=22, k=6)
    A = P.A.to_scipy()
    X0 = start_block(P.A.n, P.k, 12)
    out = {}
    r = BL.solve(A, None, 4, 22, 6, 1, s, 1e-8, X0, apply_M=lambda v: 0.25 * v,
                 trace=_block_trace(A, None, out, s), max_cycles=60)
    assert out["nblk"] >= 4 and s in out["sizes"]
    assert out["T"] <= 1e-12 * r.normA and out["orth"] <= 1e-12
    assert out["far"] <= 1e-10 * r.normA, out["far"]
    # a preconditioner that is not a multiple of I breaks the structure
    out2 = {}
    BL.solve(A, None, 4, 22, 6, 1, s, 1e-8, X0, apply_M=O.jacobi(A + 0.0 * A),
             trace=_block_trace(A, None, out2, s), max_cycles=3)
    d = A.diagonal()
    if np.ptp(d) == 0.0:   # the 2-D Laplacian's Jacobi is itself c I
        out3 = {}
        Mv = np.linspace(0.5, 1.5, A.shape[0])
        BL.solve(A, None, 4, 22, 6, 1, s, 1e-8, X0, apply_M=lambda v: Mv * v,
                 trace=_block_trace(A, None, out3, s), max_cycles=3)
        assert out3["far"] > 1e-6 * r.normA


def test_block_invariants_generalized():
    P, A, B, X0 = _prob("fem3d", dict(Ne=7, p=4, m=18, k=8))
    out = {}
    r = BL.solve(A, B, 4, 18, 8, 1, 3, 1e-8, X0, apply_M=O.jacobi(A),
                 trace=_block_trace(A, B, out, 3))
    assert r.converged.all()
    assert out["T"] <= 1e-12 * np.max(np.abs(r.theta)) * 10
    assert out["orth"] <= 1e-11 and out["BU"] <= 1e-12


@pytest.mark.parametrize("old,new", [
    ("nxt.append(M(z - shift[j] * Bg))", "nxt.append(M(g - shift[j] * Bg))"),   # no product
    ("col = U[:, :nb + 1].T @ z", "col = U[:, :nb + 1].T @ g"),                 # wrong operand
    ("w, h1 = project(W[:, j])", "w, h1 = W[:, j], np.zeros(1)"),               # no projection
])
def test_block_mutants_fail(old, new):
    import types
    src = open(BL.__file__).read()
    assert old in src
    m = types.ModuleType("oracle.block_mutant")
    m.__package__ = "oracle"
    exec(compile(src.replace(old, new), "block_mutant", "exec"), m.__dict__)
    P, A, B, X0 = _prob("lap2d", dict(N=20, p=4, m=22, k=6))
    out = {}
    try:
        r = m.solve(A, None, 4, 22, 6, 1, 2, 1e-8, X0, apply_M=lambda v: 0.25 * v,
                    trace=_block_trace(A, None, out, 2), max_cycles=200)
    except Exception:
        return
    ev = np.linalg.eigvalsh(A.toarray())[:4]
    bad = (not r.converged.all() or np.max(np.abs(r.theta - ev)) > 1e-9
           or out["T"] > 1e-10 * r.normA or out["orth"] > 1e-10 or out["far"] > 1e-8 * r.normA
           or r.matvecs != 6 + (22 - 6) * r.cycles or out["nblk"] < 4)
    assert bad

"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the expected values are closed
forms of the model operators, dense LAPACK eigendecompositions on tiny
inputs, invariants that exact arithmetic forces, values printed in the paper,
and the paper's special cases.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import trplk as O
from workloads import (make, start_block, lap2d, lap3d, fem3d, aniso3d, powerlaw,
                       lap2d_island, island_block)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solve(P, **kw):
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    X0 = start_block(P.A.n, kw.pop("k", P.k), P.seed)
    prec = kw.pop("prec", "jacobi")
    M = O.jacobi(A) if prec == "jacobi" else prec
    args = dict(p=P.p, m=P.m, k=X0.shape[1], l=P.l, tol=P.tol)
    args.update({x: kw.pop(x) for x in list(kw) if x in args})
    return O.solve(A, B, X0=X0, apply_M=M, **args, **kw), A, B


def _dense_eigs(A, B, p):
    return sl.eigh(A.toarray(), None if B is None else B.toarray(), eigvals_only=True)[:p]


def lap2d_closed(N, p):
    i = np.arange(1, N + 1)
    s = 4 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).ravel())[:p]


# --------------------------------------------------------------------------
# whole solves against closed forms
# --------------------------------------------------------------------------

def test_lap2d_64_closed_form():
    """2-D Laplacian, 64 x 64, p = 5, Jacobi: eigenvalues 4 sin^2 + 4 sin^2."""
    P = make("lap2d", "full")
    r, A, _ = _solve(P)
    ref = lap2d_closed(64, 5)
    assert np.all(np.abs(r.theta - ref) <= 1e-10 * ref)
    assert np.all(r.true_res <= P.tol * r.normA)
    assert r.normA == 8.0
    # the closed form itself: smallest value and the lambda2 = lambda3 pair
    assert abs(ref[0] - 4.671092670693646e-03) < 1e-15
    assert abs(ref[1] - ref[2]) < 1e-15
    # B-orthonormal Ritz vectors
    assert np.max(np.abs(r.X.T @ r.X - np.eye(5))) < 1e-12


def test_lap3d_closed_form_and_weyl():
    """3-D Laplacian: closed form without potential, Weyl bounds with it."""
    N = 14
    Pz = make("lap3d", "small", N=N, vmax=0.0, p=6, m=24, k=10)
    r0, _, _ = _solve(Pz)
    i = np.arange(1, N + 1)
    s = 4 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
    ref = np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())[:6]
    assert np.all(np.abs(r0.theta - ref) <= 1e-10 * ref)
    P = make("lap3d", "small", N=N, vmax=0.05, p=6, m=24, k=10)
    r, A, _ = _solve(P)
    assert np.all(r.theta >= ref - 1e-12) and np.all(r.theta <= ref + 0.05 + 1e-12)
    dense = _dense_eigs(A, None, 6)
    assert np.all(np.abs(r.theta - dense) <= 1e-10 * dense)


def fem_closed(Ne, p):
    h = 1.0 / Ne
    t = np.arange(1, Ne) * np.pi / Ne
    mu = 6 * (1 - np.cos(t)) / (h * h * (2 + np.cos(t)))
    return np.sort((mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).ravel())[:p]


def test_fem3d_generalized_closed_form():
    """Q1 FEM pencil with constant coefficient: lambda = mu_a + mu_b + mu_c."""
    P = make("fem3d", "small", Ne=11, sigma=0.0, p=8, m=24, k=12)
    r, A, B = _solve(P)
    ref = fem_closed(11, 8)
    assert np.all(np.abs(r.theta - ref) <= 1e-10 * ref)
    # B-orthonormal eigenvectors (eq. (1.1))
    assert np.max(np.abs(r.X.T @ (B @ r.X) - np.eye(8))) < 1e-12
    assert np.all(r.true_res <= P.tol * r.normA)


def test_fem3d_lognormal_dense():
    P = make("fem3d", "small", Ne=9, sigma=0.5, p=6, m=20, k=10)
    r, A, B = _solve(P)
    dense = _dense_eigs(A, B, 6)
    assert np.all(np.abs(r.theta - dense) <= 1e-10 * dense)


def test_powerlaw_shifted_laplacian():
    """Connected graph: smallest eigenvalue is the shift, eigenvector constant."""
    P = make("powerlaw", "small", n=1500, p=6, m=24, k=12)
    r, A, _ = _solve(P)
    assert abs(r.theta[0] - 0.01) <= 1e-10 * 0.01
    v = r.X[:, 0] / np.linalg.norm(r.X[:, 0])
    assert abs(abs(v.sum()) / math.sqrt(A.shape[0]) - 1.0) < 1e-6
    dense = _dense_eigs(A, None, 6)
    assert np.all(np.abs(r.theta - dense) <= 1e-9 * dense)


def test_aniso_closed_form_hard_locking():
    """Anisotropic operator, p > k forces hard locking; closed form at sigma = 0."""
    N = 10
    P = make("aniso3d", "small", N=N, sigma=0.0, p=12, m=16, k=8, tol=1e-9)
    r, A, _ = _solve(P)
    i = np.arange(1, N + 1)
    s = 4 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
    ref = np.sort((s[:, None, None] * 1e-4 + s[None, :, None] * 1e-2
                   + s[None, None, :]).ravel())[:12]
    assert np.all(np.abs(r.theta - ref) <= 1e-10 * ref + 16 * 2.2e-16 * r.normA)
    assert np.max(np.abs(r.X.T @ r.X - np.eye(12))) < 1e-10


def test_aniso_lognormal_hard_locking_dense():
    P = make("aniso3d", "small", N=8, sigma=1.0, p=10, m=16, k=6, tol=1e-9)
    r, A, _ = _solve(P)
    dense = _dense_eigs(A, None, 10)
    assert np.all(np.abs(r.theta - dense) <= 1e-10 * np.abs(dense) + 16 * 2.2e-16 * r.normA)
    assert np.all(r.true_res <= 1e-9 * r.normA * 1.01)


# --------------------------------------------------------------------------
# invariants that exact arithmetic forces, checked every cycle
# --------------------------------------------------------------------------

def _invariant_trace(A, B, checks, tridiag=False):
    Bd = None if B is None else B

    def trace(cycle, U, AU, BU, T, kact, Q, info):
        nb = U.shape[1]
        # T equals a dense recompute of U^T A U (eq. (3.1) gives it without
        # extra products)
        Tref = U.T @ (A @ U)
        checks["T"] = max(checks.get("T", 0), np.max(np.abs(T - Tref)))
        checks["Tscale"] = max(checks.get("Tscale", 0), np.max(np.abs(Tref)))
        # B-orthonormal basis, stored products consistent
        G = U.T @ (U if Bd is None else Bd @ U)
        checks["orth"] = max(checks.get("orth", 0), np.max(np.abs(G - np.eye(nb))))
        checks["AU"] = max(checks.get("AU", 0), np.max(np.abs(AU - A @ U)))
        # after a restart T(1:k,1:k) = Theta (Sec. 3)
        off = T[:kact, :kact] - np.diag(np.diag(T[:kact, :kact]))
        checks["diag"] = max(checks.get("diag", 0), np.max(np.abs(off)))
        if tridiag:
            # with M = c I and B = I the Krylov block of T is tridiagonal
            nk = nb - kact - (1 if cycle > 1 else 0)
            Gb = T[kact:kact + nk, kact:kact + nk]
            band = np.triu(Gb, 2)
            checks["tri"] = max(checks.get("tri", 0), np.max(np.abs(band)) if nk > 2 else 0.0)
    return trace


def test_invariants_standard_tridiagonal():
    P = make("lap2d", "small", N=20, p=4, m=16, k=6)
    A = P.A.to_scipy()
    checks = {}
    r = O.solve(A, None, P.p, P.m, P.k, P.l, P.tol, start_block(A.shape[0], P.k, 12),
                apply_M=lambda v: 0.25 * v, trace=_invariant_trace(A, None, checks, True),
                keep_history=True)
    nA = r.normA
    assert checks["T"] < 1e-12 * nA
    assert checks["orth"] < 1e-12
    assert checks["diag"] < 1e-12 * nA
    assert checks["tri"] < 1e-12 * nA
    # Ritz values never increase from cycle to cycle (span(X_i) is kept in
    # the next basis) and never drop below the eigenvalues (interlacing)
    lam = lap2d_closed(20, 4)
    th = np.array([h[0] for h in r.history])
    assert np.all(np.diff(th, axis=0) <= 1e-12 * nA)
    assert np.all(th >= lam[None, :] - 1e-12 * nA)


def test_invariants_generalized_preconditioned():
    P = make("fem3d", "small", Ne=8, sigma=0.5, p=4, m=16, k=6)
    A, B = P.A.to_scipy(), P.B.to_scipy()
    checks = {}
    r = O.solve(A, B, P.p, P.m, P.k, P.l, P.tol, start_block(A.shape[0], P.k, 12),
                apply_M=O.jacobi(A), trace=_invariant_trace(A, B, checks), keep_history=True)
    # B-normalised vectors are long when B is small: T scales with the
    # Ritz values, not with ||A||
    assert checks["T"] < 1e-13 * checks["Tscale"]
    assert checks["orth"] < 1e-12
    th = np.array([h[0] for h in r.history])
    assert np.all(np.diff(th, axis=0) <= 1e-12 * r.normA)


# --------------------------------------------------------------------------
# structural pins from the paper
# --------------------------------------------------------------------------

def test_paper_mv_counts_follow_restart_law():
    """Every TRPL+K MV count printed for the standard problem (Tables 2-5) is
    minRestartSize + (maxBasisSize - minRestartSize) * cycles = 8 + 10 c; the
    oracle with the same sizes spends exactly that many products."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "paper_trplk_mv.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 22
    assert all(int(r[3]) % 10 == 8 for r in rows)
    P = make("lap2d", "small", N=30, p=5, m=18, k=8, l=1)
    r, _, _ = _solve(P)
    assert r.matvecs == 8 + 10 * r.cycles


def test_exact_preconditioner_converges_in_few_cycles():
    """Remark after Thm. 4.1: with M = (A - sigma B)^{-1}, sigma < lambda_1
    close to lambda_1, the preconditioned spectrum clusters at 1 and the
    outer iteration converges in very few cycles."""
    P = make("lap2d", "small", N=16, p=1, m=8, k=2, l=1)
    A = P.A.to_scipy()
    lam = lap2d_closed(16, 1)[0]
    Minv = np.linalg.inv(A.toarray() - 0.9 * lam * np.eye(A.shape[0]))
    r = O.solve(A, None, 1, 8, 2, 1, 1e-10, start_block(A.shape[0], 2, 12),
                apply_M=lambda v: Minv @ v)
    assert r.cycles <= 3
    assert abs(r.theta[0] - lam) <= 1e-10 * lam


def test_plus_k_reduces_matvecs():
    """Sec. 5.2 / Fig. 3: one previous vector (l = 1) cuts the product count
    against l = 0, which is thick-restart Lanczos without preconditioning."""
    A = aniso3d(14, 1.0, axis_w=(1.0, 1e-1, 1e-2)).to_scipy()
    X0 = start_block(A.shape[0], 8, 12)
    r0 = O.solve(A, None, 5, 18, 8, 0, 1e-8, X0)
    r1 = O.solve(A, None, 5, 18, 8, 1, 1e-8, X0)
    r2 = O.solve(A, None, 5, 18, 8, 2, 1e-8, X0)
    assert r1.matvecs < 0.6 * r0.matvecs
    assert r2.matvecs < 0.6 * r0.matvecs
    assert np.allclose(r0.theta, r1.theta, rtol=1e-9)


def test_lopcg_special_case():
    """One inner step with p = k = l = 1 is LOPCG (Sec. 2.2, 5.1): it must
    converge to the smallest eigenpair."""
    A = lap2d(12).to_scipy()
    r = O.solve(A, None, 1, 3, 1, 1, 1e-9, start_block(A.shape[0], 1, 12),
                apply_M=O.jacobi(A), max_cycles=3000)
    lam = lap2d_closed(12, 1)[0]
    assert r.converged.all() and abs(r.theta[0] - lam) < 1e-9 * 8


def test_optimal_step_lemma():
    """Lemma 4.3 (eq. coefabc): the smallest Ritz value of span{x, p} equals
    rho(x + alpha* p), alpha* the smaller positive root of a a^2 + b a + c."""
    rng = np.random.default_rng(3)
    A = lap2d(8).to_scipy().toarray()
    Bm = np.diag(rng.uniform(1, 2, A.shape[0]))
    w, V = sl.eigh(A, Bm)
    x = V[:, 0] + 0.05 * rng.standard_normal(A.shape[0])
    x /= math.sqrt(x @ Bm @ x)
    rho = lambda v: (v @ A @ v) / (v @ Bm @ v)  # noqa: E731
    g = A @ x - rho(x) * Bm @ x
    p = -np.linalg.solve(A - 0.5 * w[0] * Bm, g)   # descent direction
    a = (p @ A @ p) * (p @ Bm @ x) - (p @ Bm @ p) * (p @ A @ x)
    b = (p @ A @ p) * (x @ Bm @ x) - (p @ Bm @ p) * (x @ A @ x)
    c = (p @ A @ x) * (x @ Bm @ x) - (p @ Bm @ x) * (x @ A @ x)
    roots = np.roots([a, b, c])
    pos = sorted(rr.real for rr in roots if abs(rr.imag) < 1e-14 and rr.real > 0)
    alpha = pos[0]
    # the oracle's Rayleigh-Ritz on the 2-D space {x, p}
    U = np.column_stack([x, p])
    W = np.zeros((U.shape[0], 0))
    q0, _ = O.b_cgs2(U[:, 0], W, W)
    q0 /= math.sqrt(q0 @ Bm @ q0)
    q1, _ = O.b_cgs2(U[:, 1], q0[:, None], (Bm @ q0)[:, None])
    q1 /= math.sqrt(q1 @ Bm @ q1)
    Qm = np.column_stack([q0, q1])
    th = np.linalg.eigh(Qm.T @ A @ Qm)[0][0]
    assert abs(th - rho(x + alpha * p)) < 1e-12 * abs(th)
    # and no other step along p does better
    for a2 in (0.5 * alpha, 2 * alpha, -alpha):
        assert rho(x + a2 * p) > th


@pytest.mark.parametrize("s,k,m,prec", [(6, 4, 12, "jacobi"), (9, 3, 16, None)])
def test_breakdown_in_an_invariant_subspace(s, k, m, prec):
    """A start block inside an s-dimensional invariant subspace (a
    disconnected path of s nodes): the Krylov block is exhausted after s - k
    vectors, the next one is zero up to rounding, the inner loop stops
    (breakdown, R7), and the Rayleigh-Ritz pairs on the s-dimensional basis
    are exact eigenpairs of the path block after one cycle."""
    A = lap2d_island(20, s).to_scipy()
    n = A.shape[0]
    ev = np.linalg.eigvalsh(A.toarray()[n - s:, n - s:])
    seen = []
    r = O.solve(A, None, 2, m, k, 1, 1e-10, island_block(n, s, k, 7),
                apply_M=O.jacobi(A) if prec else None,
                trace=lambda c, U, AU, BU, T, ka, Q, info: seen.append((U.shape[1], info["nk"])))
    assert seen == [(s, s - k)]
    assert r.cycles == 1 and r.matvecs == s
    assert np.all(np.abs(r.theta - ev[:2]) <= 1e-14 * r.normA)
    assert np.all(r.true_res <= 1e-14 * r.normA)
    assert np.all(r.X[:n - s] == 0.0)


def test_basis_filling_the_whole_space():
    """m = n: the first cycle's basis spans R^n (no breakdown on a 6 x 6 grid),
    so its Rayleigh-Ritz pairs are the exact eigenpairs (closed form)."""
    A = lap2d(6).to_scipy()
    seen = []
    r = O.solve(A, None, 3, 36, 6, 1, 1e-10, start_block(36, 6, 12), apply_M=O.jacobi(A),
                trace=lambda c, U, AU, BU, T, ka, Q, info: seen.append(U.shape[1]))
    assert seen == [36] and r.cycles == 1 and r.matvecs == 36
    assert np.all(np.abs(r.theta - lap2d_closed(6, 3)) <= 1e-13 * r.normA)


def test_input_validation():
    A = lap2d(6).to_scipy()
    with pytest.raises(ValueError):
        O.solve(A, None, 5, 10, 4, 1, 1e-8, start_block(36, 4, 1), locking="soft")
    with pytest.raises(ValueError):
        O.solve(A, None, 2, 5, 4, 1, 1e-8, start_block(36, 4, 1))


# --------------------------------------------------------------------------
# planted mistakes: a plausible error in the oracle must fail a pin
# --------------------------------------------------------------------------

def _mutant(old, new):
    import sys
    import types
    src = open(O.__file__).read()
    assert old in src, old
    mod = types.ModuleType("oracle_mutant")
    sys.modules["oracle_mutant"] = mod
    try:
        exec(compile(src.replace(old, new, 1), "oracle_mutant", "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle_mutant"]
    return mod


def _krylov_trace(A, B, M, worst):
    """The inner block must span K_m(C, u1) with C = (I - X X^T B) M (A - rho B)
    and u1 = C x_t (Sec. 3, eq. (3.2)): C applied to each Krylov vector stays
    in the span of X and the Krylov vectors up to the next one."""
    Bm = (lambda v: v) if B is None else (lambda v: B @ v)

    def resid(W, v):
        return np.linalg.norm(v - W @ (W.T @ Bm(v))) / np.linalg.norm(v)

    def trace(cycle, U, AU, BU, T, kact, Q, info):
        rho, t, nk = info["rho"], info["t"], info["nk"]
        X = U[:, :kact]
        v = M(A @ X[:, t] - rho * Bm(X[:, t]))
        worst[0] = max(worst[0], resid(U[:, :kact + 1], v))
        for j in range(nk - 1):
            g = U[:, kact + j]
            v = M(A @ g - rho * Bm(g))
            worst[0] = max(worst[0], resid(U[:, :kact + j + 2], v))
    return trace


def test_krylov_relation_generalized_jacobi():
    P = make("fem3d", "small", Ne=8, sigma=0.5, p=3, m=14, k=5)
    A, B = P.A.to_scipy(), P.B.to_scipy()
    M = O.jacobi(A)
    worst = [0.0]
    O.solve(A, B, 3, 14, 5, 1, 1e-8, start_block(A.shape[0], 5, 12), apply_M=M,
            trace=_krylov_trace(A, B, M, worst), max_cycles=15)
    assert worst[0] < 1e-7


@pytest.mark.parametrize("old,new", [
    ("w = M(z - rho * Bg)", "w = M(z + rho * Bg)"),                 # wrong sign
    ("w = M(AX[:, t] - rho * BX[:, t])", "w = M(AX[:, t])"),        # dropped term
    ("w = M(z - rho * Bg)", "w = M(z - rho * g)"),                  # B dropped
])
def test_mutant_fails_krylov_relation(old, new):
    Om = _mutant(old, new)
    P = make("fem3d", "small", Ne=8, sigma=0.5, p=3, m=14, k=5)
    A, B = P.A.to_scipy(), P.B.to_scipy()
    M = O.jacobi(A)
    worst = [0.0]
    Om.solve(A, B, 3, 14, 5, 1, 1e-8, start_block(A.shape[0], 5, 12), apply_M=M,
             trace=_krylov_trace(A, B, M, worst), max_cycles=15)
    assert worst[0] > 1e-4


@pytest.mark.parametrize("old,new", [
    ("col = U[:, :nb + 1].T @ z", "col = U[:, :nb + 1].T @ g"),      # wrong operand
    ("T[nb, :nb + 1] = col", "T[nb, :nb] = col[1:]"),               # row shifted
    ("h2 = BU.T @ w\n    w = w - U @ h2", "h2 = BU.T @ w\n    w = w + U @ h2"),
])
def test_mutant_fails_invariants(old, new):
    Om = _mutant(old, new)
    P = make("lap2d", "small", N=20, p=4, m=16, k=6)
    A = P.A.to_scipy()
    checks = {}
    try:
        r = Om.solve(A, None, 4, 16, 6, 1, 1e-8, start_block(A.shape[0], 6, 12),
                     apply_M=lambda v: 0.25 * v, trace=_invariant_trace(A, None, checks, True),
                     max_cycles=40)
    except Exception:
        return
    bad = (checks["T"] > 1e-10 * r.normA or checks["orth"] > 1e-10
           or checks.get("tri", 0) > 1e-10 * r.normA)
    assert bad


def test_mutant_prev_vectors_fail_mv_pin():
    """Taking the +K vectors after the new Rayleigh-Ritz breaks the count law
    only if it changes the loop length; placing X_prev before the Krylov
    block shrinks the inner loop and the law catches that."""
    Om = _mutant("m_in = m - kact - Xprev.shape[1]", "m_in = m - kact")
    P = make("lap2d", "small", N=30, p=5, m=18, k=8, l=1)
    A = P.A.to_scipy()
    try:
        r = Om.solve(A, None, 5, 18, 8, 1, 1e-8, start_block(A.shape[0], 8, 12),
                     apply_M=O.jacobi(A))
    except IndexError:
        return  # the basis overflows its m columns
    assert r.matvecs != 8 + 10 * r.cycles


# --------------------------------------------------------------------------
# the paper's stopping norm and the un-flag branch of the convergence test
# --------------------------------------------------------------------------

def test_frobenius_norm_and_paper_stopping_rule():
    """eq. (5.1) stops on ||A u - theta u|| <= ||A||_F tol.  For the 64 x 64
    5-point Laplacian ||A||_F^2 = 4096 * 4^2 + 2 * (2 * 64 * 63) * 1^2 =
    81664 (diagonal entries plus both triangles of the 2 * 64 * 63 grid
    edges), ||A||_F = 285.769..., and ||A||_inf = 8 (max row sum)."""
    A = lap2d(64).to_scipy()
    assert O.matrix_norm(A, "fro") == math.sqrt(81664.0)
    assert abs(math.sqrt(81664.0) - 285.769) < 5e-4
    assert O.matrix_norm(A, "inf") == 8.0
    # a hand-sized matrix: [[3, -4], [-4, 0]]: F = sqrt(9 + 32) , inf = 7
    M = sp.csr_matrix(np.array([[3.0, -4.0], [-4.0, 0.0]]))
    assert O.matrix_norm(M, "fro") == math.sqrt(41.0)
    assert O.matrix_norm(M, "inf") == 7.0
    # the solve under the Frobenius rule: threshold tol * 285.769, every
    # returned pair meets it, the inf-norm run (a 35x tighter threshold)
    # needs more cycles
    P = make("lap2d", "small", N=24, p=5, m=20, k=8)
    r_f, A24, _ = _solve(P, norm="fro")
    r_i, _, _ = _solve(P, norm="inf")
    nf = math.sqrt(float(np.sum(A24.data ** 2)))
    assert r_f.normA == nf
    assert np.all(r_f.true_res <= P.tol * nf)
    assert r_f.cycles < r_i.cycles
    assert np.any(r_f.true_res > P.tol * 8.0)   # looser than the inf rule
    ref = lap2d_closed(24, 5)
    assert np.all(np.abs(r_f.theta - ref) <= 1e-8 * nf)


def weak_island_problem(delta=1e-2, eps=1e-12, N=16, s=16, k=4):
    """A 2-D Laplacian next to a disconnected path whose lowest eigenvalue
    lies delta below the grid's, started from a block whose path part is
    scaled by eps.  The grid's lowest pair converges first; the path's mode,
    amplified from eps, then enters below it (R8 un-flag), and the solve
    recovers both.  Block-diagonal A and a diagonal M keep the path part of
    every vector a function of the path part alone, so the event does not
    hang on rounding."""
    lam1 = 8 * np.sin(np.pi / (2 * (N + 1))) ** 2
    dg = lam1 - delta + 2 * np.cos(np.pi / (s + 1))
    A = lap2d_island(N, s, dg)
    X0 = start_block(A.n, k, 12).copy(order="F")
    X0[N * N:, :] *= eps
    return A, X0


def test_soft_locked_pair_unflagged_when_a_lower_mode_appears():
    """R8: a flagged (soft-locked) pair whose residual leaves the tolerance is
    unflagged and the target moves back; the final pairs are the two lowest
    eigenpairs of the whole matrix (dense LAPACK)."""
    Ac, X0 = weak_island_problem()
    A = Ac.to_scipy()
    r = O.solve(A, None, 2, 12, 4, 1, 1e-8, X0, apply_M=O.jacobi(A), keep_history=True)
    ts = [h[2] for h in r.history]
    drops = [c for c in range(1, len(ts)) if ts[c] < ts[c - 1]]
    assert drops, ts
    c = drops[0]
    thr = 1e-8 * r.normA
    # the pair flagged before the drop had met the tolerance, the new lowest
    # Ritz value after it is far from converged and lies below the old one
    assert r.history[c - 1][1][0] <= thr
    assert r.history[c][1][0] > 100 * thr
    assert r.history[c][0][0] < r.history[c - 1][0][0] - 1e-3
    ev = np.linalg.eigvalsh(A.toarray())[:2]
    assert r.converged.all()
    assert np.all(np.abs(r.theta - ev) <= 1e-12)
    assert (r.cycles, r.matvecs) == (20, 4 + 8 * 20)


@pytest.mark.parametrize("gen", ["standard", "generalized"])
def test_start_depends_only_on_the_span_of_x0(gen):
    """Reading R2: Alg. 1 starts from a B-orthonormal basis of span(X0)
    followed by a Rayleigh-Ritz on it, so any such basis gives the same
    first cycle.  X0 and X0 R (R upper triangular, well conditioned: the
    Cholesky-QR route the GPU takes for k >= 8 is of this form) give the
    same Ritz values after one and after three cycles, and the same product
    counts; a start block with one column replaced does not."""
    if gen == "standard":
        P = make("lap2d", "small", N=20, p=4, m=16, k=8)
        A, B = P.A.to_scipy(), None
    else:
        P = make("fem3d", "small", Ne=6, p=4, m=16, k=8)
        A, B = P.A.to_scipy(), P.B.to_scipy()
    X0 = start_block(A.shape[0], P.k, 12)
    rng = np.random.default_rng(7)
    R = np.triu(rng.uniform(-0.3, 0.3, (P.k, P.k))) + np.eye(P.k) * 2.0
    Xr = X0 @ R
    Xo = X0.copy()
    Xo[:, -1] = rng.uniform(-1.0, 1.0, A.shape[0])
    M = O.jacobi(A)
    for cycles in (1, 3):
        a = O.solve(A, B, P.p, P.m, P.k, P.l, 1e-300, X0, apply_M=M, max_cycles=cycles)
        b = O.solve(A, B, P.p, P.m, P.k, P.l, 1e-300, Xr, apply_M=M, max_cycles=cycles)
        c = O.solve(A, B, P.p, P.m, P.k, P.l, 1e-300, Xo, apply_M=M, max_cycles=cycles)
        scale = np.max(np.abs(a.theta))
        assert a.matvecs == b.matvecs
        assert np.max(np.abs(a.theta - b.theta)) <= 1e-12 * scale
        assert np.max(np.abs(a.theta - c.theta)) > 1e-9 * scale

"""Plain, slow, FP64 CPU oracle of TRPL+K.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import this module.  It shares no code with the HIP library: every step is
written out here with NumPy / SciPy primitives (sparse products, dense
products, numpy.linalg.eigh) and no blocking, fusion or reordering beyond
what the method states.

What it follows (Wu, Xue, Stathopoulos, "TRPL+K", arXiv 1711.10128):

* the problem, eq. (1.1): the p smallest eigenpairs of A v = lambda B v with
  A symmetric, B symmetric positive definite, B-orthonormal eigenvectors;
* Algorithm 1 (TRPL+K) for the cycle structure: an initial Rayleigh-Ritz on
  the start block, then per cycle an inner Krylov loop on the projected,
  preconditioned operator C = (I - X X^T B) M (A - rho B) started from
  u1 = C x_t, the T update of eq. (3.1) that gives T = U^T A U without extra
  products, +K augmentation with the previous cycle's Ritz vectors placed
  after the Krylov block (Sec. 3, eq. (3.2)), Rayleigh-Ritz on T, the
  convergence test and target advance, and the thick restart;
* Sec. 3 last paragraph / Sec. 4.2 (Algorithm 2) for the generalized
  problem: B-inner products, B-normalized basis, residual A x - theta B x;
* the stopping rule of eq. (5.1), ||A u - theta u|| <= ||A|| * tol.

Readings where the paper is silent or garbled (each one is listed in the
design notes of the repository):

R2  the start block has k columns (the thick-restart size), not p;
R3  the next inner direction is M (A g_j - rho B g_j), projected against X
    and all previous inner vectors (full B-orthogonalisation, classical
    Gram-Schmidt applied twice);
R6  the inner loop runs m - k - |X_prev| steps so that the basis fills to m
    each cycle (m = maximum basis size, k = restart size);
R7  breakdown: the inner loop stops when the new B-norm squared is at most
    (1e-14)^2 times (|h1|^2 + beta^2), h1 the first-pass coefficients; a +K
    vector is dropped under the same test with 1e-12;
R8  the convergence test loops over consecutive targets; a soft-locked
    pair whose residual grows above the tolerance is unflagged;
R9  ||A|| is the infinity norm by default ('fro' reproduces the paper);
R11 with hard locking a converged pair leaves the basis for a locked set Q
    that every new vector is B-orthogonalised against; a final p x p
    Rayleigh-Ritz on Q gives the returned pairs;
    the residual of a pair is ||A x - theta B x||_2 / ||x||_2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

BREAKDOWN_TOL = 1e-14   # R7, inner steps
PLUSK_DROP_TOL = 1e-12  # R7, +K vectors


@dataclasses.dataclass
class Result:
    theta: np.ndarray        # (p,) ascending Ritz values
    X: np.ndarray            # (n, p) B-orthonormal Ritz vectors
    res: np.ndarray          # (p,) residual norms from the stored A X, B X
    true_res: np.ndarray     # (p,) residual norms from fresh products
    converged: np.ndarray    # (p,) bool
    cycles: int
    matvecs: int             # products with A
    bvecs: int               # products with B (0 when B = I)
    precs: int               # preconditioner applications
    normA: float
    history: list            # per cycle: (theta[:p].copy(), res[:p].copy(), t)


def matrix_norm(A, kind: str = "inf") -> float:
    """||A||_inf (max absolute row sum) or ||A||_F."""
    A = sp.csr_matrix(A)
    if kind == "inf":
        return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))
    if kind == "fro":
        return float(math.sqrt(float(np.sum(A.data ** 2))))
    raise ValueError(kind)


class _Pencil:
    """Products with A and B, counted."""

    def __init__(self, A, B):
        self.A = sp.csr_matrix(A)
        self.B = None if B is None else sp.csr_matrix(B)
        self.nA = 0
        self.nB = 0

    def Av(self, x):
        self.nA += 1 if x.ndim == 1 else x.shape[1]
        return self.A @ x

    def Bv(self, x):
        if self.B is None:
            return x.copy()
        self.nB += 1 if x.ndim == 1 else x.shape[1]
        return self.B @ x


def b_cgs2(w, U, BU):
    """Classical Gram-Schmidt in the B-inner product, applied twice.

    U has B-orthonormal columns and BU = B U.  Returns the projected vector
    and the first-pass coefficients h1 = (B U)^T w.
    """
    if U.shape[1] == 0:
        return w.copy(), np.zeros(0)
    h1 = BU.T @ w
    w = w - U @ h1
    h2 = BU.T @ w
    w = w - U @ h2
    return w, h1


def solve(A, B, p: int, m: int, k: int, l: int, tol: float, X0: np.ndarray,
          apply_M: Optional[Callable[[np.ndarray], np.ndarray]] = None,
          norm: str = "inf", locking: str = "auto", max_cycles: int = 5000,
          keep_history: bool = False, trace=None) -> Result:
    """TRPL+K for the p smallest eigenpairs of (A, B); B None means B = I.

    m  maximum basis size (the paper's q), k  thick-restart size (>= p for
    soft locking), l  number of previous Ritz vectors (+K), tol  stopping
    tolerance relative to ||A||, X0 (n, k) start block, apply_M(r) the
    preconditioner (None = identity).  trace(cycle, U, AU, BU, T, kact, Q,
    info) is called before each Rayleigh-Ritz with the basis, its products,
    the projected matrix, the restart size, the locked set and a dict with
    the shift, the target and the Krylov block length (tests only).
    """
    P = _Pencil(A, B)
    n = P.A.shape[0]
    if locking == "auto":
        locking = "soft" if p <= k else "hard"
    if locking == "soft" and p > k:
        raise ValueError("soft locking needs p <= k")
    if not (1 <= k and k + l + 1 <= m <= n):
        raise ValueError("need k >= 1 and k + l + 1 <= m <= n")
    if X0.shape != (n, k):
        raise ValueError("X0 must be n x k")
    M = apply_M if apply_M is not None else (lambda r: r.copy())
    precs = 0
    normA = matrix_norm(P.A, norm)
    thr = tol * normA
    hard = locking == "hard"

    # locked set (hard locking only)
    Q = np.zeros((n, 0))
    AQ = np.zeros((n, 0))
    BQ = np.zeros((n, 0))

    # --- Alg. 1 start: B-orthonormalise X0 and Rayleigh-Ritz on span(X0) ---
    X = np.zeros((n, k))
    BX = np.zeros((n, k))
    for c in range(k):
        w, h1 = b_cgs2(X0[:, c].astype(np.float64), X[:, :c], BX[:, :c])
        Bw = P.Bv(w)
        beta = math.sqrt(float(w @ Bw))
        if not beta > 0.0:
            raise ValueError("start block is rank deficient")
        X[:, c] = w / beta
        BX[:, c] = Bw / beta
    AX = P.Av(X)
    T0 = X.T @ AX
    T0 = 0.5 * (T0 + T0.T)
    theta, Y = np.linalg.eigh(T0)
    X, AX, BX = X @ Y, AX @ Y, BX @ Y

    t = 0
    Xprev = np.zeros((n, 0))
    history = []
    cycles = 0
    done = False
    theta_lock = np.zeros(0)
    kact = k  # active restart size this cycle (hard locking may shrink it)
    res = np.full(k, np.inf)

    for cycle in range(1, max_cycles + 1):
        cycles = cycle
        rho = float(theta[t])
        # u1 = C x_t: projected preconditioned residual of the target (Alg. 1 restart)
        w = M(AX[:, t] - rho * BX[:, t])
        precs += 1
        U = np.zeros((n, m))
        AU = np.zeros((n, m))
        BU = np.zeros((n, m))
        U[:, :kact], AU[:, :kact], BU[:, :kact] = X, AX, BX
        T = np.zeros((m, m))
        T[np.arange(kact), np.arange(kact)] = theta[:kact]
        nb = kact
        m_in = m - kact - Xprev.shape[1]
        nk = 0

        def project(v):
            # B-orthogonalise against the locked set and the current basis
            W = np.hstack([Q, U[:, :nb]])
            BW = np.hstack([BQ, BU[:, :nb]])
            return b_cgs2(v, W, BW)

        def append(w, h1, drop_tol):
            nonlocal nb
            Bw = P.Bv(w)
            beta2 = float(w @ Bw)
            if not beta2 > drop_tol ** 2 * (float(h1 @ h1) + beta2):
                return None
            beta = math.sqrt(beta2)
            g = w / beta
            z = P.Av(g)
            U[:, nb], AU[:, nb], BU[:, nb] = g, z, Bw / beta
            col = U[:, :nb + 1].T @ z           # eq. (3.1): new column of T
            T[:nb + 1, nb] = col
            T[nb, :nb + 1] = col
            nb += 1
            return g, z, Bw / beta

        # --- inner preconditioned Krylov loop (Alg. 1, eq. (3.1)) ---
        for s in range(m_in):
            w, h1 = project(w)
            out = append(w, h1, BREAKDOWN_TOL)
            if out is None:
                break
            nk = s + 1
            g, z, Bg = out
            if s < m_in - 1:
                w = M(z - rho * Bg)
                precs += 1
        # --- +K: previous Ritz vectors placed after the Krylov block (Sec. 3) ---
        for c in range(Xprev.shape[1]):
            w, h1 = project(Xprev[:, c])
            append(w, h1, PLUSK_DROP_TOL)
        # previous vectors are taken from X before the new Rayleigh-Ritz (Alg. 1)
        want = (p - Q.shape[1]) if hard else p
        Xprev_new = X[:, t:min(t + l, want)].copy()
        # --- Rayleigh-Ritz on T (Alg. 1) ---
        Tb = T[:nb, :nb]
        if trace is not None:
            trace(cycle, U[:, :nb], AU[:, :nb], BU[:, :nb], Tb, kact, Q,
                  {"rho": rho, "t": t, "nk": nk})
        theta_all, Yall = np.linalg.eigh(Tb)
        kk = min(k, nb)
        Yk = Yall[:, :kk]
        X = U[:, :nb] @ Yk
        AX = AU[:, :nb] @ Yk
        BX = BU[:, :nb] @ Yk
        theta = theta_all[:kk].copy()
        xn = np.linalg.norm(X, axis=0)
        res = np.linalg.norm(AX - BX * theta[None, :], axis=0) / xn
        # --- convergence test and target advance (Alg. 1, R8) ---
        if not hard:
            conv = res[:p] <= thr
            t_new = int(np.argmin(conv)) if not conv.all() else p
            if t_new > t:
                Xprev_new = Xprev_new[:, min(t_new - t, Xprev_new.shape[1]):]
            t = t_new
            Xprev = Xprev_new
            if keep_history:
                history.append((theta[:p].copy(), res[:p].copy(), t))
            if t >= p:
                done = True
                break
            kact = kk
        else:
            nlock = 0
            while Q.shape[1] < p and nlock < kk and res[nlock] <= thr:
                nlock += 1
            if nlock:
                Q = np.hstack([Q, X[:, :nlock]])
                AQ = np.hstack([AQ, AX[:, :nlock]])
                BQ = np.hstack([BQ, BX[:, :nlock]])
                theta_lock = np.concatenate([theta_lock, theta[:nlock]])
                X, AX, BX = X[:, nlock:], AX[:, nlock:], BX[:, nlock:]
                theta, res = theta[nlock:], res[nlock:]
                Xprev_new = Xprev_new[:, min(nlock, Xprev_new.shape[1]):]
            Xprev = Xprev_new
            t = 0
            kact = X.shape[1]
            if keep_history:
                history.append((theta_lock.copy(), res.copy(), Q.shape[1]))
            if Q.shape[1] >= p:
                done = True
                break

    if hard:
        # final Rayleigh-Ritz on the locked set (R11)
        if Q.shape[1] > 0:
            TQ = Q.T @ AQ
            TQ = 0.5 * (TQ + TQ.T)
            thq, YQ = np.linalg.eigh(TQ)
            Q, AQ, BQ = Q @ YQ, AQ @ YQ, BQ @ YQ
        nq = Q.shape[1]
        theta_out = np.concatenate([thq if nq else np.zeros(0), theta])[:p]
        X_out = np.hstack([Q, X])[:, :p]
        AX_out = np.hstack([AQ, AX])[:, :p]
        BX_out = np.hstack([BQ, BX])[:, :p]
    else:
        theta_out, X_out, AX_out, BX_out = theta[:p], X[:, :p], AX[:, :p], BX[:, :p]
    xn = np.linalg.norm(X_out, axis=0)
    res_out = np.linalg.norm(AX_out - BX_out * theta_out[None, :], axis=0) / xn
    Ax = P.A @ X_out
    Bx = X_out if P.B is None else P.B @ X_out
    true_res = np.linalg.norm(Ax - Bx * theta_out[None, :], axis=0) / xn
    return Result(theta_out, X_out, res_out, true_res, res_out <= thr,
                  cycles, P.nA, P.nB, precs, normA, history)


# ---------------------------------------------------------------------------
# preconditioners of the oracle (each builds the operator r -> M r)
# ---------------------------------------------------------------------------

def jacobi(A):
    """M = diag(A)^{-1}."""
    d = sp.csr_matrix(A).diagonal().astype(np.float64)
    dinv = 1.0 / d
    return lambda r: dinv * r


def factorized(G):
    """M = G^T G for a sparse lower-triangular factor G (FSAI / learned)."""
    G = sp.csr_matrix(G)
    GT = sp.csr_matrix(G.T)
    return lambda r: GT @ (G @ r)

"""Plain FP64 CPU oracle of block TRPL+K.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import this module.  It shares no code with the HIP library; it reuses the
TRPL+K oracle's products, Gram-Schmidt and result type (oracle/trplk.py).

The paper ends its generalized-problem experiments (Sec. 5.5) by noting that
a block TRPL+K is possible and leaving it to future work; it gives no
algorithm.  This module writes out the block form the GPU implements, as
readings of Algorithm 1 (each listed in the design notes of the repository):

B1  block size s >= 1; each cycle targets the s lowest not yet converged Ritz
    pairs t, ..., t + s - 1 (fewer when the restart block holds fewer), each
    with its own shift rho_j = theta_{t+j};
B2  the first inner block is W = M R, R(:, j) = A x_{t+j} - theta_{t+j} B x_{t+j}
    (Alg. 1's u1 = C x_t for every target);
B3  the inner loop appends blocks: every column of W is B-orthogonalised
    against the locked set, the basis and the columns of its own block
    already appended (classical Gram-Schmidt applied twice, as R3), dropped
    under the breakdown rule of R7, and appended with its product A g; the
    next block is W(:, j) = M (A g_j - rho_j B g_j) over the appended columns
    g_j of the block (the block analogue of eq. (3.1)); the loop ends when
    the basis holds m - |X_prev| vectors (the last block is cut to fit, R6)
    or when every column of a block breaks down;
B4  T gets one column per appended vector, T(:, new) = U^T A g (eq. (3.1));
B5  +K, Rayleigh-Ritz, restart, convergence test and locking are those of
    TRPL+K unchanged (oracle/trplk.py, R6-R11).
With s = 1 every step is the TRPL+K oracle's step, in the same order.
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np

from .trplk import (BREAKDOWN_TOL, PLUSK_DROP_TOL, Result, _Pencil, b_cgs2, matrix_norm)


def solve(A, B, p: int, m: int, k: int, l: int, s: int, tol: float, X0: np.ndarray,
          apply_M: Optional[Callable[[np.ndarray], np.ndarray]] = None,
          norm: str = "inf", locking: str = "auto", max_cycles: int = 5000,
          keep_history: bool = False, trace=None) -> Result:
    """Block TRPL+K for the p smallest eigenpairs of (A, B) (B None: B = I).

    The arguments are those of oracle.trplk.solve plus the block size s.
    trace(cycle, U, AU, BU, T, kact, Q, info) is called before each
    Rayleigh-Ritz; info carries the shifts, the targets and the block sizes
    of the cycle (tests only).
    """
    if s < 1:
        raise ValueError("block size s must be >= 1")
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

    Q = np.zeros((n, 0))
    AQ = np.zeros((n, 0))
    BQ = np.zeros((n, 0))

    # --- start: B-orthonormalise X0 and Rayleigh-Ritz on span(X0) (Alg. 1) ---
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
    theta_lock = np.zeros(0)
    kact = k
    res = np.full(k, np.inf)

    for cycle in range(1, max_cycles + 1):
        cycles = cycle
        # B1: the targets of this cycle and their shifts
        nt = max(1, min(s, kact - t))
        tg = list(range(t, t + nt))
        rho = [float(theta[j]) for j in tg]
        # B2: first block, the preconditioned residuals of the targets
        W = np.column_stack([M(AX[:, j] - rho[i] * BX[:, j]) for i, j in enumerate(tg)])
        precs += nt
        U = np.zeros((n, m))
        AU = np.zeros((n, m))
        BU = np.zeros((n, m))
        U[:, :kact], AU[:, :kact], BU[:, :kact] = X, AX, BX
        T = np.zeros((m, m))
        T[np.arange(kact), np.arange(kact)] = theta[:kact]
        nb = kact
        room = m - Xprev.shape[1]
        blocks = []

        def project(v):
            Wb = np.hstack([Q, U[:, :nb]])
            BWb = np.hstack([BQ, BU[:, :nb]])
            return b_cgs2(v, Wb, BWb)

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
            col = U[:, :nb + 1].T @ z           # B4 (eq. (3.1))
            T[:nb + 1, nb] = col
            T[nb, :nb + 1] = col
            nb += 1
            return g, z, Bw / beta

        # --- B3: the inner loop, one block at a time; column j of a block
        # carries the shift of the target it descends from ---
        shift = list(rho)
        while nb < room and W.shape[1] > 0:
            take = min(W.shape[1], room - nb)
            nxt, nxt_shift = [], []
            for j in range(take):
                w, h1 = project(W[:, j])
                out = append(w, h1, BREAKDOWN_TOL)
                if out is None:
                    continue
                g, z, Bg = out
                if nb < room:
                    nxt.append(M(z - shift[j] * Bg))
                    nxt_shift.append(shift[j])
                    precs += 1
            blocks.append(take)
            W = np.column_stack(nxt) if nxt else np.zeros((n, 0))
            shift = nxt_shift
        # --- +K: previous Ritz vectors after the Krylov blocks (Sec. 3) ---
        for c in range(Xprev.shape[1]):
            w, h1 = project(Xprev[:, c])
            append(w, h1, PLUSK_DROP_TOL)
        want = (p - Q.shape[1]) if hard else p
        Xprev_new = X[:, t:min(t + l, want)].copy()
        # --- Rayleigh-Ritz on T (Alg. 1) ---
        Tb = T[:nb, :nb]
        if trace is not None:
            trace(cycle, U[:, :nb], AU[:, :nb], BU[:, :nb], Tb, kact, Q,
                  {"rho": rho, "t": t, "targets": tg, "blocks": blocks})
        theta_all, Yall = np.linalg.eigh(Tb)
        kk = min(k, nb)
        Yk = Yall[:, :kk]
        X = U[:, :nb] @ Yk
        AX = AU[:, :nb] @ Yk
        BX = BU[:, :nb] @ Yk
        theta = theta_all[:kk].copy()
        xn = np.linalg.norm(X, axis=0)
        res = np.linalg.norm(AX - BX * theta[None, :], axis=0) / xn
        # --- convergence test and target advance (Alg. 1, R8, R11) ---
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
                break

    if hard:
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

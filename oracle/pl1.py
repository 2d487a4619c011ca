"""Plain FP64 CPU oracle of PL+1.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import this module.  It shares no code with the HIP library.

PL+1 is the preconditioned Lanczos+1 method of Sec. 4.2 (Algorithm 2) of
Wu, Xue, Stathopoulos, arXiv 1711.10128, for the smallest eigenpair of
A v = lambda B v.  Each outer step k builds a B-orthonormal basis G_k of the
preconditioned Krylov space M K_m((A - rho_k B) M, r_k), takes the lowest
Ritz pair of the pencil projected on Q_k = [x_k, G_k, p_{k-1}], forms the
next iterate from it, and keeps one search direction p_k.  Two choices of
p_k are written out: the one of Algorithm 2 (g_k made conjugate to p_{k-1}
with respect to A - rho_{k-1} B) and the one the paper calls common in
practice (g_k + p_{k-1} w(m+2), the combination the Ritz vector itself uses).

Readings where the passage is silent or garbled:

P1  G_k spans M K_m((A - rho_k B) M, r_k) alone: its vectors are
    B-orthonormalised among themselves (classical Gram-Schmidt applied
    twice) but not against x_k or p_{k-1}; they are generated as
    v_1 = M r_k, v_{j+1} = M (A - rho_k B) g_j, which spans the same space
    as the powers the passage lists;
P2  the projected problem is the generalized one the passage writes,
    Q^T A Q w = rho Q^T B Q w (Q is not B-orthonormal); when Q^T B Q is
    numerically singular (p_{k-1} inside span{x_k, G_k}) p_{k-1} is left out;
P3  step 5 calls the new Ritz value rho_k; it is rho_{k+1} = rho(x_{k+1}) of
    step 6 (the Ritz vector's Rayleigh quotient is the Ritz value).  The
    shift of step 7, rho_{k-1}, is rho(x_{k-1}), the Rayleigh quotient of
    the iterate before x_k, as in the near-conjugacy lemma that follows;
P4  the stopping test is the TRPL+K one, ||A x - rho B x||_2 / ||x||_2 <=
    tol * ||A|| (||A||_inf by default), checked before each outer step;
P5  the practical search direction g_k + p_{k-1} w(m+2) is B-normalised
    like the one of step 7 (a scale does not change the spanned space);
P6  the Krylov block stops early when a new vector's B-norm squared is at
    most (1e-14)^2 (|h1|^2 + beta^2), the TRPL+K breakdown rule.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

from .trplk import BREAKDOWN_TOL, _Pencil, b_cgs2, matrix_norm


@dataclasses.dataclass
class PL1Result:
    theta: float            # the Ritz value
    x: np.ndarray           # (n,) B-normalised Ritz vector
    res: float              # ||A x - theta B x|| / ||x||
    converged: bool
    cycles: int             # outer steps taken
    matvecs: int            # products with A
    normA: float
    history: list           # per step: dict(rho, res, and with keep_history the vectors)


def solve(A, B, m: int, tol: float, x0: np.ndarray,
          apply_M: Optional[Callable[[np.ndarray], np.ndarray]] = None,
          variant: str = "conjugate", norm: str = "inf", max_cycles: int = 5000,
          keep_history: bool = False) -> PL1Result:
    """PL+1 for the smallest eigenpair of (A, B) (B None means B = I).

    m  dimension of the preconditioned Krylov block G_k, tol  stopping
    tolerance relative to ||A||, x0 (n,) start vector, apply_M the
    preconditioner (None = identity), variant 'conjugate' (Algorithm 2,
    step 7) or 'practical' (p_k = g_k + p_{k-1} w(m+2)).
    """
    if variant not in ("conjugate", "practical"):
        raise ValueError(variant)
    if m < 1:
        raise ValueError("m must be >= 1")
    P = _Pencil(A, B)
    M = apply_M if apply_M is not None else (lambda r: r.copy())
    normA = matrix_norm(P.A, norm)
    thr = tol * normA

    # step 2: x_0 B-normalised, rho_0, r_0 (A x and B x kept alongside x)
    x = np.asarray(x0, dtype=np.float64).copy()
    Bx = P.Bv(x)
    s = np.sqrt(x @ Bx)
    x, Bx = x / s, Bx / s
    Ax = P.Av(x)
    rho = float(x @ Ax)
    p = Ap = Bp = None          # p_{k-1} and its products
    rho_prev = None             # rho(x_{k-1})
    history = []
    k = 0
    res = np.linalg.norm(Ax - rho * Bx) / np.linalg.norm(x)
    while k < max_cycles and res > thr:
        r = Ax - rho * Bx
        # step 4: G_k, a B-orthonormal basis of M K_m((A - rho B) M, r)   (P1, P6)
        G = np.zeros((x.shape[0], 0))
        AG = np.zeros_like(G)
        BG = np.zeros_like(G)
        v = M(r)
        for _ in range(m):
            w, h1 = b_cgs2(v, G, BG)
            Bw = P.Bv(w)
            beta2 = float(w @ Bw)
            if not beta2 > (BREAKDOWN_TOL ** 2) * (float(h1 @ h1) + beta2):
                break
            beta = np.sqrt(beta2)
            g, Bg = w / beta, Bw / beta
            Ag = P.Av(g)
            G = np.column_stack([G, g])
            AG = np.column_stack([AG, Ag])
            BG = np.column_stack([BG, Bg])
            v = M(Ag - rho * Bg)
        ng = G.shape[1]
        # step 5: Rayleigh-Ritz on Q = [x, G, p]   (P2)
        Q, AQ, BQ = np.column_stack([x, G]), np.column_stack([Ax, AG]), np.column_stack([Bx, BG])
        use_p = p is not None
        if use_p:
            Q2 = np.column_stack([Q, p])
            S2 = Q2.T @ np.column_stack([BQ, Bp])
            S2 = (S2 + S2.T) / 2
            ev = np.linalg.eigvalsh(S2)
            if ev[0] > 1e-12 * ev[-1]:
                Q, AQ, BQ = Q2, np.column_stack([AQ, Ap]), np.column_stack([BQ, Bp])
            else:
                use_p = False
        TA = Q.T @ AQ
        TA = (TA + TA.T) / 2
        TB = Q.T @ BQ
        TB = (TB + TB.T) / 2
        vals, W = la.eigh(TA, TB)
        wv = W[:, 0]
        # step 6: g_k = G w(2:m+1), x_{k+1} = x w(1) + g_k (+ p w(m+2)), normalised
        zg = np.zeros_like(wv)
        zg[1:1 + ng] = wv[1:1 + ng]
        xt, Axt, Bxt = Q @ wv, AQ @ wv, BQ @ wv
        sx = np.sqrt(xt @ Bxt)
        x_new, Ax_new, Bx_new = xt / sx, Axt / sx, Bxt / sx
        rho_new = float(x_new @ Ax_new) / float(x_new @ Bx_new)
        # step 7: the search direction p_k   (P3, P5)
        if variant == "conjugate" and use_p:
            # (p_{k-1} and g_k in the coordinates of Q: e_last and zg)
            ep = np.zeros_like(wv)
            ep[-1] = 1.0
            K = TA - rho_prev * TB
            c = (ep @ K @ zg) / (ep @ K @ ep)
            zp = zg - c * ep
        elif variant == "practical" and use_p:
            zp = zg.copy()
            zp[-1] = wv[-1]
        else:
            zp = zg
        pt, Apt, Bpt = Q @ zp, AQ @ zp, BQ @ zp
        sp_ = np.sqrt(pt @ Bpt)
        entry = {"rho": rho_new, "ng": ng, "used_p": use_p}
        if keep_history:
            entry.update({"p_prev": None if p is None else p.copy(), "rho_prev_shift": rho_prev,
                          "x": x.copy(), "x_new": x_new.copy()})
        rho_prev = rho
        p, Ap, Bp = pt / sp_, Apt / sp_, Bpt / sp_
        if keep_history:
            entry["p"] = p.copy()
        x, Ax, Bx, rho = x_new, Ax_new, Bx_new, rho_new
        res = np.linalg.norm(Ax - rho * Bx) / np.linalg.norm(x)
        entry["res"] = res
        history.append(entry)
        k += 1
    # a fresh product for the returned residual
    true_res = np.linalg.norm(P.A @ x - rho * (x if P.B is None else P.B @ x)) / np.linalg.norm(x)
    return PL1Result(theta=rho, x=x, res=float(true_res), converged=bool(true_res <= thr),
                     cycles=k, matvecs=P.nA, normA=normA, history=history)

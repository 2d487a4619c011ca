"""Global quasi-optimality of TRPL+K with one inner step.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may use
this module.  FP64, NumPy only; it calls the PL+1 oracle (oracle/pl1.py) for
the restarted iterates and writes the unrestarted method out here.

Sec. 4.3 defines the global quasi-optimality of an iterate x_k lying in a
nested subspace U_k: with y_k* the minimiser of the Rayleigh quotient rho
over U_k and lambda_1 the smallest eigenvalue, the ratio

    (rho(x_k) - rho(y_k*)) / (rho(x_k) - lambda_1)

tends to 0 as the angle theta_0 between the start vector and the wanted
eigenvector goes to 0.  Sec. 5.1 (Fig. 1) measures it for TRPL+K with a
single inner step and no preconditioner, against the unrestarted method,
for the first iterations and several start angles.

"TRPL+K with one inner iteration" is LOPCG (the paper says so): every outer
step projects on span{x_k, g_k, x_{k-1}} with g_k = M r_k, one Krylov
vector.  With the thick-restart size k = 1 the library's TRPL+K gives its
first cycle two inner vectors (the basis fills to m = 3 before the first +K
vector exists), so the one-inner-step method of the experiment is run as
PL+1 with the practical direction p_k = g_k + p_{k-1} w(m+2) and a Krylov
block of one vector (Sec. 4.2; span{x_{k+1}, p_k} = span{x_{k+1}, x_k}, so
each step searches span{x_k, g_k, x_{k-1}}), here through the PL+1 oracle
(oracle/pl1.py).  With M = I, x_k lies in the Krylov space K_{k+1}(A, x_0)
and the spaces nest, so the unrestarted method's space is
U_k = K_{k+1}(A, x_0) and rho(y_k*) its smallest Ritz value, computed here
by Lanczos with full re-orthogonalisation (classical Gram-Schmidt twice),
the textbook unrestarted method.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import pl1


def start_vector(v1: np.ndarray, theta0: float, rng: np.random.Generator) -> np.ndarray:
    """x_0 = v_1 cos(theta0) + f sin(theta0), f a random unit vector
    orthogonal to the unit eigenvector v_1: the angle between x_0 and v_1 is
    exactly theta0."""
    v1 = v1 / np.linalg.norm(v1)
    f = rng.standard_normal(v1.shape[0])
    f -= (f @ v1) * v1
    f -= (f @ v1) * v1
    f /= np.linalg.norm(f)
    return math.cos(theta0) * v1 + math.sin(theta0) * f


def krylov_ritz_min(A, x0: np.ndarray, dmax: int) -> np.ndarray:
    """Smallest Ritz value of A over K_d(A, x0) for d = 1 .. dmax: Lanczos
    with full re-orthogonalisation (each new vector A q_j made orthogonal to
    all previous ones by classical Gram-Schmidt applied twice), then the
    eigenvalues of Q^T A Q."""
    A = sp.csr_matrix(A)
    n = x0.shape[0]
    Q = np.zeros((n, dmax))
    AQ = np.zeros((n, dmax))
    out = np.full(dmax, np.nan)
    q = x0 / np.linalg.norm(x0)
    for d in range(dmax):
        Q[:, d] = q
        AQ[:, d] = A @ q
        H = Q[:, :d + 1].T @ AQ[:, :d + 1]
        out[d] = np.linalg.eigvalsh(0.5 * (H + H.T))[0]
        w = AQ[:, d].copy()
        for _ in range(2):
            w -= Q[:, :d + 1] @ (Q[:, :d + 1].T @ w)
        nw = np.linalg.norm(w)
        if not nw > 1e-14 * np.linalg.norm(AQ[:, d]):
            out[d + 1:] = out[d]   # invariant subspace: the space stops growing
            break
        q = w / nw
    return out


def one_inner_step(A, x0: np.ndarray, cycles: int) -> np.ndarray:
    """rho(x_k), k = 1 .. cycles, of the one-inner-step method (PL+1 with
    the practical direction and a one-vector Krylov block, M = I), run for
    exactly `cycles` outer steps."""
    r = pl1.solve(A, None, 1, 1e-300, x0, apply_M=None, variant="practical",
                  max_cycles=cycles, keep_history=True)
    return np.array([h["rho"] for h in r.history])


def ratio(rho_x: np.ndarray, rho_star: np.ndarray, lam1: float) -> np.ndarray:
    """The quasi-optimality ratio of Sec. 4.3 per iteration."""
    return (rho_x - rho_star) / (rho_x - lam1)


def quasi_optimality(A, x0: np.ndarray, lam1: float, cycles: int, rho_x=None):
    """Ratio for iterations k = 1 .. cycles.  rho_x: the one-inner-step
    iterates' Rayleigh quotients (default: the oracle's); U_k = K_{k+1}(A, x0)."""
    if rho_x is None:
        rho_x = one_inner_step(A, x0, cycles)
    rho_star = krylov_ritz_min(A, x0, cycles + 1)[1:cycles + 1]
    return ratio(np.asarray(rho_x[:cycles]), rho_star, lam1), rho_x, rho_star

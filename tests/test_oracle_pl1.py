"""Pins of the PL+1 oracle (Sec. 4.2, Algorithm 2) against what the paper and
the mathematics fix: closed-form and dense eigenvalues, the exact
conjugacy that step 7 builds in, the span identity of the practical search
direction, monotone Rayleigh quotients, the Rayleigh-Ritz minimum over the
projection space, and invariance under scaling of the preconditioner.
CPU only."""
import math

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import pl1 as PL
from oracle import trplk as O
from workloads import fem3d, lap2d, powerlaw


def _x0(n, seed=12):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def test_pl1_closed_form_both_variants():
    """2-D Dirichlet Laplacian on 24 x 24: lambda_1 = 8 sin^2(pi / 50); with
    B = I the residual bounds the eigenvalue error."""
    A = lap2d(24).to_scipy()
    lam1 = 8.0 * math.sin(math.pi / 50.0) ** 2
    for variant in ("conjugate", "practical"):
        r = PL.solve(A, None, 6, 1e-9, _x0(A.shape[0]), apply_M=O.jacobi(A), variant=variant)
        assert r.converged
        assert abs(r.theta - lam1) <= r.res * 1.0001
        assert abs(r.theta - lam1) <= 1e-9 * r.normA
        # MV = 1 + m per step (the block never breaks down here)
        assert r.matvecs == 1 + 6 * r.cycles


def test_pl1_generalized_dense():
    """Q1 FEM pencil with a lognormal coefficient: the smallest eigenvalue of
    the dense pencil (LAPACK)."""
    A, B = fem3d(6, 0.5, 12)
    A, B = A.to_scipy(), B.to_scipy()
    lam = sl.eigh(A.toarray(), B.toarray(), eigvals_only=True)[0]
    for variant in ("conjugate", "practical"):
        r = PL.solve(A, B, 5, 1e-11, _x0(A.shape[0]), apply_M=O.jacobi(A), variant=variant)
        assert r.converged
        assert abs(r.theta - lam) <= 1e-8 * abs(lam)


def test_step7_search_directions_are_exactly_conjugate():
    """p_k^T (A - rho(x_{k-1}) B) p_{k-1} = 0 for the direction of step 7,
    with rho(x_{k-1}) recomputed here from the stored iterate; the practical
    direction does not have the property."""
    A = powerlaw(400, seed=13).to_scipy()
    out = {}
    for variant in ("conjugate", "practical"):
        r = PL.solve(A, None, 3, 1e-10, _x0(A.shape[0]), apply_M=O.jacobi(A), variant=variant,
                     keep_history=True)
        assert r.converged and r.cycles >= 4
        worst = 0.0
        prev_x = None
        for h in r.history:
            if h["used_p"] and prev_x is not None:
                rho_prev = float(prev_x @ (A @ prev_x)) / float(prev_x @ prev_x)
                p, q = h["p"], h["p_prev"]
                val = abs(p @ (A @ q) - rho_prev * (p @ q))
                worst = max(worst, val / r.normA)
            prev_x = h["x"]
        out[variant] = worst
    assert out["conjugate"] <= 1e-12
    assert out["practical"] > 1e-6


def test_practical_direction_spans_previous_iterate():
    """With p_k = g_k + p_{k-1} w(m+2), span{x_{k+1}, p_k} = span{x_{k+1}, x_k}:
    the practical PL+1 keeps the previous Ritz vector, as TRPL+K with l = 1."""
    A = lap2d(18).to_scipy()
    r = PL.solve(A, None, 4, 1e-10, _x0(A.shape[0]), apply_M=O.jacobi(A), variant="practical",
                 keep_history=True)
    assert r.cycles >= 3
    for h in r.history[1:]:
        S1 = np.linalg.qr(np.column_stack([h["x_new"], h["p"]]))[0]
        S2 = np.linalg.qr(np.column_stack([h["x_new"], h["x"]]))[0]
        sv = np.linalg.svd(S1.T @ S2, compute_uv=False)
        assert sv.min() >= 1.0 - 1e-10


def test_rayleigh_quotients_decrease_and_match_a_dense_projection():
    """rho_{k+1} <= rho_k (x_k lies in the projection space) and the first
    step's Ritz value is the minimum of the Rayleigh quotient over
    span{x_0, M r_0, ...}, computed here with an orthonormal basis from QR."""
    A = powerlaw(300, seed=14).to_scipy()
    x0 = _x0(A.shape[0])
    r = PL.solve(A, None, 4, 1e-10, x0, apply_M=O.jacobi(A), variant="conjugate",
                 keep_history=True)
    rhos = [float(x0 @ (A @ x0)) / float(x0 @ x0)] + [h["rho"] for h in r.history]
    assert all(b <= a + 1e-13 * abs(a) for a, b in zip(rhos, rhos[1:]))
    d = A.diagonal()
    x = x0 / np.linalg.norm(x0)
    rho = float(x @ (A @ x))
    vecs = [x]
    v = (A @ x - rho * x) / d
    for _ in range(4):
        vecs.append(v)
        v = (A @ v - rho * v) / d
    Qo = np.linalg.qr(np.column_stack(vecs))[0]
    lam_min = np.linalg.eigvalsh(Qo.T @ (A @ Qo))[0]
    assert abs(r.history[0]["rho"] - lam_min) <= 1e-12 * abs(lam_min)


def test_preconditioner_scale_does_not_change_the_iterates():
    """M and 3 M span the same Krylov spaces, so the Ritz values agree."""
    A = powerlaw(300, seed=15).to_scipy()
    d = A.diagonal()
    x0 = _x0(A.shape[0])
    r1 = PL.solve(A, None, 3, 1e-10, x0, apply_M=lambda v: v / d, keep_history=True)
    r3 = PL.solve(A, None, 3, 1e-10, x0, apply_M=lambda v: 3.0 * v / d, keep_history=True)
    assert r1.cycles == r3.cycles
    for a, b in zip(r1.history, r3.history):
        assert abs(a["rho"] - b["rho"]) <= 1e-12 * abs(a["rho"])


def _mutant(old, new):
    """The PL+1 oracle with one planted change (source replaced once)."""
    import os
    import sys
    import types
    src = open(os.path.join(os.path.dirname(PL.__file__), "pl1.py")).read()
    assert old in src
    src = src.replace("from .trplk import", "from oracle.trplk import")
    mod = types.ModuleType("oracle_pl1_mutant")
    sys.modules["oracle_pl1_mutant"] = mod
    try:
        exec(compile(src.replace(old, new, 1), "oracle_pl1_mutant", "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle_pl1_mutant"]
    return mod


def test_mutant_wrong_conjugation_shift_fails_the_conjugacy_pin():
    """Step 7 with the current shift rho(x_k) instead of rho(x_{k-1})."""
    Pm = _mutant("K = TA - rho_prev * TB", "K = TA - rho * TB")
    A = powerlaw(400, seed=13).to_scipy()
    r = Pm.solve(A, None, 3, 1e-10, _x0(A.shape[0]), apply_M=O.jacobi(A), keep_history=True)
    worst, prev_x = 0.0, None
    for h in r.history:
        if h["used_p"] and prev_x is not None:
            rho_prev = float(prev_x @ (A @ prev_x)) / float(prev_x @ prev_x)
            worst = max(worst, abs(h["p"] @ (A @ h["p_prev"]) - rho_prev * (h["p"] @ h["p_prev"])))
        prev_x = h["x"]
    assert worst / r.normA > 1e-10

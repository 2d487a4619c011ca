"""Pins of the quasi-optimality experiment (Sec. 4.3 definition, Sec. 5.1
Fig. 1): the unrestarted method's Rayleigh quotients and the ratio, on the
64 x 64 Laplacian whose lowest eigenpair is known in closed form."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import quasiopt as Q
from workloads import lap2d

N = 64


def lowest_pair():
    """v1(i, j) = sin(i pi/(N+1)) sin(j pi/(N+1)), lambda1 = 8 sin^2(pi/(2(N+1)))."""
    s = np.sin(np.arange(1, N + 1) * np.pi / (N + 1))
    return np.outer(s, s).ravel(), 8 * math.sin(math.pi / (2 * (N + 1))) ** 2


def test_closed_form_pair_and_start_angle():
    A = lap2d(N).to_scipy()
    v1, lam1 = lowest_pair()
    assert np.linalg.norm(A @ v1 - lam1 * v1) <= 1e-14 * np.linalg.norm(v1)
    for th in (0.5, 1e-3):
        x0 = Q.start_vector(v1, th, np.random.default_rng(1))
        c = abs(x0 @ v1) / (np.linalg.norm(x0) * np.linalg.norm(v1))
        assert abs(math.acos(min(c, 1.0)) - th) < 1e-7
    # rho(x0) - lambda1 = sin^2(theta0) (rho(f) - lambda1), f the orthogonal part
    x0 = Q.start_vector(v1, 0.3, np.random.default_rng(1))
    f = (x0 - math.cos(0.3) * v1 / np.linalg.norm(v1)) / math.sin(0.3)
    rho = lambda z: (z @ (A @ z)) / (z @ z)
    assert abs((rho(x0) - lam1) - math.sin(0.3) ** 2 * (rho(f) - lam1)) < 1e-13


def test_unrestarted_krylov_minimum():
    """min over K_d(A, x0): d = 1 gives rho(x0); nonincreasing in d; equal to
    the smallest eigenvalue of a dense orthonormal basis of the same space;
    lambda1 once the space is invariant (a start vector in a 5-dimensional
    invariant subspace)."""
    A = lap2d(12).to_scipy()
    n = A.shape[0]
    x0 = np.random.default_rng(4).standard_normal(n)
    rs = Q.krylov_ritz_min(A, x0, 12)
    assert abs(rs[0] - x0 @ (A @ x0) / (x0 @ x0)) < 1e-14
    assert np.all(np.diff(rs) <= 1e-14)
    K = np.empty((n, 6))
    K[:, 0] = x0 / np.linalg.norm(x0)
    for j in range(1, 6):
        K[:, j] = A @ K[:, j - 1]
        K[:, j] /= np.linalg.norm(K[:, j])
    Qm, _ = np.linalg.qr(K)
    assert abs(np.linalg.eigvalsh(Qm.T @ (A @ Qm))[0] - rs[5]) < 1e-12
    D = sp.diags(np.arange(1.0, 21.0))
    y = np.zeros(20)
    y[:5] = 1.0
    rs = Q.krylov_ritz_min(D, y, 9)
    assert abs(rs[4] - 1.0) < 1e-13 and np.all(np.abs(rs[4:] - 1.0) < 1e-13)


def test_ratio_definition_by_hand():
    """(rho(x_k) - rho(y*)) / (rho(x_k) - lambda1): 0 when x_k is the global
    minimiser, 1 when the global minimiser is exact, 1/2 halfway."""
    assert Q.ratio(np.array([3.0]), np.array([2.0]), 1.0)[0] == 0.5
    assert Q.ratio(np.array([3.0]), np.array([3.0]), 1.0)[0] == 0.0
    assert Q.ratio(np.array([3.0]), np.array([1.0]), 1.0)[0] == 1.0


def test_first_iterates_are_global_minimisers():
    """x1 minimises rho over span{x0, r0} = K_2 and x2 over
    span{x1, r1, x0} = K_3: the ratio is zero there (rounding aside)."""
    A = lap2d(N).to_scipy()
    v1, lam1 = lowest_pair()
    x0 = Q.start_vector(v1, 0.5, np.random.default_rng(3))
    r, rx, rs = Q.quasi_optimality(A, x0, lam1, 4)
    assert np.all(np.abs(r[:2]) < 1e-11)
    # rho(y*) <= rho(x_k) always (x_k lies in U_k): the ratio is not negative
    assert np.all(r >= -1e-11) and np.all(r < 1.0)


def test_ratio_falls_with_the_start_angle():
    """Fig. 1: at each iteration the ratio decreases as the start vector's
    angle to v1 shrinks (here by far more than 10x per step of theta0)."""
    A = lap2d(N).to_scipy()
    v1, lam1 = lowest_pair()
    rows = []
    for th in (0.5, 0.1, 0.02):
        x0 = Q.start_vector(v1, th, np.random.default_rng(3))
        rows.append(Q.quasi_optimality(A, x0, lam1, 20)[0])
    # iterations 3, 5, 10, 20: theta0 = 0.5 -> 0.1 lowers the ratio about
    # sin^2 ratio-fold (25x; measured ~1000x); at theta0 = 0.02 the numerator
    # rho(x_k) - rho(y*) is down to ~1e-16, the rounding of rho itself, so
    # there only its size is checked
    for k in (2, 4, 9, 19):
        assert rows[0][k] > 100 * rows[1][k] > 0, [r[k] for r in rows]
    for k in (2, 4, 9):
        assert abs(rows[2][k]) < 2e-9 < rows[1][k], [r[k] for r in rows]


@pytest.mark.parametrize("old,new", [
    ("f -= (f @ v1) * v1\n    f -= (f @ v1) * v1", "f -= 0.5 * (f @ v1) * v1"),   # f not orthogonal
    ("for _ in range(2):\n            w -= Q", "for _ in range(0):\n            w -= Q"),  # no orth
    ("return (rho_x - rho_star) / (rho_x - lam1)", "return (rho_x - rho_star) / (rho_star - lam1 + 1e-3)"),
])
def test_mutants_fail_pins(old, new):
    import types
    src = open(Q.__file__).read()
    assert old in src
    m = types.ModuleType("oracle.quasiopt_mutant")
    m.__package__ = "oracle"
    exec(compile(src.replace(old, new), "quasiopt_mutant", "exec"), m.__dict__)
    g = globals()
    saved = g["Q"]
    g["Q"] = m
    try:
        failed = False
        for t in (test_closed_form_pair_and_start_angle, test_unrestarted_krylov_minimum,
                  test_ratio_definition_by_hand,
                  test_first_iterates_are_global_minimisers, test_ratio_falls_with_the_start_angle):
            try:
                t()
            except (AssertionError, np.linalg.LinAlgError, ValueError):
                failed = True
        assert failed
    finally:
        g["Q"] = saved

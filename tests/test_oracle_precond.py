"""Pins of the oracle's factorized preconditioners (FSAI and the learned factor)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import precond as PC
from oracle import trplk as O
from workloads import make, start_block, lap3d, fem3d, powerlaw


def _fsai_defining(A, G, cap=None):
    A = sp.csr_matrix(A)
    GA = (G @ A).tocsr()
    pats = PC.fsai_pattern(A, cap)
    worst_off, worst_diag = 0.0, 0.0
    GAGt = (G @ A @ G.T).diagonal()
    for i, P in enumerate(pats):
        row = GA[i].toarray().ravel()
        worst_off = max(worst_off, np.max(np.abs(row[P[:-1]])) if P.shape[0] > 1 else 0.0)
    worst_diag = np.max(np.abs(GAGt - 1.0))
    return worst_off, worst_diag


@pytest.mark.parametrize("which", ["lap3d", "fem3d", "powerlaw"])
def test_fsai_defining_equations(which):
    """(G A)_{ij} = 0 on the pattern off the diagonal and (G A G^T)_{ii} = 1."""
    if which == "lap3d":
        A = lap3d(8, 0.05).to_scipy()
        cap = None
    elif which == "fem3d":
        A = fem3d(7, 0.5)[0].to_scipy()
        cap = None
    else:
        A = powerlaw(800).to_scipy()
        cap = 8
    G = PC.fsai(A, cap)
    off, dg = _fsai_defining(A, G, cap)
    scale = np.max(np.abs(A.data))
    assert off < 1e-12 * scale * np.max(np.abs(G.data))
    assert dg < 1e-12
    # lower triangular with a positive diagonal
    assert sp.triu(G, 1).nnz == 0 and np.all(G.diagonal() > 0)


def test_fsai_full_pattern_is_inverse_cholesky():
    """With the full lower pattern FSAI is the exact inverse Cholesky factor:
    G^T G = A^{-1} (textbook special case)."""
    rng = np.random.default_rng(5)
    R = rng.standard_normal((30, 30))
    A = R @ R.T + 30 * np.eye(30)
    G = PC.fsai(sp.csr_matrix(A))
    assert np.max(np.abs((G.T @ G).toarray() - np.linalg.inv(A))) < 1e-13
    # and for a diagonal matrix it is D^{-1/2}
    D = sp.diags(rng.uniform(1, 3, 10)).tocsr()
    assert np.allclose(PC.fsai(D).diagonal(), 1 / np.sqrt(D.diagonal()), rtol=1e-15)


def test_fsai_solve_small_dense():
    """A full solve with the FSAI preconditioner reaches the dense eigenvalues
    and needs fewer products than Jacobi on the FEM stiffness."""
    P = make("fem3d", "small", Ne=9, sigma=0.5, p=6, m=20, k=10)
    A, B = P.A.to_scipy(), P.B.to_scipy()
    X0 = start_block(A.shape[0], 10, 12)
    rj = O.solve(A, B, 6, 20, 10, 1, 1e-8, X0, apply_M=O.jacobi(A))
    rf = O.solve(A, B, 6, 20, 10, 1, 1e-8, X0, apply_M=O.factorized(PC.fsai(A)))
    import scipy.linalg as sl
    ev = sl.eigh(A.toarray(), B.toarray(), eigvals_only=True)[:6]
    assert np.all(np.abs(rf.theta - ev) <= 1e-10 * ev)
    assert rf.matvecs < rj.matvecs


def test_row_features_by_hand():
    A = sp.csr_matrix(np.array([[4.0, -1.0, 0.0, -2.0],
                                [-1.0, 3.0, 0.0, 0.0],
                                [0.0, 0.0, 5.0, 0.0],
                                [-2.0, 0.0, 0.0, 6.0]]))
    raw = np.array([
        [2, 4, 3, 1.5, 1, 2, 0.5, 4 / 3],
        [1, 3, 1, 1, 1, 1, 0, 3],
        [0, 5, 0, 0, 0, 0, 0, 0],
        [1, 6, 2, 2, 2, 2, 0, 3],
    ], dtype=float)
    z = (raw - raw.mean(0)) / raw.std(0)
    assert np.allclose(PC.row_features(A), z, atol=1e-14)


def test_learned_zero_output_is_jacobi():
    """A zero output layer gives G = D^{-1/2}, hence M = D^{-1}: the solve is
    the Jacobi solve."""
    P = make("powerlaw", "small", n=1200, p=4, m=16, k=8)
    A = P.A.to_scipy()
    params = PC.init_params(seed=1, zero_last=True)
    o, _ = PC.mlp_forward(params, PC.mlp_inputs(A))
    G = PC.assemble_G(A, o)
    D = A.diagonal()
    assert np.allclose((G.T @ G).toarray(), np.diag(1 / D), rtol=1e-15, atol=0)
    X0 = start_block(A.shape[0], 8, 12)
    rj = O.solve(A, None, 4, 16, 8, 1, 1e-8, X0, apply_M=O.jacobi(A))
    rl = O.solve(A, None, 4, 16, 8, 1, 1e-8, X0, apply_M=O.factorized(G))
    assert rl.cycles == rj.cycles
    assert np.allclose(rl.theta, rj.theta, rtol=1e-12)


def _pairs(A, S, seed=3):
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((A.shape[0], S))
    return A @ E, E


def test_loss_gradient_G_finite_differences():
    A = powerlaw(200).to_scipy()
    params = PC.init_params(seed=2, zero_last=False)
    o, _ = PC.mlp_forward(params, PC.mlp_inputs(A))
    G = PC.assemble_G(A, o)
    R, E = _pairs(A, 3)
    L0, grad = PC.loss_and_grad_G(G, R, E)
    rng = np.random.default_rng(0)
    for idx in rng.choice(G.nnz, 12, replace=False):
        h = 1e-6 * max(1.0, abs(G.data[idx]))
        Gp, Gm = G.copy(), G.copy()
        Gp.data[idx] += h
        Gm.data[idx] -= h
        fd = (PC.loss_and_grad_G(Gp, R, E)[0] - PC.loss_and_grad_G(Gm, R, E)[0]) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_loss_gradient_params_finite_differences():
    A = powerlaw(150).to_scipy()
    params = PC.init_params(seed=4, zero_last=False)
    params["w2"] *= 0.1
    R, E = _pairs(A, 2)
    x = PC.mlp_inputs(A)
    L0, g, _ = PC.loss_and_grad_params(params, A, R, E, x)
    rng = np.random.default_rng(1)
    checks = [("b2", ())] + [("w2", (int(i),)) for i in rng.choice(PC.NHID, 4, replace=False)]
    checks += [("b1", (int(i),)) for i in rng.choice(PC.NHID, 3, replace=False)]
    checks += [("W1", (int(i), int(j))) for i, j in zip(rng.choice(PC.NHID, 4), rng.choice(PC.NIN, 4))]
    for key, ix in checks:
        h = 1e-6
        pp = {kk: np.array(v, copy=True) for kk, v in params.items()}
        pm = {kk: np.array(v, copy=True) for kk, v in params.items()}
        pp[key][ix] += h
        pm[key][ix] -= h
        fd = (PC.loss_and_grad_params(pp, A, R, E, x)[0]
              - PC.loss_and_grad_params(pm, A, R, E, x)[0]) / (2 * h)
        an = float(np.asarray(g[key])[ix])
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (key, ix, fd, an)


def test_angle_loss_closed_forms():
    """The loss is 0 when M r is parallel to e (any scale) and 1 when they are
    orthogonal; G = c I gives M = c^2 I, so with r = A e the loss is the
    squared sine of the angle between A e and e."""
    n = 6
    I = sp.identity(n, format="csr")
    rng = np.random.default_rng(2)
    E = rng.standard_normal((n, 3))
    L, _ = PC.loss_and_grad_G(3.0 * I, E, E)
    assert abs(L) < 1e-15
    R = np.zeros((n, 1)); R[0, 0] = 1.0
    Eo = np.zeros((n, 1)); Eo[1, 0] = 1.0
    assert abs(PC.loss_and_grad_G(I, R, Eo)[0] - 1.0) < 1e-15
    Ad = np.diag(np.arange(1.0, n + 1))
    e = rng.standard_normal((n, 1))
    r = Ad @ e
    cos2 = float((r[:, 0] @ e[:, 0]) ** 2 / ((r[:, 0] @ r[:, 0]) * (e[:, 0] @ e[:, 0])))
    assert abs(PC.loss_and_grad_G(2.0 * I, r, e)[0] - (1 - cos2)) < 1e-14


def test_adam_training_lowers_loss():
    """A few Adam steps on solver-generated pairs lower the loss below the
    Jacobi starting point."""
    P = make("powerlaw", "small", n=1000, p=4, m=16, k=8)
    A = P.A.to_scipy()
    r = O.solve(A, None, 4, 16, 8, 1, 1e-6, start_block(A.shape[0], 8, 12),
                apply_M=O.jacobi(A), max_cycles=3)
    E = r.X
    R = A @ E
    params = PC.init_params(seed=0, zero_last=True)
    x = PC.mlp_inputs(A)
    L0, g, _ = PC.loss_and_grad_params(params, A, R, E, x)
    st = {}
    for _ in range(30):
        L, g, _ = PC.loss_and_grad_params(params, A, R, E, x)
        PC.adam_step(params, g, st, lr=1e-3)
    L1 = PC.loss_and_grad_params(params, A, R, E, x)[0]
    assert L1 < 0.9 * L0


def test_learned_offdiagonal_scale_by_hand():
    """G[i,j] = -o a_ij / (cbar a_jj sqrt(a_ii)), cbar the mean of
    |a_ij| / sqrt(a_ii a_jj) over the strictly lower entries.  Checked on a
    1-D Laplacian (every coupling 1/2, so the scale is 1/sqrt(a_jj) = 1/sqrt 2)
    and on a 3 x 3 matrix with unequal couplings, worked out by hand."""
    import scipy.sparse as sp
    T1 = sp.diags([-np.ones(4), 2 * np.ones(5), -np.ones(4)], [-1, 0, 1], format="csr")
    assert PC.coupling_scale(T1) == 0.5
    o = np.full(9, 0.3)                      # 5 diagonal + 4 lower entries
    G = PC.assemble_G(T1, o).toarray()
    assert np.isclose(G[1, 0], 0.3 / np.sqrt(2.0), rtol=1e-15)
    assert np.isclose(G[3, 3], np.exp(0.3) / np.sqrt(2.0), rtol=1e-15)
    # a_00 = 9, a_11 = 4, a_22 = 1; a_10 = -3 (coupling 3/6 = 1/2), a_20 = -1
    # (coupling 1/3), a_21 = 0.5 (coupling 1/4): cbar = (1/2 + 1/3 + 1/4)/3 = 13/36
    A = sp.csr_matrix(np.array([[9.0, -3.0, -1.0], [-3.0, 4.0, 0.5], [-1.0, 0.5, 1.0]]))
    assert np.isclose(PC.coupling_scale(A), 13.0 / 36.0, rtol=1e-15)
    G = PC.assemble_G(A, np.array([0.0, 2.0, 0.0, 2.0, 2.0, 0.0])).toarray()
    cb = 13.0 / 36.0
    assert np.isclose(G[1, 0], 2.0 * 3.0 / (cb * 9.0 * 2.0), rtol=1e-15)
    assert np.isclose(G[2, 0], 2.0 * 1.0 / (cb * 9.0 * 1.0), rtol=1e-15)
    assert np.isclose(G[2, 1], 2.0 * -0.5 / (cb * 4.0 * 1.0), rtol=1e-15)
    assert np.isclose(G[0, 0], 1.0 / 3.0, rtol=1e-15)


def test_adam_step_by_hand():
    """One and two Adam steps (Kingma and Ba, Algorithm 1: biased moments
    m_t = b1 m + (1 - b1) g, v_t = b2 v + (1 - b2) g^2, bias corrections
    1 - b^t, update lr * mhat / (sqrt(vhat) + eps)) worked out by hand.

    Step 1 with g = 2: m = 0.2, v = 0.004, mhat = 2, vhat = 4, so the update
    is lr * 2 / (2 + eps).  Step 2 with g = -1: m = 0.18 - 0.1 = 0.08,
    v = 0.003996 + 0.001 = 0.004996, mhat = 0.08 / 0.19, vhat = 0.004996 /
    0.001999.  A missing bias correction or a wrong moment weight changes
    both numbers by far more than the tolerance."""
    lr, eps = 1e-2, 1e-8
    p = {"w": np.array([1.0, -3.0])}
    st = {}
    PC.adam_step(p, {"w": np.array([2.0, 0.5])}, st, lr=lr, eps=eps)
    # the second entry: g = 0.5, mhat = 0.5, vhat = 0.25 -> lr * 0.5 / (0.5 + eps)
    assert np.allclose(p["w"], [1.0 - lr * 2.0 / (2.0 + eps), -3.0 - lr * 0.5 / (0.5 + eps)],
                       rtol=0, atol=1e-15)
    assert st["t"] == 1
    assert np.allclose(st["m_w"], [0.2, 0.05], rtol=1e-15)
    assert np.allclose(st["v_w"], [0.004, 0.00025], rtol=1e-15)
    w1 = p["w"].copy()
    PC.adam_step(p, {"w": np.array([-1.0, 0.5])}, st, lr=lr, eps=eps)
    m2 = 0.9 * 0.2 + 0.1 * -1.0
    v2 = 0.999 * 0.004 + 0.001 * 1.0
    mh, vh = m2 / (1 - 0.9 ** 2), v2 / (1 - 0.999 ** 2)
    assert abs(m2 - 0.08) < 1e-15 and abs(v2 - 0.004996) < 1e-15
    assert abs(p["w"][0] - (w1[0] - lr * mh / (math.sqrt(vh) + eps))) < 1e-15
    # the numbers themselves: mhat = 0.421052..., vhat = 0.004996 / 0.001999 = 2.49925...
    assert abs(mh - 0.08 / 0.19) < 1e-15
    assert abs(vh - 2.4992496) < 1e-7
    # a constant gradient keeps the step at lr (mhat / sqrt(vhat) = 1)
    q = {"w": np.zeros(1)}
    s2 = {}
    for _ in range(5):
        PC.adam_step(q, {"w": np.array([3.0])}, s2, lr=0.1, eps=0.0)
    assert abs(q["w"][0] + 0.5) < 1e-14


@pytest.mark.parametrize("old,new", [
    ("mh = mk / (1 - b1 ** t)", "mh = mk"),                          # no bias correction
    ("vh = vk / (1 - b2 ** t)", "vh = vk"),
    ("mk[...] = b1 * mk + (1 - b1) * grads[key]",
     "mk[...] = b1 * mk + 0.5 * (1 - b1) * grads[key]"),             # halved first moment
    ("np.sqrt(vh) + eps", "vh + eps"),                               # missing square root
    ('state["t"] = state.get("t", 0) + 1', 'state["t"] = 1'),        # step count stuck
])
def test_mutant_adam_fails_hand_pin(old, new):
    """Planted mistakes in a copy of the oracle's Adam step fail the pin."""
    import types
    src = open(PC.__file__).read()
    assert old in src
    m = types.ModuleType("precond_mutant")
    exec(compile(src.replace(old, new), "precond_mutant", "exec"), m.__dict__)
    g = globals()
    saved = g["PC"]
    g["PC"] = m
    try:
        with pytest.raises(AssertionError):
            test_adam_step_by_hand()
    finally:
        g["PC"] = saved

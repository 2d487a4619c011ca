r"""CPU oracle of the factorized preconditioners.  TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may use
this module.  FP64 throughout, plain loops and NumPy / SciPy calls.

Both preconditioners are applied as M = G^T G with G sparse lower triangular
on (a subset of) the lower-triangular pattern of A, so M is symmetric positive
definite whenever G has a positive diagonal.  The paper itself uses
incomplete factorisations (Sec. 5.3, 5.4); these two stand in for them and
are defined here:

FSAI (factorized sparse approximate inverse, Kolotilina and Yeremin): for
each row i with pattern P_i (columns j <= i of row i of A, optionally capped
to the `cap` largest |a_ij| plus the diagonal), solve A[P_i, P_i] y = e_i and
set G[i, P_i] = y / sqrt(y_i).  Then (G A)_{ij} = 0 for j in P_i \ {i} and
(G A G^T)_{ii} = 1.

Learned factor: a two-layer MLP maps features of each lower-triangular
nonzero (i, j) to a scalar o_ij.  G[i, i] = exp(o_ii) / sqrt(a_ii) and
G[i, j] = -o_ij a_ij / (cbar a_jj sqrt(a_ii)) for j < i, with cbar the
mean normalised coupling |a_ij| / sqrt(a_ii a_jj) over the strictly lower
entries.  G has a positive diagonal (M is SPD by construction) and a zero
output layer gives G = D^{-1/2}, i.e. M equals the Jacobi preconditioner.
Up to cbar the off-diagonal scale is that of a first-order factor: o = cbar
off the diagonal and 0 on it gives D^{-1/2}(I - L D^{-1}) (L the strict
lower triangle of A), the first-order expansion of D^{1/2}(D + L)^{-1},
whose G^T G is the symmetric Gauss-Seidel approximation of A^{-1}; for a
constant-coefficient stencil the scale is 1 / sqrt(a_jj).  So a column
shared by many rows (a graph hub) enters G^T with weights that fall as
1/a_jj and the network only has to learn an O(1) factor.  The loss over pairs (r_s, e_s) = (A u_s, u_s)
from the solver's basis is the mean squared sine of the angle between the
preconditioned residual M r_s and e_s,
L = (1/S) sum_s [1 - <M r_s, e_s>^2 / (||M r_s||^2 ||e_s||^2)],
which does not depend on the scale of M r_s: the Krylov space the inner
iteration builds from C = (I - X X^T B) M (A - rho B) (Sec. 3) depends on M
only up to a scalar per vector, so an absolute-scale target (M A = I) would
ask for gains the sparse factor cannot give on the low modes.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

NFEAT = 8               # per-row features
NIN = 2 * NFEAT + 1     # MLP input width per nonzero
NHID = 64               # hidden width


# ---------------------------------------------------------------------------
# FSAI
# ---------------------------------------------------------------------------

def fsai_pattern(A, cap=None):
    """Lower-triangular pattern of A per row, optionally capped.

    Returns a list of sorted int arrays, P_i ending with i.
    """
    A = sp.csr_matrix(A)
    pats = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        low = cols < i
        c, v = cols[low], vals[low]
        if cap is not None and c.shape[0] > cap - 1:
            # keep the cap-1 largest |a_ij|; ties broken by smaller column
            order = np.lexsort((c, -np.abs(v)))[:cap - 1]
            c = np.sort(c[order])
        pats.append(np.concatenate([c, [i]]).astype(np.int64))
    return pats


def fsai(A, cap=None):
    """FSAI factor G (CSR, lower triangular) of an SPD matrix A."""
    A = sp.csr_matrix(A)
    Ad = A.toarray() if A.shape[0] <= 2000 else None
    n = A.shape[0]
    pats = fsai_pattern(A, cap)
    rows, cols, vals = [], [], []
    for i in range(n):
        P = pats[i]
        if Ad is not None:
            S = Ad[np.ix_(P, P)]
        else:
            S = A[P][:, P].toarray()
        e = np.zeros(P.shape[0])
        e[-1] = 1.0
        y = np.linalg.solve(S, e)
        if not y[-1] > 0.0:
            raise ValueError(f"FSAI: non-positive pivot in row {i}")
        g = y / math.sqrt(y[-1])
        rows.append(np.full(P.shape[0], i))
        cols.append(P)
        vals.append(g)
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    G.sort_indices()
    return G


# ---------------------------------------------------------------------------
# learned factor: features, MLP, loss and gradients
# ---------------------------------------------------------------------------

def row_features(A):
    """Per-row features, z-scored over the rows of A (shape n x NFEAT).

    raw features of row i (off-diagonal entries o = {|a_ij| : j != i}):
      degree, a_ii, sum(o), mean(o), min(o), max(o), std(o), a_ii / sum(o)
    (statistics of an empty o are 0; the ratio of an empty row is 0).
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    F = np.zeros((n, NFEAT))
    for i in range(n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        d = float(vals[cols == i][0]) if np.any(cols == i) else 0.0
        o = np.abs(vals[cols != i])
        deg = o.shape[0]
        if deg:
            s = float(o.sum())
            mean = s / deg
            F[i] = [deg, d, s, mean, o.min(), o.max(),
                    math.sqrt(max(float(np.mean((o - mean) ** 2)), 0.0)), d / s]
        else:
            F[i] = [0.0, d, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    mu = F.mean(axis=0)
    sd = F.std(axis=0)
    sd[sd == 0.0] = 1.0
    return (F - mu) / sd


def tril_entries(A):
    """(rows, cols, vals) of the lower triangle of A including the diagonal,
    in CSR order."""
    L = sp.tril(sp.csr_matrix(A), format="csr")
    L.sort_indices()
    r = np.repeat(np.arange(L.shape[0]), np.diff(L.indptr))
    return r, L.indices.astype(np.int64), L.data.astype(np.float64), L


def mlp_inputs(A, feats=None):
    """Input matrix (nnz_tril x NIN): [f_i, f_j, |a_ij| / sqrt(a_ii a_jj)]."""
    A = sp.csr_matrix(A)
    if feats is None:
        feats = row_features(A)
    r, c, v, _ = tril_entries(A)
    d = A.diagonal()
    x = np.hstack([feats[r], feats[c], (np.abs(v) / np.sqrt(d[r] * d[c]))[:, None]])
    return x


def init_params(seed=0, zero_last=True):
    """MLP parameters {W1 (NHID x NIN), b1 (NHID), w2 (NHID), b2 ()}."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((NHID, NIN)) * math.sqrt(2.0 / NIN)
    b1 = np.zeros(NHID)
    w2 = np.zeros(NHID) if zero_last else rng.standard_normal(NHID) * math.sqrt(1.0 / NHID)
    return {"W1": W1, "b1": b1, "w2": w2, "b2": np.zeros(())}


def mlp_forward(params, x):
    """o = w2 . relu(W1 x + b1) + b2 for each input row.  Returns (o, cache)."""
    pre = x @ params["W1"].T + params["b1"][None, :]
    h = np.maximum(pre, 0.0)
    o = h @ params["w2"] + params["b2"]
    return o, (x, pre, h)


def mlp_backward(params, cache, do):
    """Gradients of sum(do * o) with respect to the MLP parameters."""
    x, pre, h = cache
    gw2 = h.T @ do
    gb2 = np.sum(do)
    dh = np.outer(do, params["w2"])
    dpre = dh * (pre > 0.0)
    gW1 = dpre.T @ x
    gb1 = dpre.sum(axis=0)
    return {"W1": gW1, "b1": gb1, "w2": gw2, "b2": np.asarray(gb2)}


def coupling_scale(A):
    """Mean of |a_ij| / sqrt(a_ii a_jj) over the strictly lower entries of A
    (1 when there are none)."""
    r, c, v, _ = tril_entries(A)
    d = sp.csr_matrix(A).diagonal()
    off = r != c
    if not np.any(off):
        return 1.0
    cb = float(np.mean(np.abs(v[off]) / np.sqrt(d[r[off]] * d[c[off]])))
    return cb if cb > 0.0 else 1.0


def offdiag_scale(A):
    """dG[i,j]/do_ij = -a_ij / (cbar a_jj sqrt(a_ii)) per lower nonzero (the
    diagonal entries' values are unused)."""
    r, c, v, _ = tril_entries(A)
    d = sp.csr_matrix(A).diagonal()
    return -v / (coupling_scale(A) * d[c] * np.sqrt(d[r]))


def assemble_G(A, o):
    """G on the lower pattern of A from MLP outputs o (one per tril nonzero)."""
    r, c, v, L = tril_entries(A)
    d = sp.csr_matrix(A).diagonal()
    g = np.where(r == c, np.exp(o) / np.sqrt(d[c]), o * offdiag_scale(A))
    return sp.csr_matrix((g, L.indices, L.indptr), shape=L.shape)


def loss_and_grad_G(G, R, E):
    """Angle loss L and dL/dG on G's pattern (values in G's CSR order).

    R, E are n x S (columns are the pairs).  With y = G r, q = G^T y = M r,
    a = <q, e>, b = ||q||^2, c = ||e||^2 the pair's loss is 1 - a^2/(b c) and
    its gradient is y z^T + (G z) r^T with
    z = (-2 a / (b c) e + 2 a^2 / (b^2 c) q) / S, restricted to the nonzeros.
    """
    G = sp.csr_matrix(G)
    S = R.shape[1]
    Y = G @ R
    Q = G.T @ Y
    a = np.sum(Q * E, axis=0)
    b = np.sum(Q * Q, axis=0)
    c = np.sum(E * E, axis=0)
    L = float(np.mean(1.0 - a * a / (b * c)))
    Z = ((-2.0 * a / (b * c))[None, :] * E + (2.0 * a * a / (b * b * c))[None, :] * Q) / S
    Uz = G @ Z
    r = np.repeat(np.arange(G.shape[0]), np.diff(G.indptr))
    col = G.indices
    grad = np.sum(Y[r] * Z[col] + Uz[r] * R[col], axis=1)
    return L, grad


def loss_and_grad_params(params, A, R, E, x=None):
    """Loss of the learned factor and its gradient with respect to the MLP."""
    if x is None:
        x = mlp_inputs(A)
    o, cache = mlp_forward(params, x)
    G = assemble_G(A, o)
    L, gG = loss_and_grad_G(G, R, E)
    r, c, v, _ = tril_entries(A)
    # chain rule through G[i,i] = exp(o)/sqrt(a_ii), G[i,j] = o * offdiag_scale
    gvals = G.data
    do = np.where(r == c, gG * gvals, gG * offdiag_scale(A))
    return L, mlp_backward(params, cache, do), G


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) in place; state holds m, v and t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for key in params:
        mk = state.setdefault("m_" + key, np.zeros_like(params[key]))
        vk = state.setdefault("v_" + key, np.zeros_like(params[key]))
        mk[...] = b1 * mk + (1 - b1) * grads[key]
        vk[...] = b2 * vk + (1 - b2) * grads[key] ** 2
        mh = mk / (1 - b1 ** t)
        vh = vk / (1 - b2 ** t)
        params[key] = params[key] - lr * mh / (np.sqrt(vh) + eps)
    return params

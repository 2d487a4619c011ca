"""Seeded synthetic operators shaped like the workloads TRPL+K is run on.

This module holds no arithmetic of the eigensolver itself: it only builds the
input pencils (A, B) in CSR form, the starting block X0 and the random draws
both sides consume.  The HIP library and the CPU oracle read the same arrays,
so the two are compared on byte-identical inputs.

The paper (Sec. 5, Tables 1 and 6) measures on SuiteSparse / Matrix Market
matrices.  Those are not reproduced here; the operators below stand in for
them with the sizes, sparsity structure and spectra of the five workloads:

  lap2d      2-D 5-point Dirichlet Laplacian, stencil [4, -1]
  lap3d      3-D 7-point Dirichlet Laplacian [6, -1] plus a random diagonal
             potential V ~ U[0, vmax] (clustered low spectrum)
  fem3d      trilinear (Q1) hexahedral FEM stiffness with a lognormal element
             coefficient field, and the consistent Q1 mass matrix (27-point)
  powerlaw   shifted weighted graph Laplacian L + shift*I of a Chung-Lu
             power-law graph with a Hamiltonian ring for connectivity
  aniso3d    3-D 7-point flux-form anisotropic diffusion with axis weights
             (1, 1e-2, 1e-4) times the harmonic mean of a lognormal field

All CSR arrays are int32 row pointers / column indices (sorted, no duplicate
columns) and float64 values.  Every random draw goes through numpy's PCG64
generator seeded with the given seed, so a (name, size, seed) triple fixes
the operator exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class CSR:
    """A square sparse matrix in CSR form (int32 indices, float64 values)."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(M) -> "CSR":
        M = M.tocsr()
        M.sum_duplicates()
        M.sort_indices()
        return CSR(int(M.shape[0]), M.indptr.astype(np.int32), M.indices.astype(np.int32),
                   M.data.astype(np.float64))


@dataclasses.dataclass
class Problem:
    """A pencil (A, B) with solver parameters; B is None for B = I."""

    name: str
    A: CSR
    B: Optional[CSR]
    p: int
    m: int
    k: int
    l: int
    tol: float
    seed: int
    meta: dict


# ---------------------------------------------------------------------------
# stencil helpers
# ---------------------------------------------------------------------------

def _stencil_to_csr(shape, offsets, coeffs) -> CSR:
    """Assemble a structured-grid operator from per-node stencil coefficients.

    shape   grid extents (nz, ny, nx) or (ny, nx); node linear index is C-order
    offsets list of integer offset tuples, one per stencil entry
    coeffs  array (len(offsets), *shape) of the coefficient for each entry;
            entries pointing outside the grid are dropped (Dirichlet)
    """
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[d + 1:])) for d in range(nd)]
    lin = [sum(o[d] * strides[d] for d in range(nd)) for o in offsets]
    order = np.argsort(lin, kind="stable")  # column order within a row
    S = len(offsets)
    valid = np.ones((S,) + shape, dtype=bool)
    for s, o in enumerate(offsets):
        for d in range(nd):
            if o[d] == 0:
                continue
            idx = [slice(None)] * nd
            if o[d] > 0:
                idx[d] = slice(shape[d] - o[d], shape[d])
            else:
                idx[d] = slice(0, -o[d])
            valid[(s,) + tuple(idx)] = False
    valid = valid[order].reshape(S, n).T          # (n, S) in column order
    vals = np.asarray(coeffs)[order].reshape(S, n).T
    rows = np.arange(n, dtype=np.int64)
    cols = rows[:, None] + np.asarray([lin[s] for s in order], dtype=np.int64)[None, :]
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[valid].astype(np.int32)
    val = np.ascontiguousarray(vals[valid], dtype=np.float64)
    return CSR(n, rowptr.astype(np.int32), col, val)


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------

def lap2d(N: int) -> CSR:
    """2-D 5-point Dirichlet Laplacian on an N x N interior grid, stencil [4, -1].

    Eigenvalues are 4 sin^2(i pi / (2(N+1))) + 4 sin^2(j pi / (2(N+1))).
    """
    shape = (N, N)
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    co = np.empty((5, N, N))
    co[0] = 4.0
    co[1:] = -1.0
    return _stencil_to_csr(shape, offs, co)


def lap3d(N: int, vmax: float = 0.0, seed: int = 12) -> CSR:
    """3-D 7-point Dirichlet Laplacian on N^3 [6, -1] plus diag V_i ~ U[0, vmax]."""
    shape = (N, N, N)
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    co = np.empty((7,) + shape)
    co[0] = 6.0
    if vmax != 0.0:
        rng = np.random.default_rng(seed)
        co[0] += rng.uniform(0.0, vmax, size=shape)
    co[1:] = -1.0
    return _stencil_to_csr(shape, offs, co)


def _q1_element():
    """Element stiffness and consistent mass of a trilinear cube of unit size.

    Returns (K, M) as (2,2,2,2,2,2) arrays indexed [cz,cy,cx, dz,dy,dx]; the
    physical element of side h has K_h = h * K and M_h = h^3 * M.
    """
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    K = (np.einsum("ad,be,cf->abcdef", k1, m1, m1)
         + np.einsum("ad,be,cf->abcdef", m1, k1, m1)
         + np.einsum("ad,be,cf->abcdef", m1, m1, k1))
    M = np.einsum("ad,be,cf->abcdef", m1, m1, m1)
    return K, M


def fem3d(Ne: int, sigma: float = 0.5, seed: int = 12):
    """Q1 hexahedral FEM pencil on the unit cube with Ne^3 elements, h = 1/Ne.

    Nodes on the boundary are Dirichlet and eliminated, leaving (Ne-1)^3
    unknowns.  A = sum_e kappa_e K_e with kappa_e = exp(sigma z_e), z_e iid
    N(0,1); B = sum_e M_e (consistent mass).  Both have the 27-point pattern.
    With sigma = 0 the generalized eigenvalues are mu_a + mu_b + mu_c with
    mu_j = 6 (1 - cos t_j) / (h^2 (2 + cos t_j)), t_j = j pi / Ne.
    """
    h = 1.0 / Ne
    Ni = Ne - 1
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((Ne, Ne, Ne))
    kappa = np.exp(sigma * z) if sigma != 0.0 else np.ones((Ne, Ne, Ne))
    Ke, Me = _q1_element()
    shape = (Ni, Ni, Ni)
    offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    coA = np.zeros((27,) + shape)
    coB = np.zeros((27,) + shape)
    # interior node (iz,iy,ix) in 0..Ni-1 is global node (iz+1,...); the
    # element with lower corner e = node - c holds the node at local corner c.
    for s, (dz, dy, dx) in enumerate(offs):
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    ez_, ey_, ex_ = cz + dz, cy + dy, cx + dx
                    if not (0 <= ez_ <= 1 and 0 <= ey_ <= 1 and 0 <= ex_ <= 1):
                        continue
                    kv = Ke[cz, cy, cx, ez_, ey_, ex_] * h
                    mv = Me[cz, cy, cx, ez_, ey_, ex_] * h ** 3
                    # element lower corner index = (node+1) - c, node in 0..Ni-1
                    sl = (slice(1 - cz, 1 - cz + Ni), slice(1 - cy, 1 - cy + Ni),
                          slice(1 - cx, 1 - cx + Ni))
                    coA[s] += kv * kappa[sl]
                    if mv != 0.0:
                        coB[s] += mv
    A = _stencil_to_csr(shape, offs, coA)
    B = _stencil_to_csr(shape, offs, coB)
    return A, B


def aniso3d(N: int, sigma: float = 1.0, axis_w=(1.0, 1e-2, 1e-4), seed: int = 12) -> CSR:
    """3-D 7-point flux-form diffusion on N^3 cells with Dirichlet walls.

    Face coefficient between neighbouring cells = axis weight times the
    harmonic mean of the two cells' kappa, kappa = exp(sigma z), z iid N(0,1).
    A wall face uses the interior cell's kappa.  axis_w is ordered (x, y, z)
    with x the fastest-varying index.  With sigma = 0 the eigenvalues are
    sum_d axis_w[d] 4 sin^2(i_d pi / (2(N+1))).
    """
    shape = (N, N, N)  # (z, y, x)
    if sigma != 0.0:
        rng = np.random.default_rng(seed)
        kap = np.exp(sigma * rng.standard_normal(shape))
    else:
        kap = np.ones(shape)
    wx, wy, wz = axis_w
    co = np.zeros((7,) + shape)

    def face(axis, w):
        # harmonic mean across the faces normal to `axis`; shape N-1 along axis
        a = np.take(kap, np.arange(N - 1), axis=axis)
        b = np.take(kap, np.arange(1, N), axis=axis)
        return w * 2.0 * a * b / (a + b)

    for axis, w, (sm, sp_) in ((0, wz, (5, 6)), (1, wy, (3, 4)), (2, wx, (1, 2))):
        f = face(axis, w)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, N - 1)
        hi[axis] = slice(1, N)
        # coupling to the + neighbour for cells 0..N-2, to the - neighbour for 1..N-1
        co[sp_][tuple(lo)] = -f
        co[sm][tuple(hi)] = -f
        co[0][tuple(lo)] += f
        co[0][tuple(hi)] += f
        # wall faces: first and last cell along the axis
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = slice(0, 1)
        last[axis] = slice(N - 1, N)
        co[0][tuple(first)] += w * kap[tuple(first)]
        co[0][tuple(last)] += w * kap[tuple(last)]
    # reorder offsets from (z,y,x) stencil slots into the helper's tuple layout
    offs_zyx = [(0, 0, 0), (0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)]
    return _stencil_to_csr(shape, offs_zyx, co)


def powerlaw(n: int, avg_deg: float = 16.0, gamma: float = 2.5, shift: float = 0.01,
             wlo: float = 0.5, whi: float = 2.0, seed: int = 12,
             max_deg: Optional[float] = None) -> CSR:
    """Shifted weighted Laplacian L + shift*I of a Chung-Lu power-law graph.

    Expected degrees w_i proportional to (i+1)^(-1/(gamma-1)), scaled to mean
    avg_deg and capped at sqrt(avg_deg n).  A random Hamiltonian ring (degree 2
    per vertex) keeps the graph connected; the Chung-Lu part is scaled down by
    those 2 so the mean degree stays near avg_deg.  Edge weights U[wlo, whi].
    The graph is connected, so the smallest eigenvalue is exactly `shift`
    with eigenvector n^{-1/2} * ones.
    """
    rng = np.random.default_rng(seed)
    if max_deg is None:
        max_deg = math.sqrt(avg_deg * n)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= (avg_deg - 2.0) / w.mean()
    w = np.minimum(w, max_deg)
    n_draw = int(round(n * (avg_deg - 2.0) / 2.0))
    prob = w / w.sum()
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    i = np.searchsorted(cdf, rng.random(n_draw), side="right").astype(np.int64)
    j = np.searchsorted(cdf, rng.random(n_draw), side="right").astype(np.int64)
    i = np.minimum(i, n - 1)
    j = np.minimum(j, n - 1)
    perm = rng.permutation(n).astype(np.int64)
    ri = perm
    rj = np.roll(perm, -1)
    ii = np.concatenate([i, ri])
    jj = np.concatenate([j, rj])
    keep = ii != jj
    ii, jj = ii[keep], jj[keep]
    lo = np.minimum(ii, jj)
    hi = np.maximum(ii, jj)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    wt = rng.uniform(wlo, whi, size=key.shape[0])
    import scipy.sparse as sp
    W = sp.coo_matrix((np.concatenate([wt, wt]), (np.concatenate([lo, hi]),
                                                   np.concatenate([hi, lo]))), shape=(n, n)).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    L = sp.diags(deg + shift) - W
    return CSR.from_scipy(L)


def start_block(n: int, k: int, seed: int = 12) -> np.ndarray:
    """Starting block X0: n x k, uniform[-1, 1], Fortran (column-major) order."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(k, n)).T  # column c is the c-th draw of n values
    return np.asfortranarray(X)


def splitmix64_block(n: int, k: int, seed: int = 12) -> np.ndarray:
    """n x k uniform[-1, 1) block (Fortran order) from the counter-based
    SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014): entry
    e = column * n + row is b * 2^-52 - 1, b the top 53 bits of
    mix(seed + (e + 1) * 0x9e3779b97f4a7c15), mix the generator's 64-bit
    finaliser.  The GPU library draws its default start block (x0 = NULL) by
    the same definition, so the two blocks are identical."""
    X = np.empty((n, k), order="F")
    s = np.uint64(seed % (1 << 64))
    for c in range(k):   # one column at a time keeps the temporaries at n words
        e = np.arange(c * n, (c + 1) * n, dtype=np.uint64)
        z = s + (e + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        X[:, c] = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
    return X


def lap2d_island(N: int, s: int, diag: float = 2.5) -> CSR:
    """lap2d(N) with a disconnected path of s extra nodes appended: the
    block-diagonal matrix diag(lap2d(N), tridiag(-1, diag, -1) of order s).
    Coordinates N^2 .. N^2 + s - 1 span an invariant subspace of dimension s."""
    import scipy.sparse as sp
    P = sp.diags([-np.ones(s - 1), np.full(s, diag), -np.ones(s - 1)], [-1, 0, 1])
    return CSR.from_scipy(sp.block_diag([lap2d(N).to_scipy(), P], format="csr"))


def island_block(n: int, s: int, k: int, seed: int = 12) -> np.ndarray:
    """n x k start block that is zero outside the last s coordinates, where it
    is uniform[-1, 1].  Fortran (column-major) order."""
    X = np.zeros((n, k), order="F")
    X[n - s:, :] = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(k, s)).T
    return X


# ---------------------------------------------------------------------------
# the five workloads (full size) and their small variants for tests
# ---------------------------------------------------------------------------

def make(name: str, scale: str = "full", seed: int = 12, **kw) -> Problem:
    """Build a named workload.

    name   'lap2d' | 'lap3d' | 'fem3d' | 'powerlaw' | 'aniso3d'
    scale  'full' (the sizes the method is measured on) or 'small' (the same
           generator at a size a dense eigendecomposition or the CPU oracle
           finishes in seconds); keyword overrides are passed through.
    """
    if name == "lap2d":
        N = kw.pop("N", 64 if scale == "full" else 24)
        A = lap2d(N)
        return Problem(name, A, None, kw.pop("p", 5), kw.pop("m", 20), kw.pop("k", 8),
                       kw.pop("l", 1), kw.pop("tol", 1e-8), seed, {"N": N})
    if name == "lap3d":
        N = kw.pop("N", 128 if scale == "full" else 16)
        vmax = kw.pop("vmax", 0.05)
        A = lap3d(N, vmax, seed)
        return Problem(name, A, None, kw.pop("p", 10), kw.pop("m", 40), kw.pop("k", 20),
                       kw.pop("l", 1), kw.pop("tol", 1e-8), seed, {"N": N, "vmax": vmax})
    if name == "fem3d":
        Ne = kw.pop("Ne", 97 if scale == "full" else 10)
        sigma = kw.pop("sigma", 0.5)
        A, B = fem3d(Ne, sigma, seed)
        return Problem(name, A, B, kw.pop("p", 16), kw.pop("m", 48), kw.pop("k", 24),
                       kw.pop("l", 1), kw.pop("tol", 1e-8), seed, {"Ne": Ne, "sigma": sigma})
    if name == "powerlaw":
        n = kw.pop("n", 1_000_000 if scale == "full" else 3000)
        gkw = {x: kw.pop(x) for x in ("avg_deg", "gamma", "shift", "max_deg") if x in kw}
        A = powerlaw(n, seed=seed, **gkw)
        return Problem(name, A, None, kw.pop("p", 20), kw.pop("m", 48), kw.pop("k", 24),
                       kw.pop("l", 1), kw.pop("tol", 1e-8), seed, {"n": n})
    if name == "aniso3d":
        N = kw.pop("N", 256 if scale == "full" else 12)
        sigma = kw.pop("sigma", 1.0)
        A = aniso3d(N, sigma, seed=seed)
        return Problem(name, A, None, kw.pop("p", 50), kw.pop("m", 64), kw.pop("k", 32),
                       kw.pop("l", 1), kw.pop("tol", 1e-8), seed, {"N": N, "sigma": sigma})
    raise ValueError(f"unknown workload {name!r}")

"""Kernel-level parity of the HIP building blocks, through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import CSR, lap2d, lap3d, fem3d, powerlaw, aniso3d  # noqa: E402
from spmv_format import dia_ndiag as _dia_ndiag  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_10128_amd as T
    T.lib()
    return T


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


MATS = {
    "lap2d": lambda: lap2d(37),
    "lap3d": lambda: lap3d(13, 0.05),
    "fem3d_A": lambda: fem3d(9, 0.5)[0],
    "fem3d_B": lambda: fem3d(9, 0.5)[1],
    "aniso": lambda: aniso3d(11, 1.0),
    # hub rows longer than 256 entries exercise the workgroup-per-row kernel
    "powerlaw_hubs": lambda: powerlaw(6000, avg_deg=24.0, max_deg=900.0),
    # rows of 6..25 entries: CSR-stream with shorter tiles
    "powerlaw_flat": lambda: powerlaw(3000, avg_deg=6.0, max_deg=8.0),
    # rows of ~20..60 entries: 8-row tiles
    "powerlaw_dense": lambda: powerlaw(2000, avg_deg=24.0, max_deg=32.0),
}


def _stream_rows(A):
    """Tile height the SpMV plan picks with lanes=0: the tallest of 64, 32,
    16, 8 rows whose fullest tile holds at most 512 entries, else 0 (the
    CSR-Adaptive blocks plus the workgroup-per-row kernel for rows of more
    than 512 entries)."""
    rp = A.rowptr
    for rows in (64, 32, 16, 8):
        if max(int(rp[min(r + rows, A.n)] - rp[r]) for r in range(0, A.n, rows)) <= 512:
            return rows
    return 0


def _band(n, offsets, seed, drop=0.0, dup=0):
    """n x n matrix with random values on the given diagonals (entries that
    leave the matrix are absent); a fraction `drop` of the entries removed;
    `dup` entries stored twice (CSR with repeated positions, summed)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for o in offsets:
        i = np.arange(max(0, -o), min(n, n - o))
        rows.append(i)
        cols.append(i + o)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    keep = rng.random(r.size) >= drop
    r, c = r[keep], c[keep]
    if dup:
        pick = rng.choice(r.size, dup, replace=False)
        r = np.concatenate([r, r[pick]])
        c = np.concatenate([c, c[pick]])
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, r + 1, 1)
    return CSR(n, np.cumsum(rowptr).astype(np.int32), c.astype(np.int32), rng.standard_normal(r.size))


BANDS = {
    # 27 and 14 diagonals: the 32- and 16-diagonal instances of the kernel
    "band27": lambda: _band(5000, list(range(-299, 300, 23)), 3),
    "band14": lambda: _band(3001, [-1200, -700, -64, -9, -2, -1, 0, 1, 2, 9, 64, 700, 1200, 1999], 4),
    "diagonal": lambda: _band(777, [0], 5),
    # holes inside the diagonals (zero padding) and repeated positions
    "band_gaps": lambda: _band(4099, [-90, -1, 0, 1, 90], 6, drop=0.08),
    "band_dup": lambda: _band(2500, [-50, -1, 0, 1, 50], 7, dup=40),
}


def test_spmv_cases_cover_every_kernel():
    dia = {k: _dia_ndiag(f()) for k, f in {**MATS, **BANDS}.items()}
    assert dia["lap2d"] == 5 and dia["lap3d"] == 7 and dia["aniso"] == 7
    assert dia["band27"] == 27 and dia["band14"] == 14 and dia["diagonal"] == 1
    assert dia["band_gaps"] == 5 and dia["band_dup"] == 5
    # too few entries per diagonal at this size, or not banded: CSR kernels
    assert dia["fem3d_A"] == 0 and dia["fem3d_B"] == 0
    assert all(dia[k] == 0 for k in MATS if k.startswith("powerlaw"))
    picked = {k: _stream_rows(f()) for k, f in MATS.items()}
    assert picked["lap3d"] == 64 and picked["fem3d_A"] == 16
    assert picked["powerlaw_flat"] == 32 and picked["powerlaw_dense"] == 8
    assert picked["powerlaw_hubs"] == 0
    lens = np.diff(MATS["powerlaw_hubs"]().rowptr)
    assert (lens > 512).any() and (lens <= 512).any()


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("lanes", [0, 4, 64])
def test_spmv_f64_parity(T, name, lanes):
    A = MATS[name]()
    print(f"spmv f64 {name} n={A.n} nnz={A.nnz} lanes={lanes}", flush=True)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(A.n)
    ref = A.to_scipy() @ x
    y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    T.spmv(_dev(A.rowptr), _dev(A.col), _dev(A.val), _dev(x), y, lanes)
    got = y.cpu().numpy()
    # each row sum is a different rounding order of the same terms
    bound = 4 * 2.2e-16 * (abs(A.to_scipy()) @ np.abs(x)) * np.diff(A.rowptr).max()
    assert np.all(np.abs(got - ref) <= bound + 1e-300)


@pytest.mark.parametrize("name", list(BANDS))
def test_spmv_diagonal_storage_parity(T, name):
    """Banded matrices take the diagonal-storage kernel (lanes=0) and the
    CSR-stream kernel (lanes=4); both match scipy to rounding."""
    A = BANDS[name]()
    print(f"spmv dia {name} n={A.n} nnz={A.nnz}", flush=True)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(A.n)
    S = A.to_scipy()  # repeated positions are summed
    ref = S @ x
    bound = 4 * 2.2e-16 * (abs(S) @ np.abs(x)) * np.diff(A.rowptr).max()
    for lanes in (0, 4):
        y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        T.spmv(_dev(A.rowptr), _dev(A.col), _dev(A.val), _dev(x), y, lanes)
        assert np.all(np.abs(y.cpu().numpy() - ref) <= bound + 1e-300), lanes
    x32 = x.astype(np.float32)
    y32 = torch.zeros(A.n, dtype=torch.float32, device="cuda")
    T.spmv(_dev(A.rowptr), _dev(A.col), _dev(A.val.astype(np.float32)), _dev(x32), y32, 0)
    S32 = A.to_scipy().astype(np.float32).astype(np.float64)
    ref32 = S32 @ x32.astype(np.float64)
    scale = abs(S32) @ np.abs(x32.astype(np.float64))
    assert np.all(np.abs(y32.cpu().numpy() - ref32) <= 1e-6 * scale * np.diff(A.rowptr).max())


@pytest.mark.parametrize("name,ncols", [("lap3d", 3), ("aniso", 16), ("band27", 5), ("band_gaps", 2),
                                        ("band_dup", 9), ("diagonal", 1), ("powerlaw_hubs", 4),
                                        ("fem3d_A", 7)])
def test_spmm_columns_equal_spmv(T, name, ncols):
    """Y = A X for the block form's appended columns: with diagonal storage
    one read of A serves every column, and each column is the single-vector
    product bit for bit; CSR patterns take one product per column."""
    A = {**MATS, **BANDS}[name]()
    print(f"spmm {name} n={A.n} nnz={A.nnz} ncols={ncols}", flush=True)
    rng = np.random.default_rng(ncols)
    ld = A.n + 5
    X = rng.standard_normal((ncols, ld))
    Y = torch.full((ncols, ld + 2), float("nan"), dtype=torch.float64, device="cuda")
    rp, cl, vl = _dev(A.rowptr), _dev(A.col), _dev(A.val)
    T.spmm(rp, cl, vl, _dev(X), Y)
    got = Y.cpu().numpy()
    for j in range(ncols):
        y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        T.spmv(rp, cl, vl, _dev(X[j, :A.n]), y, 0)
        assert np.array_equal(got[j, :A.n], y.cpu().numpy()), j
    assert np.all(np.isnan(got[:, A.n:]))            # nothing written past n rows
    ref = A.to_scipy() @ X[:, :A.n].T
    bound = 4 * 2.2e-16 * (abs(A.to_scipy()) @ np.abs(X[:, :A.n].T)) * np.diff(A.rowptr).max()
    assert np.all(np.abs(got[:, :A.n].T - ref) <= bound + 1e-300)


@pytest.mark.parametrize("name", ["lap3d", "powerlaw_hubs", "fem3d_A", "aniso"])
def test_spmv_f32_against_f64(T, name):
    A = MATS[name]()
    rng = np.random.default_rng(2)
    x = rng.standard_normal(A.n).astype(np.float32)
    ref = A.to_scipy().astype(np.float64) @ x.astype(np.float64)
    y = torch.zeros(A.n, dtype=torch.float32, device="cuda")
    T.spmv(_dev(A.rowptr), _dev(A.col), _dev(A.val.astype(np.float32)), _dev(x), y, 0)
    got = y.cpu().numpy().astype(np.float64)
    scale = abs(A.to_scipy()) @ np.abs(x.astype(np.float64))
    assert np.all(np.abs(got - ref) <= 1e-6 * scale * np.diff(A.rowptr).max())


@pytest.mark.parametrize("n", [1, 63, 257, 1000, 70001])
@pytest.mark.parametrize("c", [1, 7, 20, 64, 128])
def test_gemv_t_and_fused_update(T, n, c):
    print(f"gemv n={n} c={c}", flush=True)
    rng = np.random.default_rng(n + c)
    U = rng.standard_normal((c, n))          # row i of U is column i of the basis
    v = rng.standard_normal(n)
    ld = n + (n % 2)                         # row pairs: even leading dimension
    Ud = torch.full((c, ld), float("nan"), dtype=torch.float64, device="cuda")
    Ud[:, :n] = _dev(U)                      # padding rows must never be read
    h = torch.zeros(c, dtype=torch.float64, device="cuda")
    T.gemv_t(Ud, _dev(v), h, n=n)
    ref = U @ v
    tol = 8 * 2.2e-16 * (np.abs(U) @ np.abs(v)) * np.log2(n + 2)
    assert np.all(np.abs(h.cpu().numpy() - ref) <= tol)
    hh = rng.standard_normal(c)
    w = _dev(v.copy())
    h2 = torch.zeros(c, dtype=torch.float64, device="cuda")
    T.cgs_update_dot(Ud, _dev(hh), w, h2, n=n)
    wref = v - U.T @ hh
    assert np.allclose(w.cpu().numpy(), wref, rtol=1e-13, atol=1e-13 * np.abs(v).max() * c)
    h2ref = U @ wref
    tol2 = 16 * 2.2e-16 * (np.abs(U) @ (np.abs(v) + np.abs(U.T) @ np.abs(hh))) * np.log2(n + 2) * c
    assert np.all(np.abs(h2.cpu().numpy() - h2ref) <= tol2)


@pytest.mark.parametrize("b", [1, 2, 3, 8, 20, 47, 64])
def test_syev_parity(T, b):
    rng = np.random.default_rng(b)
    M = rng.standard_normal((b, b))
    S = M + M.T
    if b >= 8:
        S[0, 1] = S[1, 0] = 0.0
        S[2, 2] = S[3, 3]  # an exact tie on the diagonal
    th = torch.zeros(b, dtype=torch.float64, device="cuda")
    Y = torch.zeros((b, b), dtype=torch.float64, device="cuda")
    T.syev(_dev(S.T.copy()), th, Y)
    w = np.linalg.eigh(S)[0]
    got = th.cpu().numpy()
    Yc = Y.cpu().numpy().T  # column-major -> numpy
    nrm = np.linalg.norm(S, 2)
    assert np.all(np.diff(got) >= 0)
    assert np.max(np.abs(got - w)) <= 20 * b * 2.2e-16 * nrm
    assert np.max(np.abs(Yc.T @ Yc - np.eye(b))) <= 20 * b * 2.2e-16
    assert np.max(np.abs(S @ Yc - Yc * got[None, :])) <= 20 * b * 2.2e-16 * nrm


def test_syev_clustered_and_diagonal(T):
    """Already-diagonal input and a tight cluster: eigenvalues exact to rounding."""
    d = np.array([3.0, -1.0, 2.0, 2.0 + 1e-13, 0.5])
    S = np.diag(d)
    th = torch.zeros(5, dtype=torch.float64, device="cuda")
    Y = torch.zeros((5, 5), dtype=torch.float64, device="cuda")
    T.syev(_dev(S.T.copy()), th, Y)
    assert np.array_equal(th.cpu().numpy(), np.sort(d))


@pytest.mark.parametrize("scale", [1e-200, 1e-30, 1e30, 1e200])
def test_syev_any_magnitude(T, scale):
    """The stopping test and the angles use entries scaled by a power of two,
    so T * 2^k decomposes as T does (eigenvalues scale exactly, eigenvectors
    are orthonormal to rounding) for magnitudes whose squares over- or
    underflow."""
    b = 40
    rng = np.random.default_rng(7)
    M = rng.standard_normal((b, b))
    S = (M + M.T) * scale
    th = torch.zeros(b, dtype=torch.float64, device="cuda")
    Y = torch.zeros((b, b), dtype=torch.float64, device="cuda")
    T.syev(_dev(S.T.copy()), th, Y)
    w = np.linalg.eigh(M + M.T)[0] * scale
    got = th.cpu().numpy()
    Yc = Y.cpu().numpy().T
    nrm = np.linalg.norm(M + M.T, 2) * scale
    assert np.max(np.abs(got - w)) <= 20 * b * 2.2e-16 * nrm
    assert np.max(np.abs(Yc.T @ Yc - np.eye(b))) <= 20 * b * 2.2e-16


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 123457])
@pytest.mark.parametrize("b,k", [(4, 1), (8, 8), (20, 8), (40, 20), (48, 24), (64, 32), (64, 64)])
def test_rotate_mfma_parity(T, n, b, k):
    """X = U Y(:, :k) in place on the FP64 matrix cores (checks the lane layout
    of V_MFMA_F64_16X16X4F64 against numpy)."""
    if k > b:
        pytest.skip()
    print(f"rotate n={n} b={b} k={k}", flush=True)
    rng = np.random.default_rng(n * 7 + b)
    U = rng.standard_normal((b, n))
    Y = rng.standard_normal((b, b))
    Ud = _dev(U.copy())
    T.rotate(Ud, _dev(Y.T.copy()), k)
    got = Ud.cpu().numpy()
    ref = (U.T @ Y[:, :k]).T
    tol = 4 * b * 2.2e-16 * (np.abs(U.T) @ np.abs(Y[:, :k])).T
    assert np.all(np.abs(got[:k] - ref) <= tol)
    # columns beyond k untouched
    assert np.array_equal(got[k:], U[k:])

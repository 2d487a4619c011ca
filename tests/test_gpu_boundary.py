"""Boundary paths of the C ABI on the GPU, each against the FP64 CPU oracle
or against the library's own default path where the two must agree bit for
bit: the seeded default start block (x0 = NULL), the caller-owned
workspace, the paper's Frobenius stopping norm (eq. (5.1)), one Adam update
of the learned factor against the oracle's Kingma-Ba step, the FSAI factor
with capped hub rows entry by entry, the un-flag branch of the soft-locking
test (R8), and the hard-locking shape of the largest workload (p = 50,
m = 64, k = 32) at a size the oracle finishes."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import precond as PC  # noqa: E402
from oracle import trplk as O  # noqa: E402
from workloads import CSR, make, splitmix64_block, start_block  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_10128_amd as T
    T.lib()
    return T


def _pairs(T, P, X0=None, **kw):
    kw.setdefault("precond", "jacobi")
    s = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, **kw)
    st = s.solve(X0)
    ev, X, res, conv = s.eigpairs()
    s.close()
    return st, ev, X, res, conv


def _eig_ok(ev, ref, normA, rel=1e-10):
    return np.all(np.abs(ev - ref) <= np.maximum(rel * np.abs(ref), 16 * 2.2e-16 * normA))


# --------------------------------------------------------------------------
# x0 = NULL: the start block drawn on the device from the seed
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,kw,seed", [("lap2d", dict(N=24), 12),
                                          ("fem3d", dict(Ne=8, p=6, m=20, k=10), 5)])
def test_default_start_block_from_seed(T, name, kw, seed):
    """trplk_solve(x0 = NULL) draws SplitMix64 uniforms on the device; the
    solve is bit for bit the one started from the same block built on the
    host, and matches the oracle started from it."""
    P = make(name, "small", **kw)
    print(f"seeded start {name} n={P.A.n} seed={seed}", flush=True)
    X0 = splitmix64_block(P.A.n, P.k, seed)
    st0, ev0, X_0, res0, _ = _pairs(T, P, None, seed=seed)
    st1, ev1, X_1, res1, _ = _pairs(T, P, X0, seed=seed + 1)  # seed unused with an x0
    assert st0["cycles"] == st1["cycles"] and st0["matvecs"] == st1["matvecs"]
    assert np.array_equal(ev0, ev1) and np.array_equal(X_0, X_1)
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    ref = O.solve(A, B, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=O.jacobi(A))
    assert abs(st0["cycles"] - ref.cycles) <= 2
    scale = ref.normA if B is None else np.max(np.abs(ref.theta))
    assert _eig_ok(ev0, ref.theta, scale)
    # another seed gives another block (and still the same eigenvalues)
    st2, ev2, _, _, conv2 = _pairs(T, P, None, seed=seed + 1)
    assert conv2.all() and _eig_ok(ev2, ref.theta, scale, rel=1e-9)


def test_default_start_vector_pl1(T):
    """PL+1 takes column 0 of the seeded block."""
    P = make("lap2d", "small", N=24, p=1, m=12, k=1, l=1)
    x0 = splitmix64_block(P.A.n, 1, 3)
    st0, ev0, _, _, _ = _pairs(T, P, None, seed=3, method="pl1")
    st1, ev1, _, _, _ = _pairs(T, P, x0, seed=0, method="pl1")
    assert st0["cycles"] == st1["cycles"] and np.array_equal(ev0, ev1)


# --------------------------------------------------------------------------
# caller-owned workspace (trplk_workspace_size / trplk_create_ws)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,kw,prec", [
    ("lap2d", dict(N=24), "jacobi"),
    ("fem3d", dict(Ne=8, p=6, m=20, k=10), "fsai"),                 # B != I: B W in the workspace
    ("aniso3d", dict(N=10, p=12, m=16, k=8, tol=1e-9), "jacobi"),   # hard locking: [Q U]
])
def test_caller_workspace_matches_library_allocation(T, name, kw, prec):
    P = make(name, "small", **kw)
    print(f"workspace {name} n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    a = _pairs(T, P, X0, precond=prec)
    s = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond=prec, workspace=True)
    ws = s.workspace
    need = int(T.lib().trplk_workspace_size(P.A.n, int(P.B is not None), ctypes.byref(s.opts)))
    assert ws is not None and ws.numel() == need
    lib_bytes = s.device_bytes()
    st = s.solve(X0)
    ev, X, res, conv = s.eigpairs()
    # the basis lives in the caller's tensor: its first column is x_1
    ld = (P.A.n + 31) // 32 * 32
    w0 = ws[: 8 * ld].view(torch.float64)[: P.A.n].cpu().numpy()
    s.close()
    assert a[0]["cycles"] == st["cycles"] and np.array_equal(a[1], ev) and np.array_equal(a[2], X)
    assert np.array_equal(w0, X[:, 0])
    # the library's own allocations exclude the workspace
    s2 = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond=prec)
    assert s2.device_bytes() >= lib_bytes + need - 4096 * 16
    s2.close()


def test_caller_workspace_too_small_is_rejected(T):
    P = make("lap2d", "small", N=16, p=3, m=12, k=5)
    Ad = T.DeviceCSR(P.A)
    o = T._Opts()
    L = T.lib()
    L.trplk_default_opts(ctypes.byref(o))
    o.p, o.m, o.k = 3, 12, 5
    need = int(L.trplk_workspace_size(P.A.n, 0, ctypes.byref(o)))
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    ctx = ctypes.c_void_p()
    code = L.trplk_create_ws(ctypes.byref(ctx), ctypes.byref(Ad.c()), None, ctypes.byref(o),
                             T.MEM_DEVICE, T._stream(), T._ptr(buf), need - 256)
    assert code == -1 and not ctx.value and b"workspace" in L.trplk_last_error(None)
    code = L.trplk_create_ws(ctypes.byref(ctx), ctypes.byref(Ad.c()), None, ctypes.byref(o),
                             T.MEM_DEVICE, T._stream(), ctypes.c_void_p(buf.data_ptr() + 8), need)
    assert code == -1 and not ctx.value and b"aligned" in L.trplk_last_error(None)
    code = L.trplk_create_ws(ctypes.byref(ctx), ctypes.byref(Ad.c()), None, ctypes.byref(o),
                             T.MEM_DEVICE, T._stream(), T._ptr(buf), need)
    assert code == 0 and ctx.value
    L.trplk_destroy(ctx)
    del buf


# --------------------------------------------------------------------------
# the paper's stopping norm, eq. (5.1): ||A||_F
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,kw", [("lap2d", dict(N=64)), ("fem3d", dict(Ne=8, p=6, m=20, k=10))])
def test_frobenius_stopping_norm_parity(T, name, kw):
    P = make(name, "small", **kw)
    print(f"fro norm {name} n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    ref = O.solve(A, B, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=O.jacobi(A), norm="fro")
    st, ev, X, res, conv = _pairs(T, P, X0, norm="fro")
    if name == "lap2d":
        assert abs(ref.normA - 285.769) < 5e-4
    assert abs(st["normA"] - ref.normA) <= 1e-13 * ref.normA
    assert conv.all() and np.all(res <= P.tol * ref.normA * 1.001)
    assert abs(st["cycles"] - ref.cycles) <= 1
    scale = ref.normA if B is None else np.max(np.abs(ref.theta))
    assert _eig_ok(ev, ref.theta, scale, rel=1e-9)


# --------------------------------------------------------------------------
# learned factor: one Adam update against the oracle's Kingma-Ba step
# --------------------------------------------------------------------------

def test_adam_update_matches_oracle(T):
    """trplk_train_step applies Adam in float32 to the gradient it returns;
    the oracle's adam_step (float64) from the same gradient and moments gives
    the same parameters and moments to float32 rounding, on the first step
    (bias corrections 1 - 0.9, 1 - 0.999) and on the second."""
    P = make("powerlaw", "small", n=3000, p=6, m=20, k=10)
    X0 = start_block(P.A.n, P.k, 12)
    s = T.Solver(P.A, None, p=P.p, m=P.m, k=P.k, l=P.l, tol=1e-6, precond="jacobi")
    s.solve(X0)
    P0 = T.init_params(seed=1)
    P0[-65:-1] = np.random.default_rng(3).standard_normal(64).astype(np.float32) * 0.1
    params = P0.copy()
    m = np.zeros(T.MLP_NPARAM, dtype=np.float32)
    v = np.zeros(T.MLP_NPARAM, dtype=np.float32)
    ref = {"w": P0.astype(np.float64)}
    state = {}
    lr = 1e-2
    for step in (1, 2):
        g = np.empty(T.MLP_NPARAM)
        loss = s.train_step(params, m, v, step, lr, 8, grad=g)
        assert np.isfinite(loss) and np.any(g != 0.0)
        PC.adam_step(ref, {"w": g}, state, lr=lr)
        assert state["t"] == step
        d = np.abs(params - ref["w"])
        assert np.all(d <= 4e-7 * np.abs(ref["w"]) + 1e-4 * lr), (step, d.max())
        assert np.allclose(m, state["m_w"], rtol=1e-5, atol=1e-30)
        assert np.allclose(v, state["v_w"], rtol=1e-5, atol=1e-30)
        # the step moved the parameters by about lr (Adam's step size)
        moved = np.abs(params - P0) if step == 1 else None
        if moved is not None:
            big = np.abs(g) > 1e-6
            assert np.all(moved[big] > 0.5 * lr) and np.all(moved <= 1.001 * lr + 1e-6)
    s.close()


# --------------------------------------------------------------------------
# FSAI with capped hub rows, entry by entry
# --------------------------------------------------------------------------

def _lower_len(A):
    L = sp.tril(A, format="csr")
    return np.diff(L.indptr)


def _hubs_last(n=3000):
    """The power-law workload with its node order reversed: the generator
    numbers hubs first, so their rows hold few lower-triangular entries;
    reversed, the hub rows carry hundreds (the case the cap exists for)."""
    P = make("powerlaw", "small", n=n, p=6, m=20, k=10)
    A = P.A.to_scipy()[::-1][:, ::-1].tocsr()
    P.A = CSR.from_scipy(A)
    return P, P.A.to_scipy()


@pytest.mark.parametrize("cap", [64, 8])
def test_fsai_capped_factor_entry_by_entry(T, cap):
    P, A = _hubs_last()
    lens = _lower_len(A)
    assert lens.max() > 64    # hub rows beyond the local-solve size
    s = T.Solver(P.A, None, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond="fsai", fsai_cap=cap)
    rp, cl, vl = s.factor()
    G = PC.fsai(A, cap=cap)
    assert np.array_equal(rp, G.indptr) and np.array_equal(cl, G.indices)
    scale = np.repeat(np.maximum.reduceat(np.abs(G.data), G.indptr[:-1]), np.diff(G.indptr))
    assert np.max(np.abs(vl - G.data) / scale) < 1e-10
    assert np.array_equal(np.diff(rp), np.minimum(lens, cap))
    # the solve on this factor follows the oracle's
    X0 = start_block(P.A.n, P.k, 12)
    st = s.solve(X0)
    ev, X, res, conv = s.eigpairs()
    s.close()
    ref = O.solve(A, None, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=O.factorized(G))
    assert conv.all() and abs(st["cycles"] - ref.cycles) <= 1
    assert _eig_ok(ev, ref.theta, ref.normA)


def test_fsai_factor_entry_by_entry_on_the_fem_pencil(T):
    """FSAI of the 27-point FEM stiffness matrix (14 lower entries per
    interior row, one dense local solve each; n = 24,389 rows over many
    workgroups) against the oracle's fsai(A), entry by entry (M = G^T G of
    Sec. 2.2 with the FSAI pattern reading R19)."""
    P = make("fem3d", "small", Ne=30, sigma=0.5, p=4, m=16, k=8)
    A = P.A.to_scipy()
    print(f"fsai fem3d n={P.A.n}", flush=True)
    s = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond="fsai")
    rp, cl, vl = s.factor()
    s.close()
    G = PC.fsai(A)
    assert np.array_equal(rp, G.indptr) and np.array_equal(cl, G.indices)
    assert np.diff(rp).max() == 14
    scale = np.repeat(np.maximum.reduceat(np.abs(G.data), G.indptr[:-1]), np.diff(G.indptr))
    assert np.max(np.abs(vl - G.data) / scale) < 1e-10


def test_fsai_without_cap_rejects_hub_rows(T):
    P, _ = _hubs_last()
    with pytest.raises(T.TrplkError) as e:
        T.Solver(P.A, None, p=P.p, m=P.m, k=P.k, precond="fsai", fsai_cap=0)
    assert e.value.code == -1 and "fsai_cap" in str(e.value)
    # a matrix whose rows fit: no cap means the whole lower pattern
    Q = make("lap3d", "small", N=10, p=4, m=16, k=8)
    s = T.Solver(Q.A, None, p=Q.p, m=Q.m, k=Q.k, precond="fsai", fsai_cap=0)
    rp, cl, vl = s.factor()
    s.close()
    G = PC.fsai(Q.A.to_scipy())
    assert np.array_equal(rp, G.indptr) and np.array_equal(cl, G.indices)
    assert np.max(np.abs(vl - G.data)) < 1e-12 * np.max(np.abs(G.data))


# --------------------------------------------------------------------------
# R8: a soft-locked pair unflagged when a lower mode enters
# --------------------------------------------------------------------------

def test_soft_locked_pair_unflagged_parity(T):
    import test_oracle as TO
    Ac, X0 = TO.weak_island_problem()
    A = Ac.to_scipy()
    ref = O.solve(A, None, 2, 12, 4, 1, 1e-8, X0, apply_M=O.jacobi(A), keep_history=True)
    ts = [h[2] for h in ref.history]
    assert any(ts[c] < ts[c - 1] for c in range(1, len(ts)))
    s = T.Solver(Ac, None, p=2, m=12, k=4, l=1, tol=1e-8, precond="jacobi")
    st = s.solve(X0)
    ev, X, res, conv = s.eigpairs()
    s.close()
    print(f"  gpu cycles={st['cycles']} mv={st['matvecs']} oracle {ref.cycles}/{ref.matvecs}",
          flush=True)
    assert (st["cycles"], st["matvecs"]) == (ref.cycles, ref.matvecs) == (20, 164)
    assert conv.all()
    exact = np.linalg.eigvalsh(A.toarray())[:2]
    assert np.all(np.abs(ev - exact) <= 1e-12)


# --------------------------------------------------------------------------
# the largest workload's shape: p = 50 > k = 32, m = 64, hard locking
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def aniso_ref():
    P = make("aniso3d", "small", N=12)   # p50 m64 k32 l1, sigma = 1
    A = P.A.to_scipy()
    X0 = start_block(P.A.n, P.k, 12)
    ref = O.solve(A, None, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=O.jacobi(A))
    return P, X0, ref


@pytest.mark.parametrize("orth,precision", [("delayed", "fp64"), ("cgs2", "fp64"),
                                            ("delayed", "mixed")])
def test_hard_locking_workload_shape_parity(T, aniso_ref, orth, precision):
    """Eigenvalues against the oracle's and the dense spectrum within
    max(1e-10 |theta|, 16 eps ||A||, the certified bound ||r||^2 / gap) of
    each side (R10): at tol 1e-8 a pair is fixed only to ||r||^2 / gap, so
    two solvers that stop at different cycles agree to that bound."""
    P, X0, ref = aniso_ref
    assert (P.p, P.m, P.k) == (50, 64, 32) and P.p > P.k
    print(f"aniso N=12 p50 m64 k32 orth={orth} {precision}", flush=True)
    st, ev, X, res, conv = _pairs(T, P, X0, orth=orth, precision=precision)
    print(f"  gpu cycles={st['cycles']} mv={st['matvecs']} oracle {ref.cycles}/{ref.matvecs} "
          f"max rel={np.max(np.abs(ev - ref.theta) / ref.theta):.2e}", flush=True)
    assert conv.all() and np.all(res <= P.tol * ref.normA * 1.001)
    lam = np.linalg.eigvalsh(P.A.to_scipy().toarray())[:P.p + 1]
    gap = np.minimum(np.abs(np.diff(lam))[:P.p], np.r_[np.inf, np.abs(np.diff(lam))[:P.p - 1]])
    floor = np.maximum(1e-10 * lam[:P.p], 16 * 2.2e-16 * ref.normA)
    b_gpu, b_ref = res ** 2 / gap, ref.true_res ** 2 / gap
    assert np.all(np.abs(ev - lam[:P.p]) <= np.maximum(floor, 1.01 * b_gpu))
    assert np.all(np.abs(ref.theta - lam[:P.p]) <= np.maximum(floor, 1.01 * b_ref))
    assert np.all(np.abs(ev - ref.theta) <= np.maximum(floor, 1.01 * (b_gpu + b_ref)))
    if precision == "fp64":
        assert abs(st["cycles"] - ref.cycles) <= 3
    G = X.T @ X
    assert np.max(np.abs(G - np.eye(P.p))) < 1e-10

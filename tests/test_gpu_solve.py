"""Whole-solve parity of the HIP TRPL+K against the FP64 CPU oracle.

Both sides get byte-identical inputs (the seeded workload generators); the
eigenvalues must agree to 1e-10 relative (or the FP64 floor 16 eps ||A||),
the GPU residuals (recomputed with fresh products) must meet tol * ||A||,
and the cycle counts must agree up to rounding-order effects.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import precond as PC  # noqa: E402
from oracle import trplk as O  # noqa: E402
from workloads import CSR, island_block, lap2d_island, make, start_block  # noqa: E402
from spmv_format import dia_ndiag  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_10128_amd as T
    T.lib()
    return T


def _oracle(P, prec, X0, **kw):
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    if prec == "jacobi":
        M = O.jacobi(A)
    elif prec == "fsai":
        M = O.factorized(PC.fsai(A, kw.pop("cap", None)))
    else:
        M = None
    return O.solve(A, B, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=M, **kw)


def _gpu(T, P, prec, X0, **kw):
    s = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond=prec, **kw)
    st = s.solve(X0)
    ev, X, res, conv = s.eigpairs()
    s.close()
    return st, ev, X, res, conv


def _compare(P, st, ev, X, res, conv, ref, cycle_slack=2, eig_rel=1e-10):
    normA = ref.normA
    floor = 16 * 2.2e-16 * normA
    scale = np.abs(ref.theta)
    if P.B is not None:
        floor = 16 * 2.2e-16 * np.max(np.abs(ref.theta))
    print(f"  gpu cycles={st['cycles']} mv={st['matvecs']}  oracle cycles={ref.cycles} "
          f"mv={ref.matvecs}  max|dtheta|/theta={np.max(np.abs(ev - ref.theta) / scale):.2e} "
          f"max res/normA={np.max(res) / normA:.2e}", flush=True)
    assert conv.all()
    assert np.all(np.abs(ev - ref.theta) <= np.maximum(eig_rel * scale, floor))
    assert np.all(res <= P.tol * normA * 1.001)
    assert abs(st["cycles"] - ref.cycles) <= cycle_slack
    # B-orthonormal eigenvectors
    Bx = X if P.B is None else P.B.to_scipy() @ X
    assert np.max(np.abs(X.T @ Bx - np.eye(X.shape[1]))) < 1e-10


CASES = [
    ("lap2d", dict(N=24), "jacobi", {}),
    ("lap2d", dict(N=64), "jacobi", {}),          # the 64 x 64 workload itself
    ("lap2d", dict(N=30, p=5, m=18, k=8), "none", {}),
    ("lap3d", dict(N=16, vmax=0.05, p=10, m=40, k=20), "jacobi", {}),
    ("lap3d", dict(N=14, vmax=0.05, p=6, m=24, k=12), "fsai", {}),
    ("fem3d", dict(Ne=10, sigma=0.5, p=8, m=24, k=12), "jacobi", {}),
    ("fem3d", dict(Ne=10, sigma=0.5, p=8, m=24, k=12), "fsai", {}),
    ("powerlaw", dict(n=3000, p=8, m=24, k=12), "jacobi", {}),
    ("aniso3d", dict(N=10, sigma=1.0, p=12, m=16, k=8, tol=1e-9), "jacobi", {}),  # hard locking
    ("lap3d", dict(N=12, vmax=0.05, p=8, m=64, k=24), "jacobi", {}),   # largest basis m = 64
    ("lap2d", dict(N=6, p=3, m=36, k=6), "jacobi", {}),                # m = n = 36: one cycle
]


@pytest.mark.parametrize("name,kw,prec,extra", CASES,
                         ids=[f"{c[0]}-{c[2]}-{i}" for i, c in enumerate(CASES)])
def test_solve_parity(T, name, kw, prec, extra):
    P = make(name, "small", **kw)
    print(f"solve {name} {kw} prec={prec} n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, prec, X0)
    st, ev, X, res, conv = _gpu(T, P, prec, X0, **extra)
    # storage of the products: by diagonals for the grid operators that qualify
    assert st["a_ndiag"] == dia_ndiag(P.A)
    assert st["b_ndiag"] == (dia_ndiag(P.B) if P.B is not None else 0)
    if prec == "fsai":  # G has the pattern of tril(A)
        assert st["g_ndiag"] == dia_ndiag(CSR.from_scipy(PC.fsai(P.A.to_scipy())))
    else:
        assert st["g_ndiag"] == 0
    # matvec law on the standard problem: k + (m - k) per cycle (Sec. 5)
    if P.B is None and P.p <= P.k:
        assert st["matvecs"] == P.k + (P.m - P.k) * st["cycles"]
    _compare(P, st, ev, X, res, conv, ref)


def test_mixed_precision_matches_fp64_oracle(T):
    """Float32 SpMV / preconditioner with float64 projection: the final pairs
    still meet the float64 tolerance and match the float64 oracle."""
    P = make("lap3d", "small", N=16, vmax=0.05, p=8, m=32, k=16)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, "fsai", X0)
    st, ev, X, res, conv = _gpu(T, P, "fsai", X0, precision="mixed")
    print(f"  mixed: fp32 cycles {st['fp32_cycles']} of {st['cycles']}", flush=True)
    _compare(P, st, ev, X, res, conv, ref, cycle_slack=10)
    assert st["fp32_cycles"] >= 1


def test_fsai_factor_matches_oracle(T):
    """The factor built on the GPU equals the oracle's FSAI factor: the same
    solve with the oracle's G installed explicitly gives identical results."""
    P = make("fem3d", "small", Ne=8, sigma=0.5, p=4, m=16, k=8)
    A = P.A.to_scipy()
    G = PC.fsai(A)
    X0 = start_block(P.A.n, P.k, 12)
    from workloads.generators import CSR
    s1 = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond="fsai")
    st1 = s1.solve(X0)
    ev1 = s1.eigpairs()[0]
    s2 = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond="jacobi")
    s2.set_factor(CSR.from_scipy(G))
    st2 = s2.solve(X0)
    ev2 = s2.eigpairs()[0]
    assert st1["cycles"] == st2["cycles"]
    assert np.allclose(ev1, ev2, rtol=1e-12)


def test_deterministic(T):
    P = make("lap3d", "small", N=12, vmax=0.05, p=4, m=16, k=8)
    X0 = start_block(P.A.n, P.k, 12)
    a = _gpu(T, P, "jacobi", X0)
    b = _gpu(T, P, "jacobi", X0)
    assert a[0]["cycles"] == b[0]["cycles"]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_device_resident_inputs(T):
    """A, X0 handed over as device pointers (torch tensors): same answer."""
    P = make("lap2d", "small", N=24)
    X0 = start_block(P.A.n, P.k, 12)
    Ad = T.DeviceCSR(P.A)
    Xd = torch.from_numpy(np.ascontiguousarray(X0.T)).cuda()
    s = T.Solver(Ad, None, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol)
    st = s.solve(Xd)
    ev = s.eigpairs()[0]
    _, ev2, _, _, _ = _gpu(T, P, "jacobi", X0)
    assert np.array_equal(ev, ev2)


def test_error_paths(T):
    P = make("lap2d", "small", N=10)
    with pytest.raises(T.TrplkError) as e:
        T.Solver(P.A, None, p=9, m=12, k=8, locking="soft")
    assert e.value.code == -1
    with pytest.raises(T.TrplkError):
        T.Solver(P.A, None, p=2, m=9, k=8, l=1)          # k + l + 1 > m
    s = T.Solver(P.A, None, p=2, m=12, k=4)
    X0 = start_block(P.A.n, 4, 1)
    X0[3, 1] = np.nan
    with pytest.raises(T.TrplkError) as e:
        s.solve(X0)
    assert e.value.code == -4
    X0 = start_block(P.A.n, 4, 1)
    X0[:, 2] = X0[:, 1]                                  # rank deficient
    with pytest.raises(T.TrplkError):
        s.solve(X0)
    s.close()


def test_max_cycles_partial_results(T):
    P = make("lap2d", "small", N=40, p=5, m=18, k=8)
    X0 = start_block(P.A.n, P.k, 12)
    s = T.Solver(P.A, None, p=5, m=18, k=8, max_cycles=3, precond="none")
    st = s.solve(X0)
    assert st["status"] == 1 and st["cycles"] == 3
    ev, X, res, conv = s.eigpairs()
    assert not conv.all() and np.all(np.isfinite(ev))


def test_hard_locking_at_the_column_limit(T):
    """p = m = 64: the locked set plus the basis fill the 128 columns the
    projection passes take; 64 locked pairs and a final 64 x 64
    Rayleigh-Ritz on them.  The cycle count of this case moves with
    rounding: the oracle itself needs 110 cycles from X0 and 112 from X0
    perturbed by 1e-15 relative or from X0 orthonormalised beforehand by
    Cholesky QR (as the GPU's start does), hence the wider cycle slack;
    eigenvalues and residuals keep the usual bounds."""
    P = make("lap3d", "small", N=12, vmax=0.05, p=64, m=64, k=24)
    print(f"solve lap3d N=12 p=64 m=64 k=24 n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, "jacobi", X0)
    st, ev, X, res, conv = _gpu(T, P, "jacobi", X0)
    _compare(P, st, ev, X, res, conv, ref, cycle_slack=6)


@pytest.mark.parametrize("keep", [1e-3, 1e-7])
def test_start_block_cholesky_qr_and_column_fallback(T, keep):
    """k = 8 start vectors, the last one keeping only `keep` of its norm
    outside the span of the others: at 1e-3 the start block is
    orthonormalised by Cholesky QR twice, at 1e-7 (below the Gram route's
    1e-5 limit) column by column; both match the oracle, whose start is
    column-by-column Gram-Schmidt (R2)."""
    P = make("lap2d", "small", N=30, p=4, m=20, k=8)
    X0 = start_block(P.A.n, P.k, 5)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(X0[:, :-1])
    f = rng.standard_normal(P.A.n)
    f -= Q @ (Q.T @ f)
    f -= Q @ (Q.T @ f)
    X0[:, -1] = X0[:, :-1] @ rng.standard_normal(P.k - 1) + keep * np.linalg.norm(X0[:, 0]) * f / np.linalg.norm(f)
    print(f"start block keep={keep} n={P.A.n}", flush=True)
    ref = _oracle(P, "jacobi", X0)
    st, ev, X, res, conv = _gpu(T, P, "jacobi", X0)
    assert st["matvecs"] == P.k + (P.m - P.k) * st["cycles"]
    _compare(P, st, ev, X, res, conv, ref)


@pytest.mark.parametrize("s,k,m,prec", [(6, 4, 12, "jacobi"), (9, 3, 16, "none")])
def test_breakdown_in_an_invariant_subspace(T, s, k, m, prec):
    """A start block inside the s-dimensional invariant subspace of a
    disconnected path: the device detects the breakdown after s - k Krylov
    vectors, skips the rest of the cycle, and returns the exact pairs of the
    path block after one cycle with s products, as the oracle does."""
    A = lap2d_island(20, s)
    n = A.n
    print(f"breakdown island s={s} k={k} m={m} prec={prec} n={n}", flush=True)
    X0 = island_block(n, s, k, 7)
    As = A.to_scipy()
    ref = O.solve(As, None, 2, m, k, 1, 1e-10, X0, apply_M=O.jacobi(As) if prec == "jacobi" else None)
    assert ref.cycles == 1 and ref.matvecs == s
    sv = T.Solver(A, None, p=2, m=m, k=k, l=1, tol=1e-10, precond=prec)
    st = sv.solve(X0)
    ev, X, res, conv = sv.eigpairs()
    sv.close()
    print(f"  gpu cycles={st['cycles']} mv={st['matvecs']} ev={ev} ref={ref.theta}", flush=True)
    assert conv.all()
    assert st["cycles"] == 1 and st["matvecs"] == s
    assert np.all(np.abs(ev - ref.theta) <= 16 * 2.2e-16 * ref.normA)
    assert np.all(X[:n - s] == 0.0)
    assert np.max(np.abs(X.T @ X - np.eye(2))) < 1e-12


@pytest.mark.parametrize("name,kw,prec", [
    ("lap3d", dict(N=16, vmax=0.05, p=10, m=40, k=20), "jacobi"),
    ("powerlaw", dict(n=3000, p=8, m=24, k=12), "jacobi"),
    ("lap3d", dict(N=14, vmax=0.05, p=6, m=24, k=12), "fsai"),
    ("fem3d", dict(Ne=10, sigma=0.5, p=8, m=24, k=12), "jacobi"),
    ("fem3d", dict(Ne=10, sigma=0.5, p=8, m=24, k=12), "fsai"),
    ("aniso3d", dict(N=10, sigma=1.0, p=12, m=16, k=8, tol=1e-9), "jacobi"),   # hard locking
])
def test_delayed_and_cgs2_orthogonalisation_agree(T, name, kw, prec):
    """The inner vectors orthogonalised with both Gram-Schmidt passes before
    the product (three basis passes per step) and with the second pass
    delayed to the next step (two passes, T column and A U corrected from
    small matrices) give the oracle's pairs with the same cycle and product
    counts."""
    P = make(name, "small", **kw)
    print(f"orth {name} {kw} prec={prec} n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, prec, X0)
    out = {}
    for orth in ("cgs2", "delayed"):
        st, ev, X, res, conv = _gpu(T, P, prec, X0, orth=orth)
        assert st["orth_delayed"] == (orth == "delayed")
        _compare(P, st, ev, X, res, conv, ref)
        out[orth] = (st, ev)
    assert abs(out["cgs2"][0]["cycles"] - out["delayed"][0]["cycles"]) <= 1
    assert np.all(np.abs(out["cgs2"][1] - out["delayed"][1]) <= 1e-10 * np.abs(ref.theta))


def test_orth_option_rules(T):
    """AUTO picks the delayed form for TRPL+K (B = I or not, soft or hard
    locking); CGS2 on request."""
    P = make("fem3d", "small", Ne=6, sigma=0.5, p=4, m=16, k=8)
    Q = make("lap2d", "small", N=12)
    X0 = start_block(P.A.n, 8, 12)
    s = T.Solver(P.A, P.B, p=4, m=16, k=8)
    assert s.solve(X0)["orth_delayed"] == 1                      # generalized, soft
    s.close()
    X0 = start_block(Q.A.n, 4, 12)
    s = T.Solver(Q.A, None, p=6, m=16, k=4)
    assert s.solve(X0)["orth_delayed"] == 1                      # hard locking
    s.close()
    s = T.Solver(Q.A, None, p=6, m=16, k=4, orth="cgs2")
    assert s.solve(X0)["orth_delayed"] == 0
    s.close()
    s = T.Solver(Q.A, None, p=2, m=16, k=4)
    assert s.solve(X0)["orth_delayed"] == 1
    s.close()


@pytest.mark.parametrize("l,m,k", [(0, 24, 12), (2, 24, 12), (3, 28, 12), (1, 6, 4)])
def test_delayed_form_plus_k_counts(T, l, m, k):
    """The delayed form with no, one or several +K vectors, and with a single
    Krylov vector per cycle (m = k + l + 1: the first inner vector is
    corrected by the +K vector's pass): cycles, products and pairs match the
    oracle."""
    P = make("lap3d", "small", N=12, vmax=0.05, p=min(4, k), m=m, k=k, l=l)
    print(f"delayed +K l={l} m={m} k={k} n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, "jacobi", X0)
    st, ev, X, res, conv = _gpu(T, P, "jacobi", X0)
    assert st["orth_delayed"] == 1
    _compare(P, st, ev, X, res, conv, ref)


def test_delayed_form_mixed_precision(T):
    """Float32 products in the delayed form: the float64 oracle's pairs."""
    P = make("powerlaw", "small", n=3000, p=8, m=24, k=12)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, "jacobi", X0)
    st, ev, X, res, conv = _gpu(T, P, "jacobi", X0, precision="mixed")
    assert st["orth_delayed"] == 1 and st["fp32_cycles"] >= 1
    _compare(P, st, ev, X, res, conv, ref, cycle_slack=10)


@pytest.mark.parametrize("orth", ["delayed", "cgs2"])
def test_loose_breakdown_tolerance_still_converges(T, orth):
    """A loose breakdown tolerance (0.5) ends many Krylov blocks early,
    also in cycles that append +K vectors after the break (the delayed form
    then finds no pending column to correct); the pairs still match the
    oracle's."""
    P = make("lap3d", "small", N=12, vmax=0.05, p=6, m=24, k=12)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, "jacobi", X0)
    st, ev, X, res, conv = _gpu(T, P, "jacobi", X0, orth=orth, breakdown_tol=0.5)
    print(f"  {orth}: cycles={st['cycles']} mv={st['matvecs']} (oracle {ref.cycles} / {ref.matvecs})",
          flush=True)
    assert conv.all()
    assert np.all(np.abs(ev - ref.theta) <= np.maximum(1e-10 * np.abs(ref.theta), 16 * 2.2e-16 * ref.normA))
    assert np.all(res <= P.tol * ref.normA * 1.001)
    assert st["matvecs"] < P.k + (P.m - P.k) * st["cycles"]   # blocks did end early
    assert np.max(np.abs(X.T @ X - np.eye(X.shape[1]))) < 1e-10


@pytest.mark.parametrize("name,kw,prec,extra,slack", [
    ("fem3d", dict(Ne=8, sigma=0.5, p=10, m=18, k=6), "jacobi", {}, 2),              # B != I, hard
    ("aniso3d", dict(N=10, sigma=1.0, p=12, m=16, k=8, l=0, tol=1e-9), "jacobi", {}, 2),  # hard, l = 0
    ("fem3d", dict(Ne=16, sigma=0.5, p=8, m=24, k=12), "fsai", {"precision": "mixed"}, 10),
    ("aniso3d", dict(N=10, sigma=1.0, p=12, m=16, k=8, tol=1e-9), "jacobi", {"precision": "mixed"}, 40),
])
def test_delayed_form_locking_and_precision_mix(T, name, kw, prec, extra, slack):
    """The delayed form with B != I and hard locking, hard locking without
    +K, and float32 products with B != I and with hard locking: the oracle's
    pairs."""
    P = make(name, "small", **kw)
    print(f"mix {name} {kw} prec={prec} {extra} n={P.A.n}", flush=True)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, prec, X0)
    st, ev, X, res, conv = _gpu(T, P, prec, X0, **extra)
    assert st["orth_delayed"] == 1
    _compare(P, st, ev, X, res, conv, ref, cycle_slack=slack)


def test_mixed_form_switches_when_float32_stalls(T):
    """On a coarse FEM pencil (B entries ~ h^3) the float32 products leave the
    residual far above the switch threshold; the solve must notice the stall,
    continue in float64 and converge to the float64 oracle's pairs."""
    P = make("fem3d", "small", Ne=10, sigma=0.5, p=8, m=24, k=12)
    X0 = start_block(P.A.n, P.k, 12)
    ref = _oracle(P, "fsai", X0)
    st, ev, X, res, conv = _gpu(T, P, "fsai", X0, precision="mixed", max_cycles=400)
    print(f"  fp32 cycles {st['fp32_cycles']} of {st['cycles']} (oracle {ref.cycles})", flush=True)
    assert st["fp32_cycles"] < st["cycles"]
    assert conv.all()
    assert np.all(np.abs(ev - ref.theta) <= 1e-10 * np.abs(ref.theta))

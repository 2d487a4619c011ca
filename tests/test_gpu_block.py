"""Block TRPL+K on the GPU (the block form the paper leaves to future work,
Sec. 5.5; readings B1-B5 in oracle/block.py): the MFMA block passes against
float64 NumPy products on ragged sizes, and whole solves against the block
oracle (soft and hard locking, B = I and B != I, Jacobi and FSAI), block
size 1 being TRPL+K itself."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import block as BL  # noqa: E402
from oracle import precond as PC  # noqa: E402
from oracle import trplk as O  # noqa: E402
from workloads import make, start_block  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_10128_amd as T
    T.lib()
    return T


@pytest.mark.parametrize("vpad", [3, 4], ids=["V-odd-ld", "V-even-ld"])
@pytest.mark.parametrize("n,c,r", [(1, 1, 1), (37, 5, 3), (1000, 17, 16), (12345, 64, 4),
                                   (100_003, 128, 7), (300_001, 40, 1), (70_001, 100, 16),
                                   (50_001, 3, 1), (99_999, 13, 1), (4_097, 16, 1)])
def test_block_passes_against_numpy(T, n, c, r, vpad):
    """An odd leading dimension of V takes the scalar-load form of the dot
    pass, an even one the 16-byte-load form the solver uses; one vector
    against at most 16 columns takes the row-pair pass."""
    print(f"block passes n={n} c={c} r={r} ldv=ld+{vpad}", flush=True)
    rng = np.random.default_rng(n + c + r)
    ld = n + (n % 2)
    U = rng.standard_normal((c, ld))
    V = rng.standard_normal((r, ld + vpad))
    H0 = rng.standard_normal((r, c + 2))
    Ud, Vd = torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()
    Hd = torch.full((r, c + 2), float("nan"), dtype=torch.float64, device="cuda")
    T.block_dot(Ud, Vd, Hd, n=n)
    H = Hd.cpu().numpy()[:, :c].T                    # c x r
    exact = U[:, :n] @ V[:, :n].T
    bound = 2 * n * 2.2e-16 * (np.abs(U[:, :n]) @ np.abs(V[:, :n]).T) + 1e-300
    assert np.all(np.abs(H - exact) <= bound)
    assert np.all(np.isnan(Hd.cpu().numpy()[:, c:]))   # nothing written past c rows of H
    # V += -1 * U H0^T  (H0 holds H as (r, ldh): column v of H is row v)
    Hd2 = torch.from_numpy(H0).cuda()
    T.block_update(Ud, Hd2, Vd, alpha=-1.0, n=n)
    Vn = Vd.cpu().numpy()
    ref = V[:, :n] - (U[:, :n].T @ H0[:, :c].T).T
    bound = 2 * c * 2.2e-16 * (np.abs(V[:, :n]) + (np.abs(U[:, :n]).T @ np.abs(H0[:, :c].T)).T) + 1e-300
    assert np.all(np.abs(Vn[:, :n] - ref) <= bound)
    assert np.array_equal(Vn[:, n:], V[:, n:])          # rows past n untouched


CASES = [
    ("lap2d", dict(N=24), "jacobi", 2),
    ("lap2d", dict(N=24), "jacobi", 4),
    ("lap3d", dict(N=14, vmax=0.05, p=6, m=30, k=12), "fsai", 3),
    ("fem3d", dict(Ne=8, p=6, m=20, k=10), "jacobi", 2),             # B != I
    ("aniso3d", dict(N=10, p=12, m=16, k=8, tol=1e-9), "jacobi", 2),  # hard locking
    ("powerlaw", dict(n=3000, p=8, m=24, k=12), "jacobi", 4),
]


@pytest.mark.parametrize("name,kw,prec,s", CASES, ids=[f"{c[0]}-{c[2]}-s{c[3]}" for c in CASES])
def test_block_solve_parity(T, name, kw, prec, s):
    P = make(name, "small", **kw)
    print(f"block solve {name} s={s} {prec} n={P.A.n}", flush=True)
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    X0 = start_block(P.A.n, P.k, 12)
    M = O.jacobi(A) if prec == "jacobi" else O.factorized(PC.fsai(A))
    ref = BL.solve(A, B, P.p, P.m, P.k, P.l, s, P.tol, X0, apply_M=M)
    S = T.Solver(P.A, P.B, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond=prec, block=s)
    st = S.solve(X0)
    ev, X, res, conv = S.eigpairs()
    S.close()
    print(f"  gpu cycles={st['cycles']} mv={st['matvecs']}  oracle {ref.cycles}/{ref.matvecs} "
          f"max rel={np.max(np.abs(ev - ref.theta) / np.abs(ref.theta)):.2e}", flush=True)
    assert conv.all() and np.all(res <= P.tol * ref.normA * 1.001)
    assert abs(st["cycles"] - ref.cycles) <= 2
    if B is None and P.p <= P.k:
        assert st["matvecs"] == P.k + (P.m - P.k) * st["cycles"]
    scale = ref.normA if B is None else np.max(np.abs(ref.theta))
    assert np.all(np.abs(ev - ref.theta) <= np.maximum(1e-10 * np.abs(ref.theta), 16 * 2.2e-16 * scale))
    Bx = X if B is None else B @ X
    assert np.max(np.abs(X.T @ Bx - np.eye(P.p))) < 1e-10


def test_block_size_one_is_trplk(T):
    P = make("lap2d", "small", N=24)
    X0 = start_block(P.A.n, P.k, 12)
    outs = []
    for blk, orth in ((0, "cgs2"), (1, "cgs2")):
        S = T.Solver(P.A, None, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, block=blk, orth=orth)
        st = S.solve(X0)
        outs.append((st["cycles"], st["matvecs"], S.eigpairs()[0]))
        S.close()
    assert outs[0][:2] == outs[1][:2] and np.array_equal(outs[0][2], outs[1][2])


def test_block_option_rules(T):
    P = make("lap2d", "small", N=12, p=3, m=12, k=4)
    for kw in (dict(block=5), dict(block=2, precision="mixed"), dict(block=2, orth="delayed"),
               dict(block=17)):
        with pytest.raises(T.TrplkError):
            T.Solver(P.A, None, p=P.p, m=P.m, k=P.k, **kw)

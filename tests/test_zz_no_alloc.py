"""trplk_gemv_t_noalloc (static scratch, no allocation) against
trplk_gemv_t (library-allocated scratch) through the C ABI: the same kernels
and summation order, so the coefficients agree bit for bit; both against a
float64 CPU product within the rounding bound of the row sums.  Two calls in
a row, the second with a smaller input, check that nothing the first call
left in the shared scratch leaks into the second."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_10128_amd as T
    T.lib()
    return T


def _case(n, c, ld, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((c, ld))       # column-major n x c, leading dimension ld
    v = rng.standard_normal(ld)
    return U, v


def _run(T, fn, U, v, n):
    Ud = torch.from_numpy(U).cuda()
    vd = torch.from_numpy(v).cuda()
    h = torch.full((U.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    code = fn(n, U.shape[0], T._ptr(Ud), U.shape[1], T._ptr(vd), T._ptr(h), T._stream())
    assert code == 0, T.lib().trplk_last_error(None)
    torch.cuda.synchronize()
    return h.cpu().numpy()


def test_noalloc_matches_allocating_entry_point_two_calls(T):
    L = T.lib()
    # first call: many workgroups (n = 300,001 rows -> 256 dot-pass workgroups),
    # 100 columns; second: a smaller input (3,001 rows, 7 columns)
    for n, c, ld, seed in [(300_001, 100, 300_002, 1), (3_001, 7, 3_002, 2)]:
        print(f"gemv_t_noalloc n={n} c={c}", flush=True)
        U, v = _case(n, c, ld, seed)
        h_na = _run(T, L.trplk_gemv_t_noalloc, U, v, n)
        h_ref = _run(T, L.trplk_gemv_t, U, v, n)
        assert np.array_equal(h_na, h_ref)
        exact = U[:, :n] @ v[:n]
        bound = 4 * n * 2.2e-16 * (np.abs(U[:, :n]) @ np.abs(v[:n]))
        assert np.all(np.abs(h_na - exact) <= bound)


def test_noalloc_rejects_bad_sizes(T):
    L = T.lib()
    good = ctypes.c_void_p(4096)
    assert L.trplk_gemv_t_noalloc(10, 129, good, 10, good, good, None) == -1   # c > 128
    assert L.trplk_gemv_t_noalloc(10, 2, good, 11, good, good, None) == -1     # odd ld
    assert L.trplk_gemv_t_noalloc(0, 2, good, 10, good, good, None) == -1

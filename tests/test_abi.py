"""The C ABI library loads on a machine without a GPU and exports every
function include/trplk.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "trplk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(trplk_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared()
    for n in ("trplk_create", "trplk_solve", "trplk_get_eigpairs", "trplk_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1711_10128_amd as T
    L = T.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(T.EXPORTS) <= set(declared())


def test_default_opts_and_last_error_without_gpu():
    import paper_1711_10128_amd as T
    L = T.lib()
    o = T._Opts()
    L.trplk_default_opts(ctypes.byref(o))
    assert (o.p, o.m, o.k, o.l, o.tol, o.max_cycles) == (1, 18, 8, 1, 1e-8, 5000)
    # argument validation happens before any device call
    ctx = ctypes.c_void_p()
    code = L.trplk_create(ctypes.byref(ctx), None, None, ctypes.byref(o), 0, None)
    assert code == -1 and not ctx.value
    assert b"NULL" in L.trplk_last_error(None)


def test_orth_entries_reject_misaligned_layouts_without_gpu():
    # the Gram-Schmidt passes load row pairs: an odd leading dimension or a
    # pointer off a 16-byte boundary is refused before any device call
    import paper_1711_10128_amd as T
    L = T.lib()
    good, odd = ctypes.c_void_p(4096), ctypes.c_void_p(4104)
    assert L.trplk_gemv_t(10, 2, good, 11, good, good, None) == -1
    assert L.trplk_gemv_t(10, 2, odd, 10, good, good, None) == -1
    assert L.trplk_gemv_t(10, 2, good, 10, odd, good, None) == -1
    assert L.trplk_cgs_update_dot(10, 2, good, 11, good, good, good, None) == -1
    assert L.trplk_cgs_update_dot(10, 2, good, 10, good, odd, good, None) == -1


def test_orth_option_validation_without_gpu():
    # option checks run before anything touches the device
    import numpy as np
    import paper_1711_10128_amd as T
    L = T.lib()
    n = 40
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.full(n, 2.0)
    A = T._Csr(n, n, rp.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
               val.ctypes.data_as(ctypes.c_void_p))
    o = T._Opts()
    L.trplk_default_opts(ctypes.byref(o))
    assert o.orth == T.ORTH["auto"] and o.breakdown_tol == 0.0
    ctx = ctypes.c_void_p()
    o.orth = 3
    assert L.trplk_create(ctypes.byref(ctx), ctypes.byref(A), None, ctypes.byref(o), 0, None) == -1
    assert b"orth" in L.trplk_last_error(None)
    o.orth = 0
    o.breakdown_tol = 1.0
    assert L.trplk_create(ctypes.byref(ctx), ctypes.byref(A), None, ctypes.byref(o), 0, None) == -1
    assert b"breakdown_tol" in L.trplk_last_error(None)
    o.breakdown_tol = 0.0
    assert not ctx.value


def test_splitmix64_start_block_published_outputs():
    """The default start block's generator: SplitMix64 seeded with 0 gives
    0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f first (the
    published outputs of the reference generator); entry e of the block is
    (output_e >> 11) * 2^-52 - 1, column-major."""
    import numpy as np
    from workloads import splitmix64_block
    X = splitmix64_block(3, 1, 0)
    outs = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    want = [(o >> 11) * 2.0 ** -52 - 1.0 for o in outs]
    assert list(X[:, 0]) == want
    Y = splitmix64_block(4, 3, 12)
    assert Y.flags.f_contiguous and Y.shape == (4, 3)
    assert np.all(Y >= -1.0) and np.all(Y < 1.0)
    # column c continues the stream: entry (i, c) is output c * n + i
    assert splitmix64_block(12, 1, 12)[:, 0].tolist() == Y.T.ravel().tolist()


def test_workspace_size_without_gpu():
    """trplk_workspace_size is host arithmetic: W, A W (and B W) with p + m
    columns under hard locking, m otherwise, each column padded to 32
    doubles, the +K block, PL+1's products and the n-vectors, each piece
    rounded to 256 bytes."""
    import paper_1711_10128_amd as T
    L = T.lib()
    o = T._Opts()
    L.trplk_default_opts(ctypes.byref(o))
    assert o.seed == 12
    o.p, o.m, o.k, o.l = 10, 40, 20, 1
    n = 1000
    ld = 1024
    d, f = 8 * ld, 4 * ld
    std = 2 * d * 40 + d + d + 4 * d + 3 * f
    assert L.trplk_workspace_size(n, 0, ctypes.byref(o)) == std
    gen = 3 * d * 40 + d + 2 * d + 5 * d + 3 * f
    assert L.trplk_workspace_size(n, 1, ctypes.byref(o)) == gen
    o.p, o.k = 50, 20   # p > k: hard locking, p + m columns
    assert L.trplk_workspace_size(n, 0, ctypes.byref(o)) == 2 * d * 90 + d + d + 4 * d + 3 * f
    o.m = 65            # invalid options
    assert L.trplk_workspace_size(n, 0, ctypes.byref(o)) == -1
    ctx = ctypes.c_void_p()
    assert L.trplk_create_ws(ctypes.byref(ctx), None, None, ctypes.byref(o), 0, None, None, 0) == -1
    assert not ctx.value

"""Python binding of libtrplk.so, the MI355X (gfx950) TRPL+K eigensolver.

Argument marshalling only: every step of the iteration runs in the HIP
library.  PyTorch supplies device memory and the stream.  Importing this
package does not touch the GPU; the first call that needs the library loads
it and raises if it has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from ._build import LIB

MEM_HOST, MEM_DEVICE = 0, 1
# outer method: TRPL+K (Alg. 1), PL+1 with the conjugate search direction of
# Alg. 2 step 7, PL+1 with the practical direction g_k + p_{k-1} w(m+2)
METHOD = {"trplk": 0, "pl1": 1, "pl1_practical": 2}
# inner-vector orthogonalisation: auto (delayed where it applies), classical
# Gram-Schmidt twice per vector, or the delayed form (second pass merged with
# the next vector's first pass)
ORTH = {"auto": 0, "cgs2": 1, "delayed": 2}
PREC = {"none": 0, "jacobi": 1, "fsai": 2, "factor": 3}
PRECISION = {"fp64": 0, "mixed": 1}
LOCKING = {"auto": 0, "soft": 1, "hard": 2}
NORM = {"inf": 0, "fro": 1}
STATUS = {0: "OK", 1: "ENOCONV", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTSPD", -4: "ENUMERIC",
          -5: "EDEVICE"}


class TrplkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("l", ctypes.c_int32), ("tol", ctypes.c_double), ("norm", ctypes.c_int32),
                ("max_cycles", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("locking", ctypes.c_int32),
                ("fsai_cap", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("mixed_switch", ctypes.c_double), ("fallback_window", ctypes.c_int32),
                ("method", ctypes.c_int32), ("orth", ctypes.c_int32),
                ("breakdown_tol", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("progress", ctypes.c_int32), ("block", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("nconv", ctypes.c_int32),
                ("matvecs", ctypes.c_int64), ("bmatvecs", ctypes.c_int64),
                ("precs", ctypes.c_int64), ("fp32_cycles", ctypes.c_int32),
                ("status", ctypes.c_int32), ("fallback_cycle", ctypes.c_int32),
                ("orth_delayed", ctypes.c_int32), ("normA", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("spmv_ms", ctypes.c_double), ("spmv_launches", ctypes.c_int64),
                ("spmv_bytes", ctypes.c_int64),
                ("orth_ms", ctypes.c_double), ("orth_launches", ctypes.c_int64),
                ("orth_bytes", ctypes.c_int64),
                ("prec_ms", ctypes.c_double), ("prec_launches", ctypes.c_int64),
                ("prec_bytes", ctypes.c_int64),
                ("rot_ms", ctypes.c_double), ("rot_launches", ctypes.c_int64),
                ("rot_bytes", ctypes.c_int64),
                ("rr_ms", ctypes.c_double), ("rr_launches", ctypes.c_int64),
                ("pass_ms", ctypes.c_double * 5), ("pass_launches", ctypes.c_int64 * 5),
                ("pass_bytes", ctypes.c_int64 * 5),
                ("a_ndiag", ctypes.c_int32), ("b_ndiag", ctypes.c_int32),
                ("g_ndiag", ctypes.c_int32), ("pad_", ctypes.c_int32)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if not isinstance(v, (int, float)) else v
        return d


_lib = None

EXPORTS = ["trplk_default_opts", "trplk_create", "trplk_workspace_size", "trplk_create_ws",
           "trplk_set_factor", "trplk_solve",
           "trplk_get_eigpairs", "trplk_device_bytes", "trplk_last_error", "trplk_destroy",
           "trplk_spmv", "trplk_spmv_f32", "trplk_gemv_t", "trplk_cgs_update_dot", "trplk_syev",
           "trplk_rotate", "trplk_learned_factor", "trplk_factor_nnz", "trplk_factor_values",
           "trplk_factor_loss_grad", "trplk_train_step", "trplk_get_factor",
           "trplk_gemv_t_noalloc", "trplk_get_history", "trplk_block_dot", "trplk_block_update",
           "trplk_spmm"]
MLP_NPARAM = 1217
MLP_NF, MLP_NIN, MLP_NH = 8, 17, 64


def lib():
    """Load libtrplk.so (built by __graft_entry__.build()); raise if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise ImportError(f"{LIB} is not built; run __graft_entry__.build() first "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.trplk_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    L.trplk_default_opts.restype = None
    L.trplk_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Csr), ctypes.POINTER(_Csr),
                               ctypes.POINTER(_Opts), i32, vp]
    L.trplk_create.restype = ctypes.c_int
    L.trplk_workspace_size.argtypes = [i32, i32, ctypes.POINTER(_Opts)]
    L.trplk_workspace_size.restype = i64
    L.trplk_create_ws.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Csr), ctypes.POINTER(_Csr),
                                  ctypes.POINTER(_Opts), i32, vp, vp, i64]
    L.trplk_create_ws.restype = ctypes.c_int
    L.trplk_set_factor.argtypes = [vp, ctypes.POINTER(_Csr), i32]
    L.trplk_set_factor.restype = ctypes.c_int
    L.trplk_solve.argtypes = [vp, vp, i32, ctypes.POINTER(_Stats)]
    L.trplk_solve.restype = ctypes.c_int
    L.trplk_get_eigpairs.argtypes = [vp, vp, vp, vp, vp, i32]
    L.trplk_get_eigpairs.restype = ctypes.c_int
    L.trplk_device_bytes.argtypes = [vp]
    L.trplk_device_bytes.restype = i64
    L.trplk_last_error.argtypes = [vp]
    L.trplk_last_error.restype = ctypes.c_char_p
    L.trplk_destroy.argtypes = [vp]
    L.trplk_destroy.restype = None
    L.trplk_spmv.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp]
    L.trplk_spmv_f32.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp]
    L.trplk_spmm.argtypes = [i32, vp, vp, vp, vp, i64, i32, vp, i64, vp]
    L.trplk_gemv_t.argtypes = [i32, i32, vp, i64, vp, vp, vp]
    L.trplk_gemv_t_noalloc.argtypes = [i32, i32, vp, i64, vp, vp, vp]
    L.trplk_cgs_update_dot.argtypes = [i32, i32, vp, i64, vp, vp, vp, vp]
    L.trplk_syev.argtypes = [i32, vp, vp, vp, vp]
    L.trplk_block_dot.argtypes = [i32, i32, vp, i64, vp, i64, i32, vp, i32, vp]
    L.trplk_block_update.argtypes = [i32, i32, vp, i64, vp, i32, i32, ctypes.c_double, vp, i64, vp]
    L.trplk_rotate.argtypes = [i32, i32, i32, vp, i64, vp, i32, vp]
    for f in ("trplk_spmv", "trplk_spmv_f32", "trplk_spmm", "trplk_gemv_t", "trplk_gemv_t_noalloc",
              "trplk_cgs_update_dot", "trplk_block_dot", "trplk_block_update",
              "trplk_syev", "trplk_rotate"):
        getattr(L, f).restype = ctypes.c_int
    L.trplk_learned_factor.argtypes = [vp, vp]
    L.trplk_learned_factor.restype = ctypes.c_int
    L.trplk_factor_nnz.argtypes = [vp]
    L.trplk_factor_nnz.restype = i64
    L.trplk_factor_values.argtypes = [vp, vp, i32]
    L.trplk_factor_values.restype = ctypes.c_int
    L.trplk_factor_loss_grad.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp]
    L.trplk_factor_loss_grad.restype = ctypes.c_int
    L.trplk_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_double, i32, vp, vp]
    L.trplk_train_step.restype = ctypes.c_int
    L.trplk_get_history.argtypes = [vp, vp, i32]
    L.trplk_get_history.restype = i32
    L.trplk_get_factor.argtypes = [vp, vp, vp, vp, i32]
    L.trplk_get_factor.restype = i64
    _lib = L
    return L


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check(code, ctx=None):
    if code < 0:
        msg = lib().trplk_last_error(ctx).decode(errors="replace")
        raise TrplkError(code, msg)
    return code


class DeviceCSR:
    """A CSR matrix held in torch device tensors (int32 / int32 / float64)."""

    def __init__(self, csr, device="cuda"):
        import torch
        self.n = int(csr.n)
        self.nnz = int(csr.col.shape[0])
        self.rowptr = torch.from_numpy(np.ascontiguousarray(csr.rowptr, dtype=np.int32)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(csr.col, dtype=np.int32)).to(device)
        self.val = torch.from_numpy(np.ascontiguousarray(csr.val, dtype=np.float64)).to(device)

    def c(self):
        return _Csr(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr())


def _host_csr(csr, keep):
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(csr.col, dtype=np.int32)
    vl = np.ascontiguousarray(csr.val, dtype=np.float64)
    keep.extend([rp, cl, vl])
    return _Csr(int(csr.n), int(cl.shape[0]), rp.ctypes.data, cl.ctypes.data, vl.ctypes.data)


class Solver:
    """One TRPL+K context on the current HIP device.

    A, B       CSR matrices: objects with n/rowptr/col/val numpy arrays (copied
               to the device by the library) or DeviceCSR (referenced)
    seed       start block drawn on the device when solve() gets no X0
    workspace  True: the n-length solver workspace is a torch tensor owned
               here and handed to trplk_create_ws (the library allocates the
               rest); False: the library allocates everything
    """

    def __init__(self, A, B=None, *, p, m, k, l=1, tol=1e-8, precond="jacobi",
                 precision="fp64", locking="auto", norm="inf", max_cycles=5000, fsai_cap=0,
                 profile=False, mixed_switch=0.0, fallback_window=0, method="trplk",
                 orth="auto", breakdown_tol=0.0, seed=12, workspace=False, progress=0,
                 block=0):
        L = lib()
        o = _Opts()
        L.trplk_default_opts(ctypes.byref(o))
        o.p, o.m, o.k, o.l, o.tol = p, m, k, l, tol
        o.norm, o.max_cycles = NORM[norm], max_cycles
        o.precond, o.precision, o.locking = PREC[precond], PRECISION[precision], LOCKING[locking]
        o.fsai_cap, o.profile, o.mixed_switch = fsai_cap, int(bool(profile)), mixed_switch
        o.fallback_window = fallback_window
        o.method = METHOD[method]
        o.orth = ORTH[orth]
        o.breakdown_tol = breakdown_tol
        o.seed = seed
        o.progress = progress
        o.block = block
        self.opts = o
        self.n = int(A.n)
        self.p = p
        self.k = k
        keep = []
        dev = isinstance(A, DeviceCSR)
        if dev:
            ca, cb = A.c(), (B.c() if B is not None else None)
        else:
            ca = _host_csr(A, keep)
            cb = _host_csr(B, keep) if B is not None else None
        self._refs = (A, B)
        ctx = ctypes.c_void_p()
        self.workspace = None
        if workspace:
            import torch
            nbytes = int(L.trplk_workspace_size(self.n, int(B is not None), ctypes.byref(o)))
            if nbytes < 0:
                raise TrplkError(-1, "invalid options for trplk_workspace_size")
            # torch's caching allocator returns 512-byte aligned blocks
            self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
            code = L.trplk_create_ws(ctypes.byref(ctx), ctypes.byref(ca),
                                     ctypes.byref(cb) if cb is not None else None,
                                     ctypes.byref(o), MEM_DEVICE if dev else MEM_HOST, _stream(),
                                     _ptr(self.workspace), nbytes)
        else:
            code = L.trplk_create(ctypes.byref(ctx), ctypes.byref(ca),
                                  ctypes.byref(cb) if cb is not None else None, ctypes.byref(o),
                                  MEM_DEVICE if dev else MEM_HOST, _stream())
        _check(code, None)
        self.ctx = ctx
        self.stats = None

    def set_factor(self, G):
        """Install M = G^T G for a lower-triangular CSR G (numpy arrays)."""
        keep = []
        cg = _host_csr(G, keep)
        _check(lib().trplk_set_factor(self.ctx, ctypes.byref(cg), MEM_HOST), self.ctx)

    def solve(self, X0=None):
        """Run the solver from the start block X0 (n x k): numpy (column-major
        is produced here), a torch device tensor holding the column-major
        block as a contiguous (k, n) tensor (PL+1: (1, n) or more rows), or
        None (the block is drawn on the device from the seed)."""
        import torch
        st = _Stats()
        if X0 is None:
            code = lib().trplk_solve(self.ctx, None, MEM_HOST, ctypes.byref(st))
        elif isinstance(X0, torch.Tensor):
            cols = self.k if self.opts.method == METHOD["trplk"] else 1
            if not (X0.is_cuda and X0.dtype == torch.float64 and X0.is_contiguous()
                    and X0.dim() == 2 and X0.shape[1] == self.n and X0.shape[0] >= cols):
                raise ValueError(f"X0 must be a contiguous float64 CUDA tensor of shape "
                                 f"({cols}, {self.n}) (the column-major n x {cols} block)")
            code = lib().trplk_solve(self.ctx, _ptr(X0), MEM_DEVICE, ctypes.byref(st))
        else:
            X = np.asfortranarray(X0, dtype=np.float64)
            if X.shape != (self.n, self.k):
                raise ValueError(f"X0 must be {self.n} x {self.k}")
            code = lib().trplk_solve(self.ctx, X.ctypes.data_as(ctypes.c_void_p), MEM_HOST,
                                     ctypes.byref(st))
        _check(code, self.ctx)
        self.stats = st.as_dict()
        return self.stats

    def eigpairs(self, vectors=True, residuals=True):
        p, n = self.p, self.n
        ev = np.empty(p)
        X = np.empty((p, n)) if vectors else None
        rs = np.empty(p) if residuals else None
        cv = np.empty(p, dtype=np.int32)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None  # noqa: E731
        _check(lib().trplk_get_eigpairs(self.ctx, vp(ev), vp(X), vp(rs), vp(cv), MEM_HOST), self.ctx)
        return ev, (X.T if X is not None else None), rs, cv.astype(bool)

    # ---- learned factor (M = G^T G, G predicted by the MLP) ----
    def learned_factor(self, params):
        """Evaluate the MLP (params: TRPLK_MLP_NPARAM float32) and install M = G^T G."""
        P = np.ascontiguousarray(params, dtype=np.float32)
        assert P.shape == (MLP_NPARAM,)
        _check(lib().trplk_learned_factor(self.ctx, P.ctypes.data_as(ctypes.c_void_p)), self.ctx)

    def factor_values(self):
        nnz = int(lib().trplk_factor_nnz(self.ctx))
        v = np.empty(nnz)
        _check(lib().trplk_factor_values(self.ctx, v.ctypes.data_as(ctypes.c_void_p), MEM_HOST),
               self.ctx)
        return v

    def factor_loss_grad(self, params, E, R):
        P = np.ascontiguousarray(params, dtype=np.float32)
        E = np.asfortranarray(E, dtype=np.float64)
        R = np.asfortranarray(R, dtype=np.float64)
        loss = ctypes.c_double()
        grad = np.empty(MLP_NPARAM)
        vp = ctypes.c_void_p
        _check(lib().trplk_factor_loss_grad(self.ctx, P.ctypes.data_as(vp), E.shape[1],
                                            E.ctypes.data_as(vp), R.ctypes.data_as(vp), MEM_HOST,
                                            ctypes.byref(loss), grad.ctypes.data_as(vp)), self.ctx)
        return loss.value, grad

    def train_step(self, params, m, v, step, lr, S, grad=None):
        """One Adam step on the pairs of the last solve; arrays updated in
        place.  grad: optional float64 array that receives the gradient."""
        loss = ctypes.c_double()
        vp = ctypes.c_void_p
        for a in (params, m, v):
            assert a.dtype == np.float32 and a.flags.c_contiguous and a.shape == (MLP_NPARAM,)
        if grad is not None:
            assert grad.dtype == np.float64 and grad.flags.c_contiguous and grad.shape == (MLP_NPARAM,)
        _check(lib().trplk_train_step(self.ctx, params.ctypes.data_as(vp), m.ctypes.data_as(vp),
                                      v.ctypes.data_as(vp), step, lr, S, ctypes.byref(loss),
                                      grad.ctypes.data_as(vp) if grad is not None else None),
               self.ctx)
        return loss.value

    def history(self):
        """Smallest active Ritz value after each restart cycle of the last solve."""
        nc = _check(int(lib().trplk_get_history(self.ctx, None, 0)), self.ctx)
        h = np.empty(max(nc, 1))
        _check(int(lib().trplk_get_history(self.ctx, h.ctypes.data_as(ctypes.c_void_p), nc)),
               self.ctx)
        return h[:nc]

    def factor(self):
        """The installed factor G (M = G^T G) as (rowptr, col, val) numpy arrays."""
        nnz = _check(int(lib().trplk_get_factor(self.ctx, None, None, None, MEM_HOST)), self.ctx)
        rp = np.empty(self.n + 1, dtype=np.int32)
        cl = np.empty(max(nnz, 1), dtype=np.int32)
        vl = np.empty(max(nnz, 1))
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(int(lib().trplk_get_factor(self.ctx, vp(rp), vp(cl), vp(vl), MEM_HOST)), self.ctx)
        return rp, cl[:nnz], vl[:nnz]

    def device_bytes(self):
        return int(lib().trplk_device_bytes(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            lib().trplk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# kernel-level wrappers (torch device tensors in, results in place)
# ---------------------------------------------------------------------------

def spmv(rowptr, col, val, x, y, lanes=0):
    import torch
    f = lib().trplk_spmv if val.dtype == torch.float64 else lib().trplk_spmv_f32
    _check(f(int(rowptr.shape[0] - 1), _ptr(rowptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y),
             lanes, _stream()))
    return y


def spmm(rowptr, col, val, X, Y):
    """Y = A X for X, Y given as (ncols, ld) contiguous float64 tensors
    (column-major n x ncols blocks, ld >= n); ncols <= 16."""
    ncols, ldx = X.shape
    _check(lib().trplk_spmm(int(rowptr.shape[0] - 1), _ptr(rowptr), _ptr(col), _ptr(val), _ptr(X), ldx,
                            ncols, _ptr(Y), Y.shape[1], _stream()))
    return Y


def gemv_t(U, v, h, n=None):
    """h = U^T v for U given as a (c, ld) contiguous tensor (column-major
    ld x c, the first n rows used; ld even)."""
    c, ld = U.shape
    n = ld if n is None else n
    _check(lib().trplk_gemv_t(n, c, _ptr(U), ld, _ptr(v), _ptr(h), _stream()))
    return h


def gemv_t_noalloc(U, v, h, n=None):
    """gemv_t through the entry point that allocates nothing (static scratch)."""
    c, ld = U.shape
    n = ld if n is None else n
    _check(lib().trplk_gemv_t_noalloc(n, c, _ptr(U), ld, _ptr(v), _ptr(h), _stream()))
    return h


def block_dot(U, V, H, n=None):
    """H = U^T V; U (c, ldu), V (r, ldv), H (r, ldh) contiguous tensors holding
    column-major blocks (the first n rows used)."""
    c, ldu = U.shape
    r, ldv = V.shape
    n = ldu if n is None else n
    _check(lib().trplk_block_dot(n, c, _ptr(U), ldu, _ptr(V), ldv, r, _ptr(H), H.shape[1],
                                 _stream()))
    return H


def block_update(U, H, V, alpha=-1.0, n=None):
    """V += alpha U H (same layouts as block_dot)."""
    c, ldu = U.shape
    r, ldv = V.shape
    n = ldu if n is None else n
    _check(lib().trplk_block_update(n, c, _ptr(U), ldu, _ptr(H), H.shape[1], r, alpha, _ptr(V), ldv,
                                    _stream()))
    return V


def cgs_update_dot(U, h, w, h2, n=None):
    c, ld = U.shape
    n = ld if n is None else n
    _check(lib().trplk_cgs_update_dot(n, c, _ptr(U), ld, _ptr(h), _ptr(w), _ptr(h2), _stream()))
    return w, h2


def syev(T, theta, Y):
    """T, Y: (b, b) contiguous tensors holding column-major matrices."""
    b = T.shape[0]
    _check(lib().trplk_syev(b, _ptr(T), _ptr(theta), _ptr(Y), _stream()))
    return theta, Y


def rotate(U, Y, k):
    """U: (b, n) contiguous tensor (column-major n x b), Y: (b, b) column-major."""
    b, n = U.shape
    _check(lib().trplk_rotate(n, b, k, _ptr(U), n, _ptr(Y), b, _stream()))
    return U


def pack_params(W1, b1, w2, b2):
    """Flat float32 parameter vector: W1 (64 x 17 row-major), b1, w2, b2."""
    return np.concatenate([np.asarray(W1, dtype=np.float64).ravel(), np.ravel(b1), np.ravel(w2),
                           np.ravel(b2)]).astype(np.float32)


def unpack_params(P):
    P = np.asarray(P, dtype=np.float64)
    k = MLP_NH * MLP_NIN
    return {"W1": P[:k].reshape(MLP_NH, MLP_NIN), "b1": P[k:k + MLP_NH],
            "w2": P[k + MLP_NH:k + 2 * MLP_NH], "b2": P[k + 2 * MLP_NH]}


def init_params(seed=0):
    """He-scaled first layer, zero output layer (the factor starts as Jacobi)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((MLP_NH, MLP_NIN)) * np.sqrt(2.0 / MLP_NIN)
    return pack_params(W1, np.zeros(MLP_NH), np.zeros(MLP_NH), 0.0)


def train(solvers, X0s, epochs, lr=1e-3, S=24, params=None, log=None):
    """Train the factor's MLP on the GPU: solve each instance once (Jacobi or
    whatever preconditioner its Solver holds) to harvest pairs (u, A u) from
    its basis, then full-batch Adam over the instances for `epochs` epochs.
    A Solver whose max_cycles stops it after a cycle or two contributes the
    rough early Krylov vectors; pairing those with a converged solve of the
    same instance constrains the rows that converged vectors barely touch."""
    P = init_params() if params is None else np.array(params, dtype=np.float32)
    m = np.zeros(MLP_NPARAM, dtype=np.float32)
    v = np.zeros(MLP_NPARAM, dtype=np.float32)
    for s, X0 in zip(solvers, X0s):
        s.solve(X0)
    step = 0
    hist = []
    for ep in range(epochs):
        tot = 0.0
        for s in solvers:
            step += 1
            tot += s.train_step(P, m, v, step, lr, S)
        hist.append(tot / len(solvers))
        if log and ep % 25 == 0:
            log(f"epoch {ep} loss {hist[-1]:.5f}")
    return P, hist

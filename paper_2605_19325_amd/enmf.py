"""Python binding of libenmf (ctypes).  Argument marshalling only.

Every computation runs in the HIP kernels of libenmf.so; PyTorch supplies
device memory and the current stream.  The names mirror the C ABI in
include/enmf.h.  There is no CPU fallback: a missing library, a tensor that
is not on the GPU or a failing call raises.
"""

import ctypes
import os
from ctypes import POINTER, Structure, byref, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libenmf.so")

F32, BF16, F16, CSR = 0, 1, 2, 3
_DTYPES = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}
MAX_RANK = 64
MAX_WIDTH = 80
TRACE_FIELDS = 8


class EnmfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"enmf status {status}: {message}")
        self.status = status


class Matrix(Structure):
    _fields_ = [("data", c_void_p), ("m", c_int64), ("n", c_int64), ("ld", c_int64),
                ("dtype", c_int32), ("reserved", c_int32)]


class SvdOpts(Structure):
    _fields_ = [("omega", c_void_p), ("oversample", c_int32), ("power_iters", c_int32)]


class RotateOpts(Structure):
    _fields_ = [("rho0", c_double), ("tol", c_double), ("max_iter", c_int32),
                ("check_every", c_int32)]


class GrotOpts(Structure):
    _fields_ = [("rho0", c_double), ("tol", c_double), ("max_iter", c_int32), ("reserved", c_int32)]


class MaskArg(Structure):
    _fields_ = [("bits", c_void_p), ("ld_words", c_int64)]


class IterOpts(Structure):
    _fields_ = [("step_u", c_double), ("step_v", c_double), ("pbcd_eps", c_double),
                ("relerr_tol", c_double), ("kkt_tol", c_double), ("relerr_svd", c_double),
                ("ext_iters", c_int32), ("pbcd_max_iter", c_int32), ("max_iter", c_int32),
                ("check_every", c_int32), ("mode", c_int32), ("graph_replay", c_int32)]


class IterReport(Structure):
    _fields_ = [("iters", c_int32), ("ext_iters_done", c_int32), ("phase", c_int32),
                ("converged", c_int32), ("step_u", c_double), ("step_v", c_double),
                ("f", c_double), ("relerr", c_double), ("re_paper", c_double), ("kkt", c_double),
                ("kkt_feas", c_double), ("kkt_pg_u", c_double), ("kkt_pg_v", c_double),
                ("delta_w", c_double), ("sigma_w", c_double)]


class Kkt(Structure):
    _fields_ = [(k, c_double) for k in ("f", "relerr", "re_paper", "kkt", "kkt_feas", "kkt_pg_u",
                                        "kkt_pg_v", "delta_w", "sigma_w", "sigma_u", "sigma_v",
                                        "min_w")]


class ServeOpts(Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", c_int32),
                ("tick_time_us", c_int32), ("ticks_per_launch", c_int32), ("direct_launch", c_int32),
                ("wide_min_elems", ctypes.c_int64), ("wide_lanes", c_int32), ("reserved", c_int32)]


class Request(Structure):
    _fields_ = [("X", Matrix), ("r", c_int32), ("reserved", c_int32), ("svd", SvdOpts),
                ("rot", RotateOpts), ("it", IterOpts), ("U_out", c_void_p), ("V_out", c_void_p)]


_lib = None

# (name, restype, argtypes) of every exported entry point.
SIGNATURES = [
    ("enmf_version", c_int32, []),
    ("enmf_status_string", c_char_p, [c_int32]),
    ("enmf_create", c_int32, [POINTER(c_void_p), c_int32, c_void_p]),
    ("enmf_destroy", None, [c_void_p]),
    ("enmf_last_error", c_char_p, [c_void_p]),
    ("enmf_set_stream", c_int32, [c_void_p, c_void_p]),
    ("enmf_synchronize", c_int32, [c_void_p]),
    ("enmf_convert", c_int32, [c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int32, c_void_p,
                               c_int64]),
    ("enmf_xv", c_int32, [c_void_p, POINTER(Matrix), c_void_p, c_int32, c_void_p]),
    ("enmf_xv_static", c_int32, [c_void_p, POINTER(Matrix), c_void_p, c_int32, c_void_p]),
    ("enmf_xtu", c_int32, [c_void_p, POINTER(Matrix), c_void_p, c_int32, c_void_p]),
    ("enmf_gram", c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p]),
    ("enmf_svd_init", c_int32, [c_void_p, POINTER(Matrix), c_int32, POINTER(SvdOpts), c_void_p,
                                c_void_p, POINTER(c_double), POINTER(c_double)]),
    ("enmf_rotate", c_int32, [c_void_p, c_int64, c_int64, c_int32, c_void_p, c_void_p,
                              POINTER(RotateOpts), POINTER(c_double), POINTER(c_int32),
                              POINTER(c_double), POINTER(c_double)]),
    ("enmf_rotate_general", c_int32, [c_void_p, c_int64, c_int64, c_int32, c_void_p, c_void_p,
                                      POINTER(GrotOpts), POINTER(c_double), POINTER(c_double),
                                      POINTER(c_double), POINTER(c_int32), POINTER(c_double),
                                      POINTER(c_double)]),
    ("enmf_iterate", c_int32, [c_void_p, POINTER(Matrix), c_int32, c_void_p, c_void_p,
                               POINTER(IterOpts), POINTER(IterReport), c_void_p, c_int32]),
    ("enmf_objective_kkt", c_int32, [c_void_p, POINTER(Matrix), c_int32, c_void_p, c_void_p,
                                     c_double, POINTER(Kkt)]),
    ("enmf_sparse_create", c_int32, [c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p,
                                     c_void_p, POINTER(c_void_p)]),
    ("enmf_sparse_destroy", None, [c_void_p]),
    ("enmf_enmc_init", c_int32, [c_void_p, POINTER(Matrix), POINTER(MaskArg), c_int32,
                                 POINTER(SvdOpts), c_int32, c_void_p, c_void_p, POINTER(c_double)]),
    ("enmf_enmc_grad", c_int32, [c_void_p, POINTER(Matrix), POINTER(MaskArg), c_int32, c_void_p,
                                 c_void_p, c_void_p, c_void_p, POINTER(c_double)]),
    ("enmf_enmc_iterate", c_int32, [c_void_p, POINTER(Matrix), POINTER(MaskArg), c_int32, c_void_p,
                                    c_void_p, POINTER(IterOpts), POINTER(IterReport)]),
    ("enmf_time_products", c_int32, [c_void_p, POINTER(Matrix), c_int32, c_int32,
                                     POINTER(c_double), POINTER(c_double)]),
    ("enmf_kernel_timing", c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                     POINTER(c_int32)]),
    ("enmf_serve_start", c_int32, [c_void_p, POINTER(ServeOpts), POINTER(c_void_p)]),
    ("enmf_serve_submit", c_int32, [c_void_p, POINTER(Request), POINTER(ctypes.c_uint64)]),
    ("enmf_serve_poll", c_int32, [c_void_p, ctypes.c_uint64, POINTER(IterReport),
                                  POINTER(c_double)]),
    ("enmf_serve_stop", c_int32, [c_void_p]),
    ("enmf_serve_last_error", c_char_p, [c_void_p]),
]


def load_library(path=LIB_PATH):
    """Load libenmf.so and declare its signatures (no device call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    return c_void_p(t.data_ptr())


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    return t


def _factor(t, rows, r, name):
    _dev(t, name)
    if t.dtype != torch.float32 or tuple(t.shape) != (rows, r) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor of shape ({rows}, {r})")
    return t


class SparseX:
    """A sparse X on the device (enmf_sparse handle), made by Context.sparse.

    Accepted wherever the calls take X (products, svd_init, iterate,
    objective_kkt, solve, time_products); `shape`, `nnz` and `device` mirror
    a dense tensor's.
    """

    def __init__(self, lib, handle, m, n, nnz, device):
        self._lib = lib
        self._h = handle
        self.shape = (m, n)
        self.nnz = nnz
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            self._lib.enmf_sparse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def matrix(X):
    """enmf_matrix view of a 2-D row-major CUDA tensor (float32, bfloat16 or
    float16) or of a SparseX."""
    if isinstance(X, SparseX):
        if not X._h:
            raise ValueError("sparse X has been closed")
        return Matrix(X._h.value, X.shape[0], X.shape[1], 0, CSR, 0)
    _dev(X, "X")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D tensor with unit column stride")
    if X.dtype not in _DTYPES:
        raise ValueError("X dtype must be float32, bfloat16 or float16")
    return Matrix(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0), _DTYPES[X.dtype], 0)


def pitched(X):
    """Copy of a 2-D CUDA tensor whose rows start on 128-byte lines (leading
    dimension rounded up to 128 bytes), returned as the m x n view.  Rows of a
    pitch that is an odd multiple of 64 bytes (n = 10000 in float32, n = 20000
    in 16-bit storage) make every other row's runs straddle one more line
    than they cover, and the streaming products fetch those lines too."""
    _dev(X, "X")
    if X.dim() != 2:
        raise ValueError("X must be a 2-D tensor")
    m, n = X.shape
    per = 128 // X.element_size()
    ld = (n + per - 1) // per * per
    buf = torch.empty((m, ld), dtype=X.dtype, device=X.device)
    out = buf[:, :n]
    out.copy_(X)
    return out


def pack_mask(observed):
    """Bit mask of the observed entries in the layout of enmf_mask: bit j % 32
    of word [i][j / 32] (numpy bool array in, int32 numpy array of shape
    (m, ceil(n / 32)) out).  Layout only: no arithmetic of the method."""
    obs = np.asarray(observed, dtype=bool)
    m, n = obs.shape
    words = (n + 31) // 32
    pad = np.zeros((m, words * 32), dtype=bool)
    pad[:, :n] = obs
    packed = np.packbits(pad, axis=1, bitorder="little")
    return np.ascontiguousarray(packed).view("<u4").view(np.int32).reshape(m, words)


def _mask(mask_words, m, n):
    words = (n + 31) // 32
    if (mask_words.dtype != torch.int32 or mask_words.dim() != 2 or mask_words.shape[0] != m or
            mask_words.shape[1] < words or mask_words.stride(1) != 1 or not mask_words.is_cuda):
        raise ValueError("mask must be an int32 device tensor of shape (m, >= ceil(n/32))")
    return MaskArg(mask_words.data_ptr(), mask_words.stride(0))


class Context:
    """One libenmf context on a device; calls enqueue on torch's current stream."""

    def __init__(self, device=0):
        self._lib = load_library()
        self.device = device
        h = c_void_p()
        st = self._lib.enmf_create(byref(h), device, None)
        if st != 0:
            raise EnmfError(st, self._lib.enmf_status_string(st).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.enmf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        self._lib.enmf_set_stream(self._h, c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        st = fn(self._h, *args)
        if st != 0:
            raise EnmfError(st, self._lib.enmf_last_error(self._h).decode())

    def synchronize(self):
        self._call(self._lib.enmf_synchronize)

    def sparse(self, rowptr, colind, vals, shape):
        """Upload a compressed-sparse-row X (host arrays: int64 rowptr of m + 1
        offsets, int32 column indices increasing within each row, float32
        values) to this context's device."""
        m, n = int(shape[0]), int(shape[1])
        rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        ci = np.ascontiguousarray(colind, dtype=np.int32)
        vv = np.ascontiguousarray(vals, dtype=np.float32)
        if rp.ndim != 1 or rp.size != m + 1 or ci.ndim != 1 or vv.ndim != 1 or ci.size != vv.size:
            raise ValueError("rowptr must hold m + 1 offsets and colind, vals nnz entries each")
        h = c_void_p()
        torch.cuda.current_stream(self.device).synchronize()
        self._call(self._lib.enmf_sparse_create, m, n, int(ci.size), rp.ctypes.data_as(c_void_p),
                   ci.ctypes.data_as(c_void_p), vv.ctypes.data_as(c_void_p), byref(h))
        return SparseX(self._lib, h, m, n, int(ci.size), torch.device("cuda", self.device))

    # ---- building blocks ----
    def convert(self, X32, dtype=torch.bfloat16):
        _dev(X32, "X32")
        if X32.dtype != torch.float32 or X32.dim() != 2 or X32.stride(1) != 1:
            raise ValueError("X32 must be a 2-D float32 tensor with unit column stride")
        m, n = X32.shape
        # each row starts on a 128-byte line, so the products' row runs fetch
        # no line they do not use
        ld = (n + 63) // 64 * 64
        buf = torch.empty((m, ld), dtype=dtype, device=X32.device)
        self._call(self._lib.enmf_convert, _ptr(X32), m, n, X32.stride(0), _DTYPES[dtype], _ptr(buf), ld)
        return buf[:, :n]

    def xv(self, X, B):
        M = matrix(X)
        k = B.shape[1]
        _factor(B, X.shape[1], k, "B")
        P = torch.empty((X.shape[0], k), dtype=torch.float32, device=X.device)
        self._call(self._lib.enmf_xv, byref(M), _ptr(B), k, _ptr(P))
        return P

    def xv_static(self, X, B, P=None):
        """P = X B through enmf_xv_static (no device allocation by the library).
        P may be passed in (float32, X.shape[0] x k) so that nothing at all is
        allocated by the call."""
        M = matrix(X)
        k = B.shape[1]
        _factor(B, X.shape[1], k, "B")
        if P is None:
            P = torch.empty((X.shape[0], k), dtype=torch.float32, device=X.device)
        else:
            _factor(P, X.shape[0], k, "P")
        self._call(self._lib.enmf_xv_static, byref(M), _ptr(B), k, _ptr(P))
        return P

    def xtu(self, X, A):
        M = matrix(X)
        k = A.shape[1]
        _factor(A, X.shape[0], k, "A")
        Q = torch.empty((X.shape[1], k), dtype=torch.float32, device=X.device)
        self._call(self._lib.enmf_xtu, byref(M), _ptr(A), k, _ptr(Q))
        return Q

    def gram(self, A):
        _factor(A, A.shape[0], A.shape[1], "A")
        k = A.shape[1]
        G = torch.empty((k, k), dtype=torch.float64, device=A.device)
        self._call(self._lib.enmf_gram, _ptr(A), A.shape[0], k, _ptr(G))
        return G

    # ---- the four blocks of the method ----
    def svd_init(self, X, r, omega, oversample=10, power_iters=2):
        M = matrix(X)
        m, n = X.shape
        _factor(omega, n, r + oversample, "omega")
        U = torch.empty((m, r), dtype=torch.float32, device=X.device)
        V = torch.empty((n, r), dtype=torch.float32, device=X.device)
        sig = (c_double * r)()
        rel = c_double()
        o = SvdOpts(omega.data_ptr(), oversample, power_iters)
        self._call(self._lib.enmf_svd_init, byref(M), r, byref(o), _ptr(U), _ptr(V), sig, byref(rel))
        return U, V, [sig[i] for i in range(r)], rel.value

    def enmc_init(self, X, mask_words, r, omega, oversample=10, power_iters=2, als_iters=50):
        """eNMC start: randomized SVD of the zero-filled X, then softImpute-ALS.
        mask_words: int32 device tensor (m x ceil(n/32)) from pack_mask."""
        M = matrix(X)
        m, n = X.shape
        mk = _mask(mask_words, m, n)
        _factor(omega, n, r + oversample, "omega")
        U = torch.empty((m, r), dtype=torch.float32, device=X.device)
        V = torch.empty((n, r), dtype=torch.float32, device=X.device)
        f = c_double()
        o = SvdOpts(omega.data_ptr(), oversample, power_iters)
        self._call(self._lib.enmf_enmc_init, byref(M), byref(mk), r, byref(o), als_iters, _ptr(U),
                   _ptr(V), byref(f))
        return U, V, f.value

    def enmc_grad(self, X, mask_words, U, V):
        """Masked gradients (gU, gV) and fhat at (U, V)."""
        M = matrix(X)
        m, n = X.shape
        mk = _mask(mask_words, m, n)
        r = U.shape[1]
        _factor(U, m, r, "U")
        _factor(V, n, r, "V")
        gU = torch.empty((m, r), dtype=torch.float32, device=X.device)
        gV = torch.empty((n, r), dtype=torch.float32, device=X.device)
        f = c_double()
        self._call(self._lib.enmf_enmc_grad, byref(M), byref(mk), r, _ptr(U), _ptr(V), _ptr(gU),
                   _ptr(gV), byref(f))
        return gU, gV, f.value

    def enmc_iterate(self, X, mask_words, U, V, max_iter, ext_iters=10, pbcd_max_iter=5,
                     kkt_tol=-1.0, step_u=0.0, step_v=0.0):
        """The eNMC loop (push, masked PBCD) in place on U and V."""
        M = matrix(X)
        m, n = X.shape
        mk = _mask(mask_words, m, n)
        r = U.shape[1]
        _factor(U, m, r, "U")
        _factor(V, n, r, "V")
        o = IterOpts(step_u, step_v, 0.0, -1.0, kkt_tol, 0.0, ext_iters, pbcd_max_iter, max_iter,
                     1, 0, 0)
        rep = IterReport()
        self._call(self._lib.enmf_enmc_iterate, byref(M), byref(mk), r, _ptr(U), _ptr(V), byref(o),
                   byref(rep))
        return {name: getattr(rep, name) for name, _ in IterReport._fields_}

    def rotate(self, U, V, rho0=1.0, max_iter=100, tol=1e-10, check_every=10):
        m, r = U.shape
        n = V.shape[0]
        _factor(U, m, r, "U")
        _factor(V, n, r, "V")
        o = RotateOpts(rho0, tol, max_iter, check_every)
        R = (c_double * (r * r))()
        steps = c_int32()
        g0, g1 = c_double(), c_double()
        self._call(self._lib.enmf_rotate, m, n, r, _ptr(U), _ptr(V), byref(o), R, byref(steps),
                   byref(g0), byref(g1))
        return dict(R=[R[i] for i in range(r * r)], steps=steps.value, neg_mass_before=g0.value,
                    neg_mass_after=g1.value)

    def rotate_general(self, U, V, rho0=1.0, max_iter=500, tol=1e-10):
        """Generalized rotation (R1, Lambda, R2) in place on U and V."""
        m, r = U.shape
        n = V.shape[0]
        _factor(U, m, r, "U")
        _factor(V, n, r, "V")
        o = GrotOpts(rho0, tol, max_iter, 0)
        R1 = (c_double * (r * r))()
        R2 = (c_double * (r * r))()
        lam = (c_double * r)()
        steps = c_int32()
        g0, g1 = c_double(), c_double()
        self._call(self._lib.enmf_rotate_general, m, n, r, _ptr(U), _ptr(V), byref(o), R1, lam, R2,
                   byref(steps), byref(g0), byref(g1))
        return dict(R1=np.array(R1[:]).reshape(r, r), lam=np.array(lam[:]),
                    R2=np.array(R2[:]).reshape(r, r), steps=steps.value, neg_mass_before=g0.value,
                    neg_mass_after=g1.value)

    def iterate(self, X, U, V, max_iter, ext_iters=10, pbcd_max_iter=5, pbcd_eps=0.0,
                step_u=0.0, step_v=0.0, check_every=1, kkt_tol=-1.0, relerr_tol=-1.0,
                relerr_svd=0.0, mode=0, trace_cap=0, graph_replay=0):
        M = matrix(X)
        m, n = X.shape
        r = U.shape[1]
        _factor(U, m, r, "U")
        _factor(V, n, r, "V")
        o = IterOpts(step_u, step_v, pbcd_eps, relerr_tol, kkt_tol, relerr_svd, ext_iters,
                     pbcd_max_iter, max_iter, check_every, mode, int(graph_replay))
        rep = IterReport()
        trace = None
        if trace_cap > 0:
            trace = torch.zeros((trace_cap, TRACE_FIELDS), dtype=torch.float64, device=X.device)
        self._call(self._lib.enmf_iterate, byref(M), r, _ptr(U), _ptr(V), byref(o), byref(rep),
                   _ptr(trace) if trace is not None else None, trace_cap)
        out = {name: getattr(rep, name) for name, _ in IterReport._fields_}
        if trace is not None:
            out["trace"] = trace
        return out

    def objective_kkt(self, X, U, V, relerr_svd=0.0):
        M = matrix(X)
        m, n = X.shape
        r = U.shape[1]
        _factor(U, m, r, "U")
        _factor(V, n, r, "V")
        k = Kkt()
        self._call(self._lib.enmf_objective_kkt, byref(M), r, _ptr(U), _ptr(V), relerr_svd, byref(k))
        return {name: getattr(k, name) for name, _ in Kkt._fields_}

    def time_products(self, X, k, reps=20):
        """Average device ms per launch of the X B and X^T A streaming kernels."""
        M = matrix(X)
        a, b = c_double(), c_double()
        self._call(self._lib.enmf_time_products, byref(M), k, reps, byref(a), byref(b))
        return a.value, b.value

    def kernel_timing(self, period):
        """Set the in-solve sampling period of the streaming kernels (0 = off) and
        return (xv_ms, xtu_ms, samples) accumulated since the previous call."""
        a, b, n = c_double(), c_double(), c_int32()
        self._call(self._lib.enmf_kernel_timing, period, byref(a), byref(b), byref(n))
        return a.value, b.value, n.value

    def solve(self, X, r, omega, oversample=10, power_iters=2, rho0=1.0, rot_max_iter=100,
              rot_tol=1e-10, **iter_opts):
        """Algorithm 3 end to end: SVD init, rotation, exterior phase and HALS."""
        U, V, sigma, rsvd = self.svd_init(X, r, omega, oversample, power_iters)
        rot = self.rotate(U, V, rho0, rot_max_iter, rot_tol)
        iter_opts.setdefault("relerr_svd", rsvd)
        rep = self.iterate(X, U, V, **iter_opts)
        rep.update(sigma=sigma, relerr_svd=rsvd, rotation=rot)
        return U, V, rep


EBUSY = 5


class Server:
    """A libenmf server: many solves of uneven shape in flight on one device.

    submit() queues a request and returns a ticket at once; poll() returns
    None while the request runs and its report once it has finished.  The
    tensors of a request (X, omega and the U/V outputs) are kept referenced
    here until the request has been polled, as the device reads and writes
    them until then.
    """

    def __init__(self, ctx, hbm_budget_bytes=0, max_slots=0, tick_time_us=0, ticks_per_launch=0,
                 direct_launch=0, wide_min_elems=0, wide_lanes=0):
        self._lib = ctx._lib
        self._ctx = ctx
        h = c_void_p()
        o = ServeOpts(hbm_budget_bytes, max_slots, tick_time_us, ticks_per_launch, direct_launch,
                      wide_min_elems, wide_lanes, 0)
        st = self._lib.enmf_serve_start(ctx._h, byref(o), byref(h))
        if st != 0:
            raise EnmfError(st, self._lib.enmf_last_error(ctx._h).decode())
        self._h = h
        self._live = {}

    def submit(self, X, r, omega, oversample=10, power_iters=2, rho0=1.0, rot_max_iter=100,
               rot_tol=1e-10, rot_check_every=10, max_iter=300, ext_iters=10, pbcd_max_iter=5,
               check_every=1, kkt_tol=-1.0, relerr_tol=-1.0, step_u=0.0, step_v=0.0, mode=0):
        """Queue one solve; returns (ticket, U, V) with U, V the output tensors."""
        M = matrix(X)
        m, n = X.shape
        _factor(omega, n, r + oversample, "omega")
        U = torch.empty((m, r), dtype=torch.float32, device=X.device)
        V = torch.empty((n, r), dtype=torch.float32, device=X.device)
        req = Request(M, r, 0, SvdOpts(omega.data_ptr(), oversample, power_iters),
                      RotateOpts(rho0, rot_tol, rot_max_iter, rot_check_every),
                      IterOpts(step_u, step_v, 0.0, relerr_tol, kkt_tol, 0.0, ext_iters,
                               pbcd_max_iter, max_iter, check_every, mode, 0),
                      U.data_ptr(), V.data_ptr())
        # inputs must be on the device before the server's own stream reads them
        torch.cuda.current_stream(X.device).synchronize()
        t = ctypes.c_uint64()
        st = self._lib.enmf_serve_submit(self._h, byref(req), byref(t))
        if st != 0:
            raise EnmfError(st, self._lib.enmf_serve_last_error(self._h).decode())
        self._live[t.value] = (X, omega, U, V)
        return t.value, U, V

    def poll(self, ticket):
        """None while running; else dict(report..., latency_s, status)."""
        rep = IterReport()
        lat = c_double()
        st = self._lib.enmf_serve_poll(self._h, ticket, byref(rep), byref(lat))
        if st == EBUSY:
            return None
        if st not in (0, 4):
            raise EnmfError(st, self._lib.enmf_serve_last_error(self._h).decode())
        self._live.pop(ticket, None)
        out = {name: getattr(rep, name) for name, _ in IterReport._fields_}
        out.update(latency_s=lat.value, status=st)
        return out

    def wait(self, ticket, timeout=120.0, interval=1e-3):
        import time
        t0 = time.perf_counter()
        while True:
            res = self.poll(ticket)
            if res is not None:
                return res
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"request {ticket} did not finish in {timeout} s")
            time.sleep(interval)

    def stop(self):
        if getattr(self, "_h", None):
            st = self._lib.enmf_serve_stop(self._h)
            self._h = None
            self._live.clear()
            if st != 0:
                raise EnmfError(st, "server stopped after a device failure")

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass

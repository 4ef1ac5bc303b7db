"""Thin ctypes binding of libhyeig (include/hyeig.h).

Argument marshalling only: every step of the computation runs inside the
library.  Torch tensors provide device memory (``data_ptr``) and the stream;
nothing here computes.  If the built library is missing this module raises
at import time: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyeig.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libhyeig.so is not built (run python -m paper_2305_15552_amd.build)")
_lib = ctypes.CDLL(LIB_PATH)

# ---- enums (mirror include/hyeig.h) ----
OK, EINVAL, ENOMEM, EDEVICE, ENOTSPD, ENOCONV, EUNSUPPORTED, ENUMERIC = range(8)
STATUS_NAMES = ["OK", "EINVAL", "ENOMEM", "EDEVICE", "ENOTSPD", "ENOCONV", "EUNSUPPORTED", "ENUMERIC"]
F64, F32, BF16 = 0, 1, 2
MMA_F64, MMA_F32, MMA_SPLIT_BF16 = 0, 1, 2
MAT_VALIDATE, MAT_BF16, MAT_ROWSTATS = 1, 2, 4
LOBPCG, BLANCZOS, LOBPCG_RMMDIIS, BLANCZOS_RMMDIIS, CHEBFSI, CHEBFSI_RMMDIIS = 0, 1, 2, 3, 4, 5
SWITCH_TAU, SWITCH_RESID, SWITCH_ITERS = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI, PRECOND_MLP = 0, 1, 2
PREC_PLAIN_F64, PREC_F32, PREC_BF16_SPMM = 0, 1, 2
NORM_HNORM, NORM_THETA = 0, 1
MLP_NPARAM = 64 * 4 + 2 * 64 + 1

_DT = {torch.float64: F64, torch.float32: F32}


class HyeigError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES[status] if 0 <= status < 8 else status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("nb", ctypes.c_int), ("method", ctypes.c_int), ("tol", ctypes.c_double),
                ("tol_norm", ctypes.c_int), ("hnorm", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("min_front", ctypes.c_int), ("switch_rule", ctypes.c_int), ("switch_thr", ctypes.c_double),
                ("s_max", ctypes.c_int), ("rmm_maxiter", ctypes.c_int), ("rmm_precond", ctypes.c_int),
                ("fallback", ctypes.c_int), ("precond", ctypes.c_int), ("mlp", ctypes.c_void_p),
                ("jacobi_floor", ctypes.c_double), ("precision", ctypes.c_int), ("refresh_every", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("lock", ctypes.c_int), ("basis", ctypes.c_int),
                ("maxiter_back", ctypes.c_int), ("nb_back", ctypes.c_int), ("rmm_decouple", ctypes.c_int),
                ("cheb_degree", ctypes.c_int), ("cheb_fixed_cutoff", ctypes.c_int), ("cheb_cutoff", ctypes.c_double),
                ("cheb_upper", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [("iters_front", ctypes.c_int), ("iters_rmm", ctypes.c_int), ("iters_back", ctypes.c_int),
                ("spmm_count", ctypes.c_int), ("spmv_count", ctypes.c_int64), ("switched", ctypes.c_int),
                ("converged", ctypes.c_int), ("fallback_used", ctypes.c_int), ("events_drop_p", ctypes.c_int),
                ("events_orth_w", ctypes.c_int), ("events_stagnation", ctypes.c_int),
                ("events_mlp_fallback", ctypes.c_int), ("refreshes", ctypes.c_int),
                ("events_deflation", ctypes.c_int), ("merged_back", ctypes.c_int),
                ("hnorm_used", ctypes.c_double),
                ("max_cond", ctypes.c_double), ("ms_total", ctypes.c_double), ("ms_spmm", ctypes.c_double),
                ("ms_dense", ctypes.c_double), ("ms_small", ctypes.c_double), ("ms_final", ctypes.c_double),
                ("resid_theta_max", ctypes.c_double), ("orth_err", ctypes.c_double),
                ("bytes_spmm", ctypes.c_double),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int), ("hist_len", ctypes.c_int),
                ("hist_t", ctypes.POINTER(ctypes.c_double)), ("iters_refine", ctypes.c_int),
                ("spmm_mc_count", ctypes.c_int), ("ms_spmm_mc", ctypes.c_double), ("bytes_spmm_mc", ctypes.c_double)]


class MatInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("ntiles", ctypes.c_int64),
                ("nblockrows", ctypes.c_int64), ("prepared_bytes", ctypes.c_int64), ("d_diag", ctypes.c_void_p),
                ("d_rowabs", ctypes.c_void_p), ("d_rownnz", ctypes.c_void_p)]


class TrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int64), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


_vp, _i64, _i32, _d, _u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint32
_pd = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "hyeig_ctx_create": [_i32, _vp, ctypes.POINTER(_vp)],
    "hyeig_ctx_destroy": [_vp],
    "hyeig_last_error": [_vp],
    "hyeig_last_spmm_ms": [_vp, _pd],
    "hyeig_mat_create": [_vp, _i64, _i64, _vp, _vp, _vp, _i32, _u32, ctypes.POINTER(_vp)],
    "hyeig_mat_destroy": [_vp],
    "hyeig_mat_get_info": [_vp, ctypes.POINTER(MatInfo)],
    "hyeig_spmm_sym": [_vp, _vp, _i32, _vp, _i64, _i32, _vp, _i64, _i32, _i32, _i32],
    "hyeig_gram": [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _i64, _i32, _i32, _vp],
    "hyeig_gram_noalloc": [_vp, _i64, _i32, _vp, _i64, _i32, _vp, _i64, _i32, _i32, _vp],
    "hyeig_block_update": [_vp, _i64, _i32, _i32, _vp, _i64, _vp, _d, _vp, _i64, _i32, _i32],
    "hyeig_cholqr": [_vp, _i64, _i32, _vp, _i64, _i32, _i32, _vp],
    "hyeig_rayleigh_ritz": [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _pd, _i32],
    "hyeig_rmm_state_create": [_vp, _vp, _i64, _i32, _i32, _vp, _i64, _vp, _i64, _d, _d, _i32, ctypes.POINTER(_vp)],
    "hyeig_rmm_diis_step": [_vp, _vp, _vp],
    "hyeig_rmm_state_get": [_vp, _vp, _vp, _i64, _vp, _vp, _vp],
    "hyeig_rmm_state_destroy": [_vp],
    "hyeig_params_default": [ctypes.POINTER(Params)],
    "hyeig_solve_lowest_k": [_vp, _vp, ctypes.POINTER(Params), _vp, _i64, _vp, _vp, ctypes.POINTER(Report)],
    "hyeig_mlp_create": [_vp, _vp, ctypes.POINTER(_vp)],
    "hyeig_mlp_get": [_vp, _vp, _vp],
    "hyeig_mlp_destroy": [_vp],
    "hyeig_mlp_forward": [_vp, _vp, _i64, _vp, _vp],
    "hyeig_mlp_precond": [_vp, _vp, _vp, ctypes.c_int, _vp, _i64, ctypes.c_int, _vp, ctypes.c_double],
    "hyeig_mlp_backward": [_vp, _vp, _i64, _vp, _vp, _vp, _pd],
    "hyeig_mlp_train": [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(TrainParams), _vp],
    "hyeig_mlp_labels": [_vp, _vp, ctypes.c_int, _vp, _i64, ctypes.c_int, ctypes.c_double, ctypes.c_int, _vp, _vp,
                         _pd],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.hyeig_ctx_destroy.restype = None
_lib.hyeig_mat_destroy.restype = None
_lib.hyeig_rmm_state_destroy.restype = None
_lib.hyeig_mlp_destroy.restype = None
_lib.hyeig_params_default.restype = None
_lib.hyeig_last_error.restype = ctypes.c_char_p


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    return t


def _ld(t):
    assert t.dim() == 2 and t.stride(1) == 1, "blocks must be row-major with unit column stride"
    return t.stride(0)


class Context:
    """A library context bound to a device and a HIP stream (torch's current
    stream of that device by default)."""

    def __init__(self, device: int = 0, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = ctypes.c_void_p()
        st = _lib.hyeig_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise HyeigError(st, "ctx_create failed")
        self.h = h

    def check(self, st):
        if st != OK:
            raise HyeigError(st, (_lib.hyeig_last_error(self.h) or b"").decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            _lib.hyeig_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_spmm_ms(self):
        v = ctypes.c_double()
        self.check(_lib.hyeig_last_spmm_ms(self.h, ctypes.byref(v)))
        return v.value


class Matrix:
    """Prepared half-stored symmetric matrix (hyeig_mat_create)."""

    def __init__(self, ctx: Context, n, rowptr, colidx, vals, flags=0, nnz=None):
        assert rowptr.dtype == torch.int64 and colidx.dtype == torch.int32 and vals.dtype == torch.float32
        nnz = colidx.numel() if nnz is None else int(nnz)
        assert nnz <= colidx.numel() and nnz <= vals.numel()
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx.check(_lib.hyeig_mat_create(ctx.h, n, nnz, _ptr(rowptr), _ptr(colidx), _ptr(vals), F32,
                                        flags, ctypes.byref(h)))
        self.h = h
        self.n = n
        info = MatInfo()
        ctx.check(_lib.hyeig_mat_get_info(h, ctypes.byref(info)))
        self.info = info

    def close(self):
        if getattr(self, "h", None):
            _lib.hyeig_mat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev_view(self, ptr, n):
        """Copy of a library-owned device vector (n floats) as a torch tensor."""
        if not ptr:
            return None

        class _Arr:
            __cuda_array_interface__ = {"shape": (n,), "typestr": "<f4", "data": (ptr, False), "version": 3}

        return torch.as_tensor(_Arr(), device="cuda:%d" % self.ctx.device).clone()

    def diag(self):
        return self._dev_view(self.info.d_diag, self.n)

    def rowabs(self):
        return self._dev_view(self.info.d_rowabs, self.n)

    def rownnz(self):
        return self._dev_view(self.info.d_rownnz, self.n)


def spmm_sym(ctx, H, X, Y, acc=None, vdt=F32, m=None):
    """Y = H X (hyeig_spmm_sym)."""
    m = X.shape[1] if m is None else m
    acc = _DT[Y.dtype] if acc is None else acc
    ctx.check(_lib.hyeig_spmm_sym(ctx.h, H.h, m, _ptr(X), _ld(X), _DT[X.dtype], _ptr(Y), _ld(Y), _DT[Y.dtype], acc,
                                  vdt))
    return Y


def gram(ctx, A, B, G, mode=None, ka=None, kb=None):
    """G (ka x kb, column-major FP64 device) = A^T B (hyeig_gram)."""
    ka = A.shape[1] if ka is None else ka
    kb = B.shape[1] if kb is None else kb
    if mode is None:
        mode = MMA_F64 if A.dtype == torch.float64 else MMA_F32
    ctx.check(_lib.hyeig_gram(ctx.h, A.shape[0], ka, _ptr(A), _ld(A), kb, _ptr(B), _ld(B), _DT[A.dtype], mode,
                              _ptr(G)))
    return G


def gram_noalloc(ctx, A, B, G, mode=None, ka=None, kb=None):
    """G = A^T B with the partial sums in the library's fixed device buffer
    (hyeig_gram_noalloc: allocates nothing)."""
    ka = A.shape[1] if ka is None else ka
    kb = B.shape[1] if kb is None else kb
    if mode is None:
        mode = MMA_F64 if A.dtype == torch.float64 else MMA_F32
    ctx.check(_lib.hyeig_gram_noalloc(ctx.h, A.shape[0], ka, _ptr(A), _ld(A), kb, _ptr(B), _ld(B), _DT[A.dtype],
                                      mode, _ptr(G)))
    return G


def block_update(ctx, S, C, Y, beta=0.0, mode=MMA_F32, k=None, m=None):
    """Y = S C + beta Y, C column-major FP64 on the device (hyeig_block_update)."""
    k = S.shape[1] if k is None else k
    m = Y.shape[1] if m is None else m
    ctx.check(_lib.hyeig_block_update(ctx.h, S.shape[0], k, m, _ptr(S), _ld(S), _ptr(C), beta, _ptr(Y), _ld(Y),
                                      _DT[S.dtype], mode))
    return Y


def cholqr(ctx, X, passes=1, R=None):
    """X <- X R^{-1} with R^T R = X^T X (hyeig_cholqr)."""
    ctx.check(_lib.hyeig_cholqr(ctx.h, X.shape[0], X.shape[1], _ptr(X), _ld(X), _DT[X.dtype], passes, _ptr(R)))
    return X


def rayleigh_ritz(ctx, A, B, nwant, on_device=False):
    """(theta, C, condB) of the pencil (A, B); A, B column-major FP64 (numpy
    arrays on the host, or torch tensors on the device with on_device=True)."""
    import numpy as np
    k = A.shape[0]
    cond = ctypes.c_double(0.0)
    if on_device:
        theta = torch.empty(nwant, dtype=torch.float64, device=A.device)
        C = torch.empty(k * nwant, dtype=torch.float64, device=A.device)
        ctx.check(_lib.hyeig_rayleigh_ritz(ctx.h, k, _ptr(A), _ptr(B), nwant, _ptr(theta), _ptr(C),
                                           ctypes.byref(cond), 1))
        return theta, C.reshape(nwant, k).T, cond.value
    Af = np.asfortranarray(A, dtype=np.float64)
    Bf = None if B is None else np.asfortranarray(B, dtype=np.float64)
    theta = np.zeros(nwant)
    C = np.zeros((k, nwant), order="F")
    ctx.check(_lib.hyeig_rayleigh_ritz(ctx.h, k, Af.ctypes.data_as(_vp), None if Bf is None else Bf.ctypes.data_as(_vp),
                                       nwant, theta.ctypes.data_as(_vp), C.ctypes.data_as(_vp), ctypes.byref(cond), 0))
    return theta, C, cond.value


def params_default(**kw):
    p = Params()
    _lib.hyeig_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k == "mlp" and isinstance(v, Mlp):
            v = v.h.value  # the caller keeps the Mlp object alive for the solve
        setattr(p, k, v)
    return p


def solve_lowest_k(ctx, H, params, X, hist_cap=0):
    """Runs hyeig_solve_lowest_k; X (n x nb FP32 device) holds X0 on entry and
    the eigenvectors on exit.  Returns (evals, resid, report, status, history);
    with a history, ``report.hist_times`` holds for each row the milliseconds
    since the solve started, the product-kernel and host small-problem
    milliseconds so far, and cond(S^T S) of the last LOBPCG Rayleigh-Ritz step."""
    import numpy as np
    k = params.k
    ev = np.zeros(k)
    rs = np.zeros(k)
    rep = Report()
    hist = None
    if hist_cap:
        hist = np.zeros(hist_cap * k)
        hist_t = np.zeros(4 * hist_cap)
        rep.hist = hist.ctypes.data_as(_pd)
        rep.hist_t = hist_t.ctypes.data_as(_pd)
        rep.hist_cap = hist_cap
    st = _lib.hyeig_solve_lowest_k(ctx.h, H.h, ctypes.byref(params), _ptr(X), _ld(X), ev.ctypes.data_as(_vp),
                                   rs.ctypes.data_as(_vp), ctypes.byref(rep))
    if st not in (OK, ENOCONV):
        ctx.check(st)
    h = None
    if hist is not None:
        h = hist[:rep.hist_len * k].reshape(rep.hist_len, k)
        rep.hist_times = hist_t[:4 * rep.hist_len].reshape(rep.hist_len, 4)
    return ev, rs, rep, st, h


class RmmState:
    """Batched RMM-DIIS state (hyeig_rmm_state_*)."""

    def __init__(self, ctx, H, X, HX=None, s_max=10, tol=1e-6, hnorm=1.0, precond=0):
        self.ctx = ctx
        self.k = X.shape[1]
        h = ctypes.c_void_p()
        ctx.check(_lib.hyeig_rmm_state_create(ctx.h, H.h, X.shape[0], X.shape[1], s_max, _ptr(X), _ld(X), _ptr(HX),
                                              _ld(HX) if HX is not None else 0, tol, hnorm, precond,
                                              ctypes.byref(h)))
        self.h = h
        self.H = H

    def step(self):
        self.ctx.check(_lib.hyeig_rmm_diis_step(self.ctx.h, self.H.h, self.h))

    def get(self, X=None):
        import numpy as np
        th = np.zeros(self.k)
        rs = np.zeros(self.k)
        cv = np.zeros(self.k, dtype=np.int32)
        self.ctx.check(_lib.hyeig_rmm_state_get(self.ctx.h, self.h, _ptr(X), _ld(X) if X is not None else 0,
                                                th.ctypes.data_as(_vp), rs.ctypes.data_as(_vp),
                                                cv.ctypes.data_as(_vp)))
        return th, rs, cv.astype(bool)

    def close(self):
        if getattr(self, "h", None):
            _lib.hyeig_rmm_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_labels(ctx, M, X, hnorm, steps=20):
    """(features [n k x 4], targets [n k], theta [k]) of the correction equation
    for the block X (n x k torch tensor on the device) (hyeig_mlp_labels)."""
    import numpy as np
    import torch
    n, k = X.shape
    F = torch.empty((n * k, 4), dtype=torch.float32, device=X.device)
    T = torch.empty(n * k, dtype=torch.float32, device=X.device)
    th = np.zeros(k)
    ctx.check(_lib.hyeig_mlp_labels(ctx.h, M.h, k, _ptr(X), _ld(X), _DT[X.dtype], hnorm, steps, _ptr(F), _ptr(T),
                                    th.ctypes.data_as(_pd)))
    return F, T, th


class Mlp:
    """Per-row MLP preconditioner weights (hyeig_mlp_*)."""

    def __init__(self, ctx, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_NPARAM
        h = ctypes.c_void_p()
        ctx.check(_lib.hyeig_mlp_create(ctx.h, p.ctypes.data_as(_vp), ctypes.byref(h)))
        self.h = h
        self.ctx = ctx

    def params(self):
        import numpy as np
        p = np.zeros(MLP_NPARAM, dtype=np.float32)
        self.ctx.check(_lib.hyeig_mlp_get(self.ctx.h, self.h, p.ctypes.data_as(_vp)))
        return p

    def forward(self, feat, out):
        self.ctx.check(_lib.hyeig_mlp_forward(self.ctx.h, self.h, feat.shape[0], _ptr(feat), _ptr(out)))
        return out

    def precond(self, M, W, theta, hnorm):
        """W (n x k device block, holding R) <- K^{-1} R with this network as the
        learned preconditioner (hyeig_mlp_precond); theta: k Ritz values."""
        import numpy as np
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self.ctx.check(_lib.hyeig_mlp_precond(self.ctx.h, self.h, M.h, W.shape[1], _ptr(W), _ld(W), _DT[W.dtype],
                                              th.ctypes.data_as(_vp), float(hnorm)))
        return W

    def backward(self, feat, target, grad):
        loss = ctypes.c_double()
        self.ctx.check(_lib.hyeig_mlp_backward(self.ctx.h, self.h, feat.shape[0], _ptr(feat), _ptr(target),
                                               _ptr(grad), ctypes.byref(loss)))
        return loss.value

    def train(self, feat, target, epochs=20, batch=65536, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        import numpy as np
        tp = TrainParams(epochs, batch, lr, beta1, beta2, eps, seed)
        losses = np.zeros(epochs)
        self.ctx.check(_lib.hyeig_mlp_train(self.ctx.h, self.h, feat.shape[0], _ptr(feat), _ptr(target),
                                            ctypes.byref(tp), losses.ctypes.data_as(_vp)))
        return losses

    def close(self):
        if getattr(self, "h", None):
            _lib.hyeig_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def matrix_from_csr(ctx, n, rowptr, colidx, vals, flags=0, device=0):
    """Uploads host CSR arrays (numpy) and builds the prepared matrix."""
    dev = "cuda:%d" % device
    rp = torch.from_numpy(rowptr).to(dev)
    ci = torch.from_numpy(colidx).to(dev)
    vv = torch.from_numpy(vals).to(dev)
    M = Matrix(ctx, n, rp, ci, vv, flags)
    torch.cuda.synchronize(device)
    del rp, ci, vv
    return M

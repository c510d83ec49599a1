"""Python binding of libfkf.so, the MI355X fast random-walk Kalman filter.

Argument marshalling only: every numeric step runs in the library's HIP
kernels.  Device arrays are torch CUDA (ROCm) float64 tensors; the library is
driven on torch's current stream.  Importing this package fails loudly when
the library has not been built (``python paper_1405_2276_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfkf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1405_2276_amd/build.py`")
try:
    _lib = ctypes.CDLL(LIB_PATH)
except OSError as e:  # pragma: no cover
    raise ImportError(f"cannot load {LIB_PATH}: {e}") from e

_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p

MATERN = {0.5: 0, 1.5: 1, 2.5: 2}

STATUS = {0: "FKF_OK", -1: "FKF_E_ARG", -2: "FKF_E_NOMEM", -3: "FKF_E_HIP",
          -4: "FKF_E_NOT_SPD", -5: "FKF_E_RANK", -6: "FKF_E_NONFINITE",
          -7: "FKF_E_ORDER", -8: "FKF_E_UNSUPPORTED"}


class FkfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class KernelParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("kind", ctypes.c_int32),
                ("variance", ctypes.c_double), ("length", ctypes.c_double)]


class HmatParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("leaf_size", ctypes.c_int32),
                ("cheb_order", ctypes.c_int32), ("cheb_order_max", ctypes.c_int32),
                ("eta", ctypes.c_double), ("block_tol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("far_eval", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64)]


class FilterParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_rank", ctypes.c_int32),
                ("rank_rtol", ctypes.c_double), ("gep_mode", ctypes.c_int32),
                ("gep_rank", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


GEP_MODE = {"exact": 0, "randomized": 1}


class CovInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("n_near_blocks", ctypes.c_int64),
                ("n_near_pairs", ctypes.c_int64), ("n_far_pairs", ctypes.c_int64),
                ("near_bytes", ctypes.c_int64), ("far_coef_per_rhs", ctypes.c_int64),
                ("cheb_p", ctypes.c_int32 * 32), ("covered_entries", ctypes.c_int64),
                ("far_interp_entries", ctypes.c_int64), ("far_bytes", ctypes.c_int64),
                ("far_pair_entries", ctypes.c_int64), ("coupling_groups", ctypes.c_int64),
                ("coupling_items", ctypes.c_int64)]


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_i = ctypes.c_int
_lib.fkf_last_error.restype = ctypes.c_char_p
_lib.fkf_version.restype = ctypes.c_char_p
_sig("fkf_cov_build", _i, [_c_dbl_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(KernelParams),
                           ctypes.POINTER(HmatParams), _vp, ctypes.POINTER(_vp)])
_sig("fkf_cov_apply", _i, [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int64, _vp])
_sig("fkf_cov_apply_noalloc", _i, [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, ctypes.c_int64,
                                   _vp])
_sig("fkf_cov_info", _i, [_vp, ctypes.POINTER(CovInfo)])
_sig("fkf_cov_perm", _i, [_vp, _c_i64_p])
_sig("fkf_cov_plan", _i, [_c_dbl_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(KernelParams),
                          ctypes.POINTER(HmatParams), ctypes.POINTER(CovInfo)])
_sig("fkf_rays_host", _i, [ctypes.c_int32, _c_i32_p, ctypes.c_int32, _c_dbl_p, _c_dbl_p, _c_i64_p,
                           _c_i64_p, _c_i32_p, _c_dbl_p, ctypes.c_int64])
_sig("fkf_cov_destroy", None, [_vp])
_sig("fkf_obs_create_csr", _i, [ctypes.c_int32, ctypes.c_int64, _c_i64_p, _c_i32_p, _c_dbl_p,
                                _c_dbl_p, _vp, ctypes.POINTER(_vp)])
_sig("fkf_obs_create_rays", _i, [ctypes.c_int32, _c_i32_p, ctypes.c_int32, _c_dbl_p, _c_dbl_p,
                                 _c_dbl_p, _vp, ctypes.POINTER(_vp)])
_sig("fkf_obs_shape", _i, [_vp, _c_i32_p, _c_i64_p, _c_i64_p])
_sig("fkf_obs_get_csr", _i, [_vp, _c_i64_p, _c_i32_p, _c_dbl_p])
_sig("fkf_obs_apply", _i, [_vp, _vp, _vp, _vp])
_sig("fkf_obs_cross_cov", _i, [_vp, _vp, _vp, ctypes.c_int64, _vp])
_sig("fkf_obs_destroy", None, [_vp])
_sig("fkf_filter_create", _i, [_vp, _vp, ctypes.c_double, ctypes.POINTER(FilterParams), _vp,
                               ctypes.POINTER(_vp)])
_sig("fkf_filter_reset", _i, [_vp, _vp, ctypes.c_double, _vp])
_sig("fkf_filter_step", _i, [_vp, _vp, _vp, _vp])
_sig("fkf_filter_step_boxcox", _i, [_vp, _vp, ctypes.c_double, _vp, _vp])
_sig("fkf_filter_loglik", _i, [_vp, _c_dbl_p, _c_dbl_p, _c_dbl_p, _c_dbl_p, _vp])
_sig("fkf_filter_track_length", _i, [_vp, _vp, _vp])
_sig("fkf_filter_step_many", _i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                  ctypes.c_int32, _vp])
_sig("fkf_filter_status", _i, [_vp, _vp])
_sig("fkf_filter_mean", _i, [_vp, _vp, _vp])
_sig("fkf_filter_variance", _i, [_vp, _vp, _vp])
_sig("fkf_filter_realize", _i, [_vp, _vp, ctypes.c_int32, ctypes.c_int64, _vp, ctypes.c_int64, _vp])
_sig("fkf_filter_info", _i, [_vp, _c_i64_p, _c_dbl_p, _c_i32_p])
_sig("fkf_gaussian_sketch", _i, [ctypes.c_uint64, ctypes.c_int64, _vp, _vp])
_sig("fkf_filter_modes", _i, [_vp, _c_dbl_p, _c_dbl_p])
_sig("fkf_filter_lowrank", _i, [_vp, _vp, ctypes.c_int64, _vp, ctypes.c_int64, _vp,
                                ctypes.c_int32, _c_i32_p, _vp])
_sig("fkf_filter_destroy", None, [_vp])
_sig("fkf_sym_eig", _i, [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, ctypes.c_int64, _vp])
_sig("fkf_trace_enable", _i, [ctypes.c_int32])
_sig("fkf_trace_query", _i, [ctypes.c_char_p, _c_i64_p, _c_dbl_p])
_sig("fkf_trace_names", _i, [ctypes.c_char_p, ctypes.c_int64])



def _check(code: int):
    if code != 0:
        raise FkfError(code, _lib.fkf_last_error().decode(errors="replace"))


def trace_enable(on: bool = True):
    """Enable/disable per-launch event timing in the library (clears records)."""
    _check(_lib.fkf_trace_enable(1 if on else 0))


def trace_report() -> dict:
    """{site: (launches, total_ms)} for every recorded launch site."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.fkf_trace_names(buf, len(buf)))
    out = {}
    for name in filter(None, buf.value.decode().split(",")):
        c, ms = ctypes.c_int64(), ctypes.c_double()
        _check(_lib.fkf_trace_query(name.encode(), ctypes.byref(c), ctypes.byref(ms)))
        out[name] = (c.value, ms.value)
    return out


def step_many(filters, obs, ys, stream=None):
    """One step of several independent filters (fkf_filter_step_many): the
    projected eigenproblems of filters that build their basis now are solved
    as one batch."""
    n = len(filters)
    if len(obs) != n or len(ys) != n:
        raise ValueError("filters, obs and ys must have the same length")
    yd = [to_device(y) for y in ys]
    fa = (_vp * n)(*[f._h.value for f in filters])
    oa = (_vp * n)(*[o.handle.value for o in obs])
    ya = (_vp * n)(*[y.data_ptr() for y in yd])
    for f, y in zip(filters, yd):
        f._y = y     # keep alive until the stream consumes it
    _check(_lib.fkf_filter_step_many(fa, oa, ya, n, _stream(stream)))


_LL_FUNCTION = None


def _loglik_function():
    """The torch.autograd.Function behind ``innovation_loglik`` (built on
    first use, so that importing the package does not import torch)."""
    global _LL_FUNCTION
    if _LL_FUNCTION is None:
        torch = _torch()

        class InnovationLogLik(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta, length, noise_var, points, make_obs, ys, cov_kw, alpha0):
                th, ln, nv = float(theta), float(length), float(noise_var)
                cov = Cov(points, variance=th, length=ln, **cov_kw)
                dcov = Cov(points, variance=th, length=ln, dlength=True, **cov_kw)
                obs = make_obs(nv)
                f = Filter(cov, alpha0=alpha0)
                try:
                    f.track_length(dcov)
                    for y in ys:
                        f.step(obs, y)
                    ll, d_th, d_nv, d_ln = f.loglik()
                finally:
                    f.close()
                    obs.close()
                    dcov.close()
                    cov.close()
                # d/d theta = (d/d log theta) / theta, likewise for the others
                ctx.grads = (d_th / th, d_ln / ln, d_nv / nv)
                return torch.tensor(ll, dtype=torch.float64, device=theta.device)

            @staticmethod
            def backward(ctx, g):
                gt, gl, gn = ctx.grads
                return g * gt, g * gl, g * gn, None, None, None, None, None

        _LL_FUNCTION = InnovationLogLik
    return _LL_FUNCTION


def innovation_loglik(theta, length, noise_var, points, make_obs, ys, alpha0: float = 0.0,
                      **cov_kw):
    """Innovation log-likelihood of observations ys (steps x n_m) under the
    random-walk model with a Matern Gamma of variance ``theta`` and length
    ``length`` and measurement noise ``noise_var`` (0-d float64 tensors;
    make_obs(noise_var) builds the observation operator with that noise
    variance), as a differentiable torch function of the three.  The forward
    pass runs the constant-H filter on the GPU with the length derivative
    tracked; the backward pass uses the exact derivatives the filter carries
    (fkf_filter_loglik).  cov_kw go to Cov (nu, leaf_size, precision, ...)."""
    return _loglik_function().apply(theta, length, noise_var, points, make_obs, ys, cov_kw,
                                    alpha0)


def gaussian_sketch(seed: int, count: int, stream=None):
    """The first `count` numbers of the randomized eigensolver's sketch stream
    (fkf_gaussian_sketch) as a CUDA float64 tensor."""
    torch = _torch()
    out = torch.empty(max(int(count), 1), dtype=torch.float64, device="cuda")
    _check(_lib.fkf_gaussian_sketch(int(seed), int(count), out.data_ptr(), _stream(stream)))
    return out[:count]


def sym_eig(A, stream=None):
    """Eigen-decomposition of a symmetric CUDA float64 matrix (n, n)
    (fkf_sym_eig): (w, W), eigenvalues descending and the unit eigenvectors
    as the columns of a column-major (n, n) tensor."""
    torch = _torch()
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    a, lda, _ = _colmajor(A)
    n = A.shape[0]
    w = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    W = fortran_empty(max(n, 1), max(n, 1))
    _check(_lib.fkf_sym_eig(a, lda, n, w.data_ptr(), W.data_ptr(), max(n, 1), _stream(stream)))
    return w[:n], W[:n, :n]


def version() -> str:
    return _lib.fkf_version().decode()


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _colmajor(t):
    """View a CUDA float64 tensor (n,) or (n, k) as column-major (ptr, ld, k)."""
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float64):
        raise TypeError("expected a CUDA float64 tensor")
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError("vector must be contiguous")
        return t.data_ptr(), t.shape[0], 1
    if t.dim() != 2:
        raise ValueError("expected a 1-D or 2-D tensor")
    if t.stride(0) != 1 and t.shape[1] > 1:
        raise ValueError("matrix must be column-major: use x.t().contiguous().t()")
    ld = t.stride(1) if t.shape[1] > 1 else t.shape[0]
    return t.data_ptr(), max(ld, t.shape[0]), t.shape[1]


def fortran_empty(n: int, k: int, device="cuda"):
    """Uninitialised column-major (n, k) float64 CUDA tensor."""
    torch = _torch()
    return torch.empty((k, n), dtype=torch.float64, device=device).t()


PRECISION = {"fp64": 0, "mixed": 1}


def _params(nu, length, variance, leaf_size, cheb_order, cheb_order_max, eta, block_tol,
            precision="fp64", far_eval=False, workspace_bytes=0):
    if nu not in MATERN:
        raise ValueError("nu must be 0.5, 1.5 or 2.5")
    if precision not in PRECISION:
        raise ValueError("precision must be 'fp64' or 'mixed'")
    kp = KernelParams(ctypes.sizeof(KernelParams), MATERN[nu], variance, length)
    hp = HmatParams(ctypes.sizeof(HmatParams), leaf_size, cheb_order, cheb_order_max,
                    eta, block_tol, PRECISION[precision], int(bool(far_eval)),
                    int(workspace_bytes))
    return kp, hp


def _info_dict(inf: CovInfo) -> dict:
    d = {f: getattr(inf, f) for f, _ in CovInfo._fields_ if f != "cheb_p"}
    d["cheb_p"] = list(inf.cheb_p)[: inf.n_levels]
    return d


def plan(points, nu=1.5, length=0.1, variance=1.0, leaf_size=64, cheb_order=6,
         cheb_order_max=16, eta=1.5, block_tol=1e-7, precision="fp64", far_eval=False) -> dict:
    """Host-only H-matrix plan (tree, partition, Chebyshev orders); no GPU."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    kp, hp = _params(nu, length, variance, leaf_size, cheb_order, cheb_order_max, eta, block_tol,
                     precision, far_eval)
    inf = CovInfo()
    _check(_lib.fkf_cov_plan(pts.ctypes.data_as(_c_dbl_p), pts.shape[0], pts.shape[1],
                             ctypes.byref(kp), ctypes.byref(hp), ctypes.byref(inf)))
    return _info_dict(inf)


def rays_host(shape, src, rcv):
    """Host-only straight-ray operator as (rowptr, col, val) CSR arrays; no GPU."""
    src = np.ascontiguousarray(src, dtype=np.float64)
    rcv = np.ascontiguousarray(rcv, dtype=np.float64)
    grid = np.ascontiguousarray(shape, dtype=np.int32)
    n_m, d = src.shape
    rowptr = np.empty(n_m + 1, dtype=np.int64)
    nnz = ctypes.c_int64()
    args = (d, grid.ctypes.data_as(_c_i32_p), n_m, src.ctypes.data_as(_c_dbl_p),
            rcv.ctypes.data_as(_c_dbl_p), rowptr.ctypes.data_as(_c_i64_p), ctypes.byref(nnz))
    _check(_lib.fkf_rays_host(*args, None, None, 0))
    col = np.empty(nnz.value, dtype=np.int32)
    val = np.empty(nnz.value, dtype=np.float64)
    _check(_lib.fkf_rays_host(*args, col.ctypes.data_as(_c_i32_p), val.ctypes.data_as(_c_dbl_p),
                              nnz.value))
    return rowptr, col, val


class Cov:
    """Gamma_sys (Matern) as an H-matrix on the GPU (fkf_cov_*).

    precision: "fp64", or "mixed" (FP32 near-field storage and far-field kernel
    evaluation, FP64 accumulation; filters built on it stream their basis in
    FP32).  far_eval: evaluate the far-field coupling matrices in every product
    instead of storing them at build.  dlength: the operator dGamma/d length
    instead of Gamma (for likelihood gradients, Filter.track_length).
    workspace_bytes: bound on the several-column workspaces (0: 16 GiB);
    wider products run in column blocks."""

    def __init__(self, points, nu: float = 1.5, length: float = 0.1, variance: float = 1.0,
                 leaf_size: int = 64, cheb_order: int = 6, cheb_order_max: int = 16,
                 eta: float = 1.5, block_tol: float = 1e-7, precision: str = "fp64",
                 far_eval: bool = False, dlength: bool = False, workspace_bytes: int = 0,
                 stream=None):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2:
            raise ValueError("points must be (N, d)")
        self.n, self.d = pts.shape
        self.nu, self.length, self.variance = nu, length, variance
        kp, hp = _params(nu, length, variance, leaf_size, cheb_order, cheb_order_max, eta,
                         block_tol, precision, far_eval, workspace_bytes)
        if dlength:
            kp.kind += 3      # FKF_MATERN_*_DLENGTH
        self.precision = precision
        h = ctypes.c_void_p()
        _check(_lib.fkf_cov_build(pts.ctypes.data_as(_c_dbl_p), self.n, self.d,
                                  ctypes.byref(kp), ctypes.byref(hp), _stream(stream),
                                  ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def apply(self, X, out=None, stream=None):
        """Y = Gamma X for a CUDA float64 (N,) or column-major (N, k) tensor."""
        ptr, ldx, k = _colmajor(X)
        if X.shape[0] != self.n:
            raise ValueError("X has the wrong number of rows")
        if out is None:
            out = (_torch().empty(self.n, dtype=X.dtype, device=X.device) if X.dim() == 1
                   else fortran_empty(self.n, k, X.device))
        optr, ldy, _ = _colmajor(out)
        _check(_lib.fkf_cov_apply(self._h, ptr, ldx, k, optr, ldy, _stream(stream)))
        return out

    def apply_noalloc(self, X, out, stream=None):
        """Y = Gamma X into the caller's ``out`` through fkf_cov_apply_noalloc
        (no device allocation in the library: its workspace is a fixed
        per-device array)."""
        ptr, ldx, k = _colmajor(X)
        if X.shape[0] != self.n or out.shape[0] != self.n:
            raise ValueError("X and out must have N rows")
        optr, ldy, ko = _colmajor(out)
        if ko != k:
            raise ValueError("out must have as many columns as X")
        _check(_lib.fkf_cov_apply_noalloc(self._h, ptr, ldx, k, optr, ldy, _stream(stream)))
        return out

    def info(self) -> dict:
        inf = CovInfo()
        _check(_lib.fkf_cov_info(self._h, ctypes.byref(inf)))
        return _info_dict(inf)

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _check(_lib.fkf_cov_perm(self._h, out.ctypes.data_as(_c_i64_p)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.fkf_cov_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(a):
    """float64 numpy array -> CUDA tensor (column-major for 2-D)."""
    torch = _torch()
    if hasattr(a, "is_cuda"):
        return a
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


class Obs:
    """Measurement operator H with diagonal noise covariance R (fkf_obs_*)."""

    def __init__(self, handle, n_m, n):
        self._h, self.n_m, self.n = handle, n_m, n

    @classmethod
    def from_rays(cls, shape, src, rcv, noise_var, stream=None):
        src = np.ascontiguousarray(src, dtype=np.float64)
        rcv = np.ascontiguousarray(rcv, dtype=np.float64)
        grid = np.ascontiguousarray(shape, dtype=np.int32)
        n_m, d = src.shape
        nv = np.ascontiguousarray(np.broadcast_to(np.asarray(noise_var, dtype=np.float64), (n_m,)))
        h = ctypes.c_void_p()
        _check(_lib.fkf_obs_create_rays(d, grid.ctypes.data_as(_c_i32_p), n_m,
                                        src.ctypes.data_as(_c_dbl_p), rcv.ctypes.data_as(_c_dbl_p),
                                        nv.ctypes.data_as(_c_dbl_p), _stream(stream), ctypes.byref(h)))
        return cls(h, n_m, int(np.prod(shape)))

    @classmethod
    def from_csr(cls, H, noise_var, stream=None):
        import scipy.sparse as sp
        H = sp.csr_matrix(H)
        H.sort_indices()
        n_m, n = H.shape
        rp = np.ascontiguousarray(H.indptr, dtype=np.int64)
        col = np.ascontiguousarray(H.indices, dtype=np.int32)
        val = np.ascontiguousarray(H.data, dtype=np.float64)
        nv = np.ascontiguousarray(np.broadcast_to(np.asarray(noise_var, dtype=np.float64), (n_m,)))
        h = ctypes.c_void_p()
        _check(_lib.fkf_obs_create_csr(n_m, n, rp.ctypes.data_as(_c_i64_p),
                                       col.ctypes.data_as(_c_i32_p), val.ctypes.data_as(_c_dbl_p),
                                       nv.ctypes.data_as(_c_dbl_p), _stream(stream), ctypes.byref(h)))
        return cls(h, n_m, n)

    @property
    def handle(self):
        return self._h

    def csr(self):
        import scipy.sparse as sp
        nm, n, nnz = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.fkf_obs_shape(self._h, ctypes.byref(nm), ctypes.byref(n), ctypes.byref(nnz)))
        rp = np.empty(nm.value + 1, dtype=np.int64)
        col = np.empty(nnz.value, dtype=np.int32)
        val = np.empty(nnz.value, dtype=np.float64)
        _check(_lib.fkf_obs_get_csr(self._h, rp.ctypes.data_as(_c_i64_p),
                                    col.ctypes.data_as(_c_i32_p), val.ctypes.data_as(_c_dbl_p)))
        return sp.csr_matrix((val, col, rp), shape=(nm.value, n.value))

    def apply(self, x, out=None, stream=None):
        torch = _torch()
        x = to_device(x)
        if out is None:
            out = torch.empty(self.n_m, dtype=torch.float64, device=x.device)
        _check(_lib.fkf_obs_apply(self._h, x.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def cross_cov(self, cov, out=None, stream=None):
        """P = Gamma H^T as a column-major (N, n_m) CUDA float64 tensor
        (fkf_obs_cross_cov: far-cluster moments summed over the nonzeros of H)."""
        if out is None:
            out = fortran_empty(self.n, self.n_m)
        optr, ldp, k = _colmajor(out)
        if out.shape[0] != self.n or k != self.n_m:
            raise ValueError("out must be (N, n_m)")
        _check(_lib.fkf_obs_cross_cov(cov._h, self._h, optr, ldp, _stream(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.fkf_obs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Filter:
    """The fast random-walk Kalman filter (fkf_filter_*)."""

    def __init__(self, cov: Cov, s0=None, alpha0: float = 0.0, max_rank: int = 4096,
                 rank_rtol: float = 0.0, gep: str = "exact", gep_rank: int = 0,
                 oversample: int = 20, seed: int = 0, stream=None):
        """gep: "exact" (Rayleigh-Ritz on range(Gamma H^T)) or "randomized"
        (Appendix B with gep_rank modes, oversample extra sketch columns and
        the sketch stream seed)."""
        self.cov = cov
        self.n = cov.n
        if gep not in GEP_MODE:
            raise ValueError("gep must be 'exact' or 'randomized'")
        fp = FilterParams(ctypes.sizeof(FilterParams), max_rank, rank_rtol, GEP_MODE[gep],
                          int(gep_rank), int(oversample), 0, int(seed))
        s0p = None
        if s0 is not None:
            self._s0 = to_device(s0)
            s0p = self._s0.data_ptr()
        h = ctypes.c_void_p()
        _check(_lib.fkf_filter_create(cov.handle, s0p, float(alpha0), ctypes.byref(fp),
                                      _stream(stream), ctypes.byref(h)))
        self._h = h

    def reset(self, s0=None, alpha0: float = 0.0, stream=None):
        """Back to the initial state (fkf_filter_reset), keeping the filter's
        device buffers."""
        s0p = None
        if s0 is not None:
            self._s0 = to_device(s0)
            s0p = self._s0.data_ptr()
        _check(_lib.fkf_filter_reset(self._h, s0p, float(alpha0), _stream(stream)))

    def step(self, obs: Obs, y, stream=None):
        y = to_device(y)
        self._y = y     # keep alive until the stream consumes it
        _check(_lib.fkf_filter_step(self._h, obs.handle, y.data_ptr(), _stream(stream)))

    def step_boxcox(self, obs: Obs, y, bc_alpha: float, stream=None):
        """One extended-filter step for measurements y = H g(x) + v, with
        g(x) = ((x + a)/a)^a, a = bc_alpha (fkf_filter_step_boxcox)."""
        y = to_device(y)
        self._y = y     # keep alive until the stream consumes it
        _check(_lib.fkf_filter_step_boxcox(self._h, obs.handle, float(bc_alpha), y.data_ptr(),
                                           _stream(stream)))

    def track_length(self, dcov: "Cov", stream=None):
        """Carry d ll / d log length (fkf_filter_track_length); dcov is the
        length derivative of this filter's covariance (Cov(..., dlength=True))."""
        self._dcov = dcov     # borrowed by the library
        _check(_lib.fkf_filter_track_length(self._h, dcov.handle, _stream(stream)))

    def loglik(self, grad: bool = True, stream=None):
        """Innovation log-likelihood of the steps so far (fkf_filter_loglik);
        with grad, (ll, d ll / d log theta, d ll / d log sigma^2), plus
        d ll / d log length after track_length."""
        ll, a, g, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        want_len = grad and getattr(self, "_dcov", None) is not None
        _check(_lib.fkf_filter_loglik(self._h, ctypes.byref(ll),
                                      ctypes.byref(a) if grad else None,
                                      ctypes.byref(g) if want_len else None,
                                      ctypes.byref(s) if grad else None, _stream(stream)))
        if not grad:
            return ll.value
        if want_len:
            return ll.value, a.value, s.value, g.value
        return ll.value, a.value, s.value

    def status(self, stream=None):
        _check(_lib.fkf_filter_status(self._h, _stream(stream)))

    def mean(self, out=None, stream=None):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out
        _check(_lib.fkf_filter_mean(self._h, out.data_ptr(), _stream(stream)))
        return out

    def variance(self, out=None, stream=None):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out
        _check(_lib.fkf_filter_variance(self._h, out.data_ptr(), _stream(stream)))
        return out

    def realize(self, g, out=None, stream=None):
        g = to_device(g)
        if g.dim() == 1:
            g2 = g.reshape(self.n, 1)
        else:
            g2 = g
        ptr, ldg, ns = _colmajor(g2)
        if out is None:
            out = fortran_empty(self.n, ns)
        optr, ldo, _ = _colmajor(out if out.dim() == 2 else out.reshape(self.n, 1))
        _check(_lib.fkf_filter_realize(self._h, ptr, ns, ldg, optr, ldo, _stream(stream)))
        return out[:, 0] if g.dim() == 1 else out

    def info(self) -> dict:
        k, a, r = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32()
        _check(_lib.fkf_filter_info(self._h, ctypes.byref(k), ctypes.byref(a), ctypes.byref(r)))
        return {"k": k.value, "alpha": a.value, "rank": r.value}

    def modes(self):
        r = self.info()["rank"]
        lam = np.empty(r)
        w = np.empty(r)
        _check(_lib.fkf_filter_modes(self._h, lam.ctypes.data_as(_c_dbl_p), w.ctypes.data_as(_c_dbl_p)))
        return lam, w

    def lowrank(self, stream=None):
        """(W, Wd, D) of Sigma = alpha Gamma - W D W^T with Wd = Gamma^-1 W
        (fkf_filter_lowrank), as CUDA float64 tensors (N, r), (N, r), (r,)."""
        torch = _torch()
        cap = max(self.info()["rank"], 1)
        W = fortran_empty(self.n, cap)
        Wd = fortran_empty(self.n, cap)
        D = torch.empty(cap, dtype=torch.float64, device="cuda")
        r = ctypes.c_int32()
        _check(_lib.fkf_filter_lowrank(self._h, W.data_ptr(), self.n, Wd.data_ptr(), self.n,
                                       D.data_ptr(), cap, ctypes.byref(r), _stream(stream)))
        k = r.value
        return W[:, :k], Wd[:, :k], D[:k]

    def close(self):
        if getattr(self, "_h", None):
            _lib.fkf_filter_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

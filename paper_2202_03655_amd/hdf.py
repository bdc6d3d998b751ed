"""Python binding of the HDF C ABI (include/hdf.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the computation runs in the library's kernels.  The
library must have been built in-tree (``__graft_entry__.build()``); importing
this module without it raises, there is no fallback path.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libhdf.so")

KERNELS = {"gaussian": 0, "cauchy": 1, "matern32": 2, "matern52": 3}
HDF_FP64, HDF_MIXED = 0, 1
HDF_MAX_DEGREE = 60
HDF_SPLIT_TOL = 1e-6
STATUS = {0: "HDF_OK", -1: "HDF_E_ARG", -2: "HDF_E_DIM", -3: "HDF_E_NONFINITE",
          -4: "HDF_E_INFEASIBLE", -5: "HDF_E_OOM", -6: "HDF_E_HIP", -7: "HDF_E_DISABLED"}

EXPORTS = ["hdf_build", "hdf_build_ex", "hdf_build_cross", "hdf_matvec", "hdf_matvec_noalloc", "hdf_backward",
           "hdf_info", "hdf_get_plan",
           "hdf_copy_factor", "hdf_copy_factor_y", "hdf_free", "hdf_status_string", "hdf_last_error",
           "hdf_plan_chebyshev", "hdf_plan_degree", "hdf_plan_cores", "hdf_plan_index_set",
           "hdf_plan_compress_cross", "hdf_kmeans", "hdf_kernel_matvec", "hdf_krr_create", "hdf_krr_apply",
           "hdf_krr_precond", "hdf_krr_solve", "hdf_krr_info", "hdf_krr_block", "hdf_krr_free"]

KMEANS_SEED = 0x48444602


class HDFInfo(ctypes.Structure):
    _fields_ = [
        ("n_dim", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_points", ctypes.c_int64),
        ("n_points_y", ctypes.c_int64),
        ("degree_p", ctypes.c_int32), ("n_degrees", ctypes.c_int32),
        ("n_harmonics", ctypes.c_int64), ("n_radial", ctypes.c_int64), ("rank", ctypes.c_int64),
        ("tau", ctypes.c_double), ("nu", ctypes.c_double), ("cheb_tail", ctypes.c_double),
        ("center_radius", ctypes.c_double), ("rho2_min", ctypes.c_double),
        ("rho2_max", ctypes.c_double), ("factor_bytes", ctypes.c_int64),
        ("t_prep_ms", ctypes.c_double), ("t_plan_ms", ctypes.c_double),
        ("t_gram_ms", ctypes.c_double), ("t_compress_ms", ctypes.c_double), ("t_finish_ms", ctypes.c_double),
        ("t_build_ms", ctypes.c_double), ("t_mv_t_ms", ctypes.c_double),
        ("t_mv_reduce_ms", ctypes.c_double), ("t_mv_n_ms", ctypes.c_double),
        ("t_adjoint_ms", ctypes.c_double),
        ("n_refined", ctypes.c_int32),
        ("s_k", ctypes.c_int32 * (HDF_MAX_DEGREE // 2 + 1)),
        ("rank_rule", ctypes.c_int32), ("tau_bound", ctypes.c_double), ("est_error", ctypes.c_double),
        ("degree_bound", ctypes.c_int32), ("storage", ctypes.c_int32), ("chunk_points", ctypes.c_int64),
        ("factor_precision", ctypes.c_int32), ("mf_fused", ctypes.c_int32),
    ]


class BuildOptions(ctypes.Structure):
    _fields_ = [("rank_rule", ctypes.c_int32), ("n_pairs", ctypes.c_int32), ("margin", ctypes.c_double),
                ("storage", ctypes.c_int32), ("chunked", ctypes.c_int32), ("chunk", ctypes.c_int64)]


RANK_RULES = {"bound": 0, "sampled": 1}
STORAGE = {"factor": 0, "none": 1}


class KRRInfo(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int64), ("n_dim", ctypes.c_int32), ("n_clusters", ctypes.c_int32),
        ("n_blocks", ctypes.c_int32), ("max_block", ctypes.c_int32), ("max_degree", ctypes.c_int32),
        ("sum_rank", ctypes.c_int64), ("factor_bytes", ctypes.c_int64), ("precond_bytes", ctypes.c_int64),
        ("t_factor_ms", ctypes.c_double), ("t_precond_ms", ctypes.c_double), ("t_offdiag_ms", ctypes.c_double),
        ("t_solve_ms", ctypes.c_double), ("last_iterations", ctypes.c_int32), ("last_relres", ctypes.c_double),
    ]


class HDFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.hdf_build.argtypes = [vp, i32, i64, i32, i64, i32, dbl, dbl, i32, vp, ctypes.POINTER(vp)]
    L.hdf_build_ex.argtypes = [vp, i32, i64, i32, i64, i32, dbl, dbl, i32, ctypes.POINTER(BuildOptions), vp,
                               ctypes.POINTER(vp)]
    L.hdf_build_cross.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, dbl, dbl, i32, vp,
                                  ctypes.POINTER(vp)]
    L.hdf_copy_factor_y.argtypes = [vp, vp, i64, vp, i64, vp]
    L.hdf_plan_compress_cross.argtypes = [i32, vp, vp, vp, dbl, dbl, ctypes.POINTER(ctypes.c_int32), vp, vp, vp]
    L.hdf_matvec.argtypes = [vp, vp, i64, i64, vp, i64, vp]
    L.hdf_matvec_noalloc.argtypes = [vp, vp, i64, i64, vp, i64, vp]
    L.hdf_backward.argtypes = [vp, vp, vp, i64, i64, ctypes.POINTER(dbl), vp, i64, vp]
    L.hdf_info.argtypes = [vp, ctypes.POINTER(HDFInfo)]
    L.hdf_get_plan.argtypes = [vp, vp, vp, vp, vp]
    L.hdf_copy_factor.argtypes = [vp, vp, i64, vp, i64, vp]
    L.hdf_free.argtypes = [vp]
    L.hdf_free.restype = None
    L.hdf_status_string.argtypes = [i32]
    L.hdf_status_string.restype = ctypes.c_char_p
    L.hdf_last_error.restype = ctypes.c_char_p
    L.hdf_plan_chebyshev.argtypes = [i32, dbl, dbl, i32, i32, vp]
    L.hdf_plan_degree.argtypes = [vp, i32, dbl, dbl, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.hdf_plan_cores.argtypes = [vp, i32, i32, dbl, dbl, vp]
    L.hdf_plan_index_set.argtypes = [i32, i32, vp, ctypes.POINTER(i64)]
    L.hdf_kmeans.argtypes = [vp, i64, i32, i64, i32, i32, ctypes.c_uint64, vp, vp, ctypes.POINTER(i32), vp]
    L.hdf_kernel_matvec.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, dbl, vp, vp, vp]
    L.hdf_krr_create.argtypes = [vp, i64, i32, i64, vp, i32, i32, dbl, dbl, dbl, vp, ctypes.POINTER(vp)]
    L.hdf_krr_apply.argtypes = [vp, vp, vp, vp]
    L.hdf_krr_precond.argtypes = [vp, vp, vp, vp]
    L.hdf_krr_solve.argtypes = [vp, vp, vp, i32, dbl, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
    L.hdf_krr_info.argtypes = [vp, ctypes.POINTER(KRRInfo)]
    L.hdf_krr_block.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.hdf_krr_free.argtypes = [vp]
    L.hdf_krr_free.restype = None
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("hdf_free", "hdf_status_string", "hdf_last_error", "hdf_krr_free"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise HDFError(status, lib().hdf_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev2d(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() == 1:
        t = t.unsqueeze(1)
    if t.dim() != 2 or t.stride(1) != 1:
        t = t.contiguous()
    return t


def _check_out(out, n, m, dtype, device):
    """A caller-supplied output of a product: n x m, the factor's dtype and device, unit inner
    stride (the library writes rows of m values at out + i * stride(0)); None allocates one."""
    if out is None:
        return torch.empty((n, m), dtype=dtype, device=device)
    if not isinstance(out, torch.Tensor) or not out.is_cuda:
        raise TypeError("out must be a CUDA (HIP) tensor")
    if out.dtype != dtype:
        raise TypeError(f"out must be {dtype}, got {out.dtype}")
    if out.device != device:
        raise ValueError(f"out must be on {device}, got {out.device}")
    if out.dim() != 2 or tuple(out.shape) != (n, m):
        raise ValueError(f"out must have shape ({n}, {m}), got {tuple(out.shape)}")
    if out.stride(1) != 1 or out.stride(0) < m:
        raise ValueError("out must have unit inner stride and row stride >= m")
    return out


class Factor:
    """Handle of a built HDF factor K ~ U D U^T (owns the library handle)."""

    def __init__(self, X, kernel="gaussian", lengthscale=1.0, tol=1e-4, precision=None, rank_rule="bound",
                 n_pairs=0, margin=0.0, storage="factor", chunk=0, fused=True):
        """rank_rule "bound": p and tau from the a-priori budget (Sec. 3.5); "sampled": the tighter
        rule of the remark after Eq. bound (n_pairs sampled pairs, error kept <= margin * tol;
        0 selects the library defaults).  storage "none": matrix-free, the factor is re-evaluated
        in every pass: inside the fused kernels when `fused` and the harmonics of 16 points fit in
        LDS, else per chunk of `chunk` points (0: the library default)."""
        L = lib()
        if precision is None:
            precision = HDF_FP64 if X.dtype == torch.float64 else HDF_MIXED
        dtype = torch.float64 if precision == HDF_FP64 else torch.float32
        X = _dev2d(X, dtype, "X")
        self.n, self.d = X.shape
        self.dtype = dtype
        self.precision = precision
        self.kernel = kernel
        self.lengthscale = float(lengthscale)
        self.tol = float(tol)
        self.device = X.device
        h = ctypes.c_void_p()
        opts = BuildOptions(RANK_RULES[rank_rule], int(n_pairs), float(margin), STORAGE[storage],
                            0 if fused else 1, int(chunk))
        with torch.cuda.device(X.device):
            _check(L.hdf_build_ex(X.data_ptr(), 0 if dtype == torch.float32 else 1, self.n, self.d,
                                  X.stride(0), KERNELS[kernel], self.lengthscale, self.tol,
                                  precision, ctypes.byref(opts), _stream(), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and getattr(self, "_owned", True):
            _lib.hdf_free(h)
            self._h = None

    # -- application ------------------------------------------------------
    def matvec(self, V, out=None):
        """K~ V for V of shape (n,) or (n, m)."""
        squeeze = V.dim() == 1
        V2 = _dev2d(V, self.dtype, "V")
        if V2.shape[0] != self.n:
            raise ValueError("V must have n rows")
        m = V2.shape[1]
        out = _check_out(out, self.n, m, self.dtype, V2.device)
        _check(lib().hdf_matvec(self._h, V2.data_ptr(), m, V2.stride(0), out.data_ptr(),
                                out.stride(0), _stream()))
        return out[:, 0] if squeeze else out

    def matvec_noalloc(self, V, out):
        """K~ V into a caller-supplied out (n x m, m <= 64) through hdf_matvec_noalloc: no device
        allocation inside the library (its work buffers are a fixed per-GPU array)."""
        V2 = _dev2d(V, self.dtype, "V")
        if V2.shape[0] != self.n:
            raise ValueError("V must have n rows")
        m = V2.shape[1]
        if out is None:
            raise ValueError("out is required (nothing is allocated)")
        out = _check_out(out, self.n, m, self.dtype, V2.device)
        _check(lib().hdf_matvec_noalloc(self._h, V2.data_ptr(), m, V2.stride(0), out.data_ptr(), out.stride(0),
                                        _stream()))
        return out

    def backward(self, W, V, need_l=True, need_x=True):
        """(dF/dl, dF/dX) for F = sum_c w_c^T K~ v_c (structure frozen)."""
        W2 = _dev2d(W, self.dtype, "W")
        V2 = _dev2d(V, self.dtype, "V")
        if W2.shape != V2.shape or W2.shape[0] != self.n:
            raise ValueError("W and V must both be n x m")
        if W2.stride(0) != V2.stride(0):
            W2, V2 = W2.contiguous(), V2.contiguous()
        m = W2.shape[1]
        dl = ctypes.c_double(0.0)
        dX = torch.empty((self.n, self.d), dtype=self.dtype, device=W2.device) if need_x else None
        _check(lib().hdf_backward(self._h, W2.data_ptr(), V2.data_ptr(), m, W2.stride(0),
                                  ctypes.byref(dl) if need_l else None,
                                  dX.data_ptr() if need_x else None, self.d, _stream()))
        return (dl.value if need_l else None), dX

    # -- inspection -------------------------------------------------------
    def info(self):
        inf = HDFInfo()
        _check(lib().hdf_info(self._h, ctypes.byref(inf)))
        out = {name: getattr(inf, name) for name, _ in HDFInfo._fields_ if name != "s_k"}
        out["s_k"] = [inf.s_k[k] for k in range(inf.n_degrees)]
        return out

    def plan(self):
        import numpy as np
        inf = self.info()
        H, S, d, p = inf["n_harmonics"], inf["n_radial"], self.d, inf["degree_p"]
        K = p // 2
        ncoef = sum((K - k + 1) * s for k, s in enumerate(inf["s_k"]))
        table = np.zeros((max(H, 1), d - 1), dtype=np.int32)
        lam = np.zeros(max(S, 1))
        coef = np.zeros(max(ncoef, 1))
        a = np.zeros(p + 1)
        _check(lib().hdf_get_plan(self._h, table.ctypes.data, lam.ctypes.data, coef.ctypes.data,
                                  a.ctypes.data))
        return dict(index_table=table[:H], lam=lam[:S], radial_coef=coef[:ncoef], a=a, info=inf)

    def factor_dtype(self):
        """Storage type of the factor (binary64 for HDF_MIXED builds at tol <= HDF_SPLIT_TOL)."""
        return torch.float32 if self.info()["factor_precision"] == HDF_MIXED else torch.float64

    def factor_parts(self):
        """(phi, q) copies: H x n harmonics and S x n radial functions, in the factor's storage type."""
        inf = self.info()
        fdt = self.factor_dtype()
        phi = torch.empty((inf["n_harmonics"], self.n), dtype=fdt, device=self.device)
        q = torch.empty((inf["n_radial"], self.n), dtype=fdt, device=self.device)
        _check(lib().hdf_copy_factor(self._h, phi.data_ptr() if phi.numel() else None, self.n,
                                     q.data_ptr() if q.numel() else None, self.n, _stream()))
        return phi, q


class CrossFactor(Factor):
    """Handle of a general factor K(X, Y) ~ U V^T (hdf_build_cross).

    matvec(W) applies K(X, Y) to W (n_y rows) and returns n_x rows; backward
    is not defined for it."""

    def __init__(self, X, Y, kernel="gaussian", lengthscale=1.0, tol=1e-4, precision=None):
        L = lib()
        if precision is None:
            precision = HDF_FP64 if X.dtype == torch.float64 else HDF_MIXED
        dtype = torch.float64 if precision == HDF_FP64 else torch.float32
        X = _dev2d(X, dtype, "X")
        Y = _dev2d(Y, dtype, "Y")
        if X.shape[1] != Y.shape[1]:
            raise ValueError("X and Y must have the same number of columns")
        self.n, self.d = X.shape
        self.n_y = Y.shape[0]
        self.dtype = dtype
        self.precision = precision
        self.kernel = kernel
        self.lengthscale = float(lengthscale)
        self.tol = float(tol)
        self.device = X.device
        h = ctypes.c_void_p()
        with torch.cuda.device(X.device):
            _check(L.hdf_build_cross(X.data_ptr(), self.n, X.stride(0), Y.data_ptr(), self.n_y, Y.stride(0),
                                     0 if dtype == torch.float32 else 1, self.d, KERNELS[kernel],
                                     self.lengthscale, self.tol, precision, _stream(), ctypes.byref(h)))
        self._h = h

    def matvec(self, W, out=None):
        """K(X, Y) W for W of shape (n_y,) or (n_y, m)."""
        squeeze = W.dim() == 1
        W2 = _dev2d(W, self.dtype, "W")
        if W2.shape[0] != self.n_y:
            raise ValueError("W must have n_y rows")
        m = W2.shape[1]
        out = _check_out(out, self.n, m, self.dtype, W2.device)
        _check(lib().hdf_matvec(self._h, W2.data_ptr(), m, W2.stride(0), out.data_ptr(),
                                out.stride(0), _stream()))
        return out[:, 0] if squeeze else out

    def backward(self, W, V, need_l=True, need_x=True):
        raise HDFError(-1, "backward is defined for the symmetric factor only")

    def factor_parts_y(self):
        """(phi, q) copies at the Y points: H x n_y and S x n_y."""
        inf = self.info()
        fdt = self.factor_dtype()
        phi = torch.empty((inf["n_harmonics"], self.n_y), dtype=fdt, device=self.device)
        q = torch.empty((inf["n_radial"], self.n_y), dtype=fdt, device=self.device)
        _check(lib().hdf_copy_factor_y(self._h, phi.data_ptr() if phi.numel() else None, self.n_y,
                                       q.data_ptr() if q.numel() else None, self.n_y, _stream()))
        return phi, q


def build(X, kernel="gaussian", lengthscale=1.0, tol=1e-4, precision=None):
    return Factor(X, kernel, lengthscale, tol, precision)


class HDFMatvec(torch.autograd.Function):
    """y = K~(X, l) V with gradients for V, l and X (structure frozen at build)."""

    @staticmethod
    def forward(ctx, X, lengthscale, V, factor):
        ctx.factor = factor
        ctx.save_for_backward(V)
        return factor.matvec(V)

    @staticmethod
    def backward(ctx, G):
        (V,) = ctx.saved_tensors
        f = ctx.factor
        G = G.contiguous()
        dV = f.matvec(G) if ctx.needs_input_grad[2] else None
        need_l, need_x = ctx.needs_input_grad[1], ctx.needs_input_grad[0]
        dl = dX = None
        if need_l or need_x:
            Vm = V if V.dim() == 2 else V.unsqueeze(1)
            Gm = G if G.dim() == 2 else G.unsqueeze(1)
            dlv, dX = f.backward(Gm, Vm, need_l=need_l, need_x=need_x)
            if need_l:
                dl = torch.tensor(dlv, dtype=f.dtype, device=G.device)
        return dX, dl, dV, None


# -- host planner (no device work) ------------------------------------------
def plan_chebyshev(kernel, D, lengthscale, n_nodes=8192, derivative=False):
    import numpy as np
    a = np.zeros(n_nodes)
    _check(lib().hdf_plan_chebyshev(KERNELS[kernel], float(D), float(lengthscale), n_nodes,
                                    int(derivative), a.ctypes.data))
    return a


def plan_degree(a, eps, nu, p_max=HDF_MAX_DEGREE):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    p = ctypes.c_int(0)
    tail = ctypes.c_double(0.0)
    _check(lib().hdf_plan_degree(a.ctypes.data, len(a), float(eps), float(nu), p_max,
                                 ctypes.byref(p), ctypes.byref(tail)))
    return p.value, tail.value


def plan_cores(a, p, d, u0, u1):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    K = p // 2
    tot = sum((K - k + 1) ** 2 for k in range(K + 1))
    out = np.zeros(tot)
    _check(lib().hdf_plan_cores(a.ctypes.data, p, d, float(u0), float(u1), out.ctypes.data))
    cores, o = [], 0
    for k in range(K + 1):
        L = K - k + 1
        cores.append(out[o:o + L * L].reshape(L, L))
        o += L * L
    return cores


def plan_compress_cross(Gx, Gy, M, tau, null_rel=1e-15):
    """Cross compression of one degree (single pass): (sig, Ex, Ey)."""
    import numpy as np
    L = M.shape[0]
    Gx, Gy, M = (np.ascontiguousarray(a, dtype=np.float64) for a in (Gx, Gy, M))
    s = ctypes.c_int32(0)
    sig = np.zeros(L)
    Ex = np.zeros(L * L)
    Ey = np.zeros(L * L)
    _check(lib().hdf_plan_compress_cross(L, Gx.ctypes.data, Gy.ctypes.data, M.ctypes.data, float(tau),
                                         float(null_rel), ctypes.byref(s), sig.ctypes.data, Ex.ctypes.data,
                                         Ey.ctypes.data))
    n = s.value
    return sig[:n], Ex[:n * L].reshape(n, L).T, Ey[:n * L].reshape(n, L).T


def plan_index_set(d, k):
    import numpy as np
    cnt = ctypes.c_int64(0)
    _check(lib().hdf_plan_index_set(d, k, None, ctypes.byref(cnt)))
    t = np.zeros((max(cnt.value, 1), d - 2), dtype=np.int32)
    _check(lib().hdf_plan_index_set(d, k, t.ctypes.data, ctypes.byref(cnt)))
    return t[:cnt.value]


# -- kernel ridge regression consumer (Sec. 4.2) -----------------------------
def _dev1d(t, name, n=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    t = t.reshape(-1).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    return t


def _dev_i32(t, name, n):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32:
        raise TypeError(f"{name} must be an int32 CUDA (HIP) tensor")
    t = t.reshape(-1).contiguous()
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    return t


def kmeans(X, k, max_iter=100, seed=KMEANS_SEED):
    """Lloyd's k-means on the device: (labels int32 (n,), centres (k, d), assignments made)."""
    X = _dev2d(X, torch.float64, "X")
    n, d = X.shape
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    centres = torch.empty((k, d), dtype=torch.float64, device=X.device)
    its = ctypes.c_int(0)
    with torch.cuda.device(X.device):
        _check(lib().hdf_kmeans(X.data_ptr(), n, d, X.stride(0), int(k), int(max_iter), int(seed),
                                labels.data_ptr(), centres.data_ptr(), ctypes.byref(its), _stream()))
    return labels, centres, its.value


def kernel_matvec(X, Y, w, kernel="gaussian", lengthscale=1.0):
    """K(X, Y) w with exact kernel values (binary64)."""
    X = _dev2d(X, torch.float64, "X")
    Y = _dev2d(Y, torch.float64, "Y")
    if X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must have the same number of columns")
    w = _dev1d(w, "w", Y.shape[0])
    out = torch.empty(X.shape[0], dtype=torch.float64, device=X.device)
    with torch.cuda.device(X.device):
        _check(lib().hdf_kernel_matvec(X.data_ptr(), X.shape[0], X.stride(0), Y.data_ptr(), Y.shape[0], Y.stride(0),
                                       X.shape[1], KERNELS[kernel], float(lengthscale), w.data_ptr(), out.data_ptr(),
                                       _stream()))
    return out


class KRR:
    """The KRR system (lambda I + K) with HDF diagonal blocks per cluster (owns the library handle)."""

    def __init__(self, X, labels, k, kernel="gaussian", lengthscale=1.0, tol=1e-4, lam=0.1):
        X = _dev2d(X, torch.float64, "X")
        self.n, self.d = X.shape
        labels = _dev_i32(labels, "labels", self.n)
        self.k, self.kernel, self.lengthscale = int(k), kernel, float(lengthscale)
        self.device = X.device
        h = ctypes.c_void_p()
        with torch.cuda.device(X.device):
            _check(lib().hdf_krr_create(X.data_ptr(), self.n, self.d, X.stride(0), labels.data_ptr(), self.k,
                                        KERNELS[kernel], self.lengthscale, float(tol), float(lam), _stream(),
                                        ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hdf_krr_free(h)
            self._h = None

    def apply(self, v):
        v = _dev1d(v, "v", self.n)
        out = torch.empty_like(v)
        _check(lib().hdf_krr_apply(self._h, v.data_ptr(), out.data_ptr(), _stream()))
        return out

    def precond(self, r):
        r = _dev1d(r, "r", self.n)
        z = torch.empty_like(r)
        _check(lib().hdf_krr_precond(self._h, r.data_ptr(), z.data_ptr(), _stream()))
        return z

    def solve(self, y, max_iter=1024, rtol=1e-6):
        """(w, iterations, relative residual) of preconditioned CG from w = 0."""
        y = _dev1d(y, "y", self.n)
        w = torch.empty_like(y)
        its, rel = ctypes.c_int(0), ctypes.c_double(0.0)
        _check(lib().hdf_krr_solve(self._h, y.data_ptr(), w.data_ptr(), int(max_iter), float(rtol),
                                   ctypes.byref(its), ctypes.byref(rel), _stream()))
        return w, its.value, rel.value

    def info(self):
        inf = KRRInfo()
        _check(lib().hdf_krr_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in KRRInfo._fields_}

    def block(self, c):
        """The HDF factor of cluster c (None if empty), borrowed from this handle."""
        h = ctypes.c_void_p()
        _check(lib().hdf_krr_block(self._h, int(c), ctypes.byref(h)))
        if not h.value:
            return None
        f = Factor.__new__(Factor)
        f._h, f._owned, f._parent = h, False, self
        inf = f.info()
        f.n, f.d, f.dtype, f.precision = inf["n_points"], inf["n_dim"], torch.float64, HDF_FP64
        f.kernel, f.lengthscale, f.device = self.kernel, self.lengthscale, self.device
        return f

"""ctypes binding of ``libcpng.so`` (the C ABI declared in include/cpng.h).

Argument marshalling only: torch tensors are checked (device, dtype,
contiguity, size) and passed as raw device pointers together with the current
HIP stream; every computation runs in the library's kernels.  There is no
fallback: if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpng.so")

CP_MAX_ORDER = 8
CP_OK, CP_EINVAL, CP_ENOMEM, CP_EDEVICE = 0, -1, -2, -3
CP_ESINGULAR, CP_EDUPLICATE, CP_ENOTFINITE = -4, -5, -6
CP_MAXITER, CP_LS_FALLBACK = 1, 2
CP_F32, CP_F64 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp32in_fp64acc": 3}
CP_METHOD_NGMRES, CP_METHOD_ALS, CP_METHOD_NCG, CP_METHOD_NGMRES_SD = 0, 1, 2, 3
CP_INIT_GIVEN, CP_INIT_SEEDED = 0, 1
LS_STATUS = {0: "converged", 1: "maxfev", 2: "xtol", 3: "stpmax", 4: "stpmin", 5: "rounding",
             -1: ""}


class CpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cpng error {code}: {msg}")
        self.code = code


class cp_tensor(C.Structure):
    _fields_ = [("order", C.c_int32), ("dims", C.c_int64 * CP_MAX_ORDER), ("sparse", C.c_int32),
                ("dtype", C.c_int32), ("values", C.c_void_p), ("nnz", C.c_int64),
                ("coords", C.c_void_p), ("prepared", C.c_void_p), ("norm_sq", C.c_double)]


class cp_iter_info(C.Structure):
    _fields_ = [("it", C.c_int32), ("f", C.c_double), ("rho", C.c_double), ("beta", C.c_double),
                ("restart", C.c_int32), ("nfev", C.c_int32), ("ls_status", C.c_int32),
                ("m", C.c_int32), ("precision", C.c_int32), ("t_passes", C.c_int32),
                ("nfev_pre", C.c_int32)]


class cp_options(C.Structure):
    _fields_ = [("method", C.c_int32), ("window", C.c_int32), ("eps", C.c_double),
                ("ls_ftol", C.c_double), ("ls_gtol", C.c_double), ("ls_stp0", C.c_double),
                ("ls_maxfev", C.c_int32), ("ls_xtol", C.c_double), ("ls_stpmin", C.c_double),
                ("ls_stpmax", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("final_precision", C.c_int32), ("switch_rho", C.c_double),
                ("normalize_accel", C.c_int32), ("trace", C.POINTER(cp_iter_info)),
                ("trace_cap", C.c_int32), ("mttkrp_tree", C.c_int32),
                ("switch_on_stall", C.c_int32), ("stop_tol", C.c_double), ("init", C.c_int32),
                ("seed", C.c_uint64)]


class cp_ngmres_meta(C.Structure):
    _fields_ = [("it", C.c_int32), ("m", C.c_int32), ("precision", C.c_int32),
                ("switched", C.c_int32), ("stalled", C.c_int32), ("cg_fresh", C.c_int32),
                ("f", C.c_double), ("rho", C.c_double), ("n_fg", C.c_int32),
                ("n_restarts", C.c_int32), ("n_ls_fallback", C.c_int32), ("switch_iter", C.c_int32)]


class cp_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("f", C.c_double),
                ("rho", C.c_double), ("n_fg", C.c_int32), ("n_restarts", C.c_int32),
                ("n_ls_fallback", C.c_int32), ("switch_iter", C.c_int32), ("n_trace", C.c_int32),
                ("seconds", C.c_double)]


class cp_batch_request(C.Structure):
    _fields_ = [("T", C.POINTER(cp_tensor)), ("R", C.c_int32), ("tol", C.c_double),
                ("u_inout", C.c_void_p), ("trace", C.POINTER(cp_iter_info)),
                ("trace_cap", C.c_int32), ("status", C.c_int32), ("report", cp_report)]


class cp_server_opts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("hbm_budget", C.c_size_t), ("decompose", cp_options),
                ("batch_elems", C.c_int64), ("batch_capacity", C.c_int32)]


class cp_result(C.Structure):
    _fields_ = [("req_id", C.c_int64), ("tag", C.c_uint64), ("status", C.c_int32),
                ("iters", C.c_int32), ("converged", C.c_int32), ("n_fg", C.c_int32),
                ("switch_iter", C.c_int32), ("slot", C.c_int32), ("f", C.c_double),
                ("rho", C.c_double), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_end", C.c_double)]


_lib = None


def lib():
    """Load libcpng.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1105_5331_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "cp_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(vp)]),
            "cp_destroy": (C.c_int, [vp]),
            "cp_last_error": (C.c_char_p, [vp]),
            "cp_options_default": (None, [C.POINTER(cp_options)]),
            "cp_tensor_prepare": (C.c_int, [vp, C.POINTER(cp_tensor), vp]),
            "cp_tensor_release": (C.c_int, [vp, C.POINTER(cp_tensor)]),
            "cp_mttkrp": (C.c_int, [vp, C.POINTER(cp_tensor), vp, i32, i32, i32, vp, vp]),
            "cp_mttkrp_noalloc": (C.c_int, [vp, C.POINTER(cp_tensor), vp, i32, i32, i32, vp, vp]),
            "cp_gram": (C.c_int, [vp, i32, C.POINTER(i64), vp, i32, vp, vp, vp, vp]),
            "cp_normalize": (C.c_int, [vp, i32, C.POINTER(i64), vp, i32, vp, vp]),
            "cp_als_sweep": (C.c_int, [vp, C.POINTER(cp_tensor), vp, i32, i32, i32, vp]),
            "cp_objective_grad": (C.c_int, [vp, C.POINTER(cp_tensor), vp, i32, i32, vp, vp, vp]),
            "cp_mode_solve": (C.c_int, [vp, vp, vp, i64, i32, vp, C.POINTER(i32), vp]),
            "ngmres_accelerate": (C.c_int, [vp, i64, i32, vp, vp, vp, vp, dp, vp, vp, vp, vp]),
            "cp_init_uniform": (C.c_int, [vp, i64, C.c_uint64, vp, vp]),
            "cp_ngmres_save": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, C.POINTER(cp_ngmres_meta)]),
            "cp_ngmres_load": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, C.POINTER(cp_ngmres_meta)]),
            "cp_ngmres_last_step": (C.c_int, [vp, vp, vp, vp, vp, vp, C.POINTER(dp), C.POINTER(dp)]),
            "cp_ngmres_create": (C.c_int, [vp, C.POINTER(cp_tensor), i32, C.POINTER(cp_options),
                                           vp, vp, C.POINTER(vp)]),
            "ngmres_step": (C.c_int, [vp, vp, C.POINTER(cp_iter_info)]),
            "cp_ngmres_get": (C.c_int, [vp, vp, vp, vp, C.POINTER(dp), C.POINTER(dp)]),
            "cp_ngmres_destroy": (C.c_int, [vp, vp]),
            "cp_decompose": (C.c_int, [vp, C.POINTER(cp_tensor), i32, dp, C.POINTER(cp_options),
                                       vp, C.POINTER(cp_report), vp]),
            "cp_batch_decompose": (C.c_int, [vp, i32, C.POINTER(cp_batch_request),
                                             C.POINTER(cp_options), vp]),
            "cp_server_create": (C.c_int, [C.c_int, C.POINTER(cp_server_opts), C.POINTER(vp)]),
            "cp_server_submit": (C.c_int, [vp, C.POINTER(cp_tensor), i32, dp, vp, C.c_uint64,
                                           C.POINTER(i64)]),
            "cp_server_poll": (C.c_int, [vp, i32, C.POINTER(cp_result), i32, C.POINTER(i32)]),
            "cp_server_stats": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32),
                                          C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
            "cp_server_destroy": (C.c_int, [vp]),
            "cp_profile": (C.c_int, [vp, i32]),
            "cp_profile_select": (C.c_int, [vp, C.c_uint32]),
            "cp_profile_read": (C.c_int, [vp, i32, C.POINTER(i64), C.POINTER(dp)]),
            "cp_stream_read": (C.c_int, [vp, vp, C.c_size_t, vp]),
            "cp_sparse_gather_read": (C.c_int, [vp, C.POINTER(cp_tensor), vp, i32, i32, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return C.c_void_p(t.data_ptr())


class Handle:
    """A library handle on one device (cp_create / cp_destroy)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        self._h = C.c_void_p()
        rc = lib().cp_create(int(device), int(workspace_bytes), C.byref(self._h))
        if rc != CP_OK:
            raise CpError(rc, "cp_create failed")
        self.device = device

    def check(self, rc, allow=(CP_OK,)):
        if rc in allow:
            return rc
        msg = lib().cp_last_error(self._h)
        raise CpError(rc, msg.decode() if msg else "")

    def close(self):
        if self._h:
            lib().cp_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tensor:
    """A cp_tensor descriptor that keeps its torch storage alive."""

    def __init__(self, dims, values, coords=None):
        dims = tuple(int(d) for d in dims)
        if not 1 <= len(dims) <= CP_MAX_ORDER:
            raise ValueError("order must be 1..8")
        if values.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        self.dims = dims
        self.values = values.contiguous()
        self.coords = None if coords is None else coords.to(torch.int32).contiguous()
        t = cp_tensor()
        t.order = len(dims)
        for k, d in enumerate(dims):
            t.dims[k] = d
        t.sparse = 0 if coords is None else 1
        t.dtype = CP_F32 if values.dtype == torch.float32 else CP_F64
        t.values = _ptr(self.values, name="values") if self.values.numel() else None
        if coords is None:
            if self.values.numel() != math.prod(dims):
                raise ValueError("dense values must have prod(dims) elements")
            t.nnz = 0
            t.coords = None
        else:
            if tuple(self.coords.shape) != (len(dims), self.values.numel()):
                raise ValueError("coords must be (order, nnz)")
            t.nnz = self.values.numel()
            t.coords = _ptr(self.coords, name="coords") if t.nnz else None
        self.c = t
        self.prepared = False

    @property
    def sparse(self):
        return bool(self.c.sparse)

    @property
    def norm_sq(self):
        return self.c.norm_sq


def iterate_length(dims, R):
    return int(sum(dims)) * int(R)


# ---------------------------------------------------------------- calls ---

def cp_tensor_prepare(h: Handle, T: Tensor):
    h.check(lib().cp_tensor_prepare(h._h, C.byref(T.c), _stream()))
    T.prepared = True
    return T.c.norm_sq


def cp_tensor_release(h: Handle, T: Tensor):
    h.check(lib().cp_tensor_release(h._h, C.byref(T.c)))
    T.prepared = False


def cp_mttkrp(h: Handle, T: Tensor, u, R: int, mode: int, prec="fp64", M_out=None):
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    rows = T.dims[mode] if 0 <= mode < len(T.dims) else 1   # the library reports a bad mode
    if M_out is None:
        M_out = torch.empty((rows, max(int(R), 1)), dtype=torch.float64, device=u.device)
    h.check(lib().cp_mttkrp(h._h, C.byref(T.c), _ptr(u, torch.float64, iterate_length(T.dims, R), "u"),
                            int(R), int(mode), p, _ptr(M_out, torch.float64, rows * R, "M_out"),
                            _stream()))
    return M_out


def cp_mttkrp_noalloc(h: Handle, T: Tensor, u, R: int, mode: int, prec="fp64", M_out=None):
    """cp_mttkrp with the library's static scratch as workspace (no device
    allocation inside the call).  With M_out given, the binding allocates
    nothing either."""
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    rows = T.dims[mode] if 0 <= mode < len(T.dims) else 1
    if M_out is None:
        M_out = torch.empty((rows, max(int(R), 1)), dtype=torch.float64, device=u.device)
    h.check(lib().cp_mttkrp_noalloc(h._h, C.byref(T.c),
                                    _ptr(u, torch.float64, iterate_length(T.dims, R), "u"),
                                    int(R), int(mode), p,
                                    _ptr(M_out, torch.float64, rows * R, "M_out"), _stream()))
    return M_out


def cp_mode_solve(h: Handle, M, Gbar, A_out=None):
    I, R = M.shape
    if A_out is None:
        A_out = torch.empty((I, R), dtype=torch.float64, device=M.device)
    kind = C.c_int32()
    h.check(lib().cp_mode_solve(h._h, _ptr(M, torch.float64, I * R, "M"),
                                _ptr(Gbar, torch.float64, R * R, "Gbar"), int(I), int(R),
                                _ptr(A_out, torch.float64, I * R, "A_out"), C.byref(kind), _stream()))
    return A_out, kind.value


def cp_gram(h: Handle, dims, u, R: int, want_bar=True, want_gamma=True):
    N = len(dims)
    S = torch.empty((N, R, R), dtype=torch.float64, device=u.device)
    Gb = torch.empty((N, R, R), dtype=torch.float64, device=u.device) if want_bar else None
    G = torch.empty((R, R), dtype=torch.float64, device=u.device) if want_gamma else None
    d = (C.c_int64 * N)(*dims)
    h.check(lib().cp_gram(h._h, N, d, _ptr(u, torch.float64, iterate_length(dims, R), "u"), int(R),
                          _ptr(S), _ptr(Gb), _ptr(G), _stream()))
    return S, Gb, G


def cp_normalize(h: Handle, dims, u, R: int, g=None):
    N = len(dims)
    d = (C.c_int64 * N)(*dims)
    L = iterate_length(dims, R)
    h.check(lib().cp_normalize(h._h, N, d, _ptr(u, torch.float64, L, "u"), int(R),
                               _ptr(g, torch.float64, L, "g"), _stream()))
    return u, g


def cp_als_sweep(h: Handle, T: Tensor, u, R: int, prec="fp64", normalize=True):
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    h.check(lib().cp_als_sweep(h._h, C.byref(T.c), _ptr(u, torch.float64, iterate_length(T.dims, R), "u"),
                               int(R), p, int(bool(normalize)), _stream()))
    return u


def cp_objective_grad(h: Handle, T: Tensor, u, R: int, prec="fp64", f_out=None, g_out=None,
                      want_grad=True):
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    L = iterate_length(T.dims, R)
    if f_out is None:
        f_out = torch.empty(1, dtype=torch.float64, device=u.device)
    if g_out is None and want_grad:
        g_out = torch.empty(L, dtype=torch.float64, device=u.device)
    h.check(lib().cp_objective_grad(h._h, C.byref(T.c), _ptr(u, torch.float64, L, "u"), int(R), p,
                                    _ptr(f_out, torch.float64, 1, "f_out"),
                                    _ptr(g_out, torch.float64, L, "g_out"), _stream()))
    return f_out, g_out


def ngmres_accelerate(h: Handle, U, G, u_bar, g_bar, eps=1e-12, u_hat_out=None, alpha_out=None,
                      gTd_out=None):
    """Step II; returns (u_hat, alpha, gTd) with gTd = g_bar^T (u_hat - u_bar)."""
    m, L = U.shape
    if u_hat_out is None:
        u_hat_out = torch.empty(L, dtype=torch.float64, device=U.device)
    if alpha_out is None:
        alpha_out = torch.empty(m, dtype=torch.float64, device=U.device)
    if gTd_out is None:
        gTd_out = torch.empty(1, dtype=torch.float64, device=U.device)
    h.check(lib().ngmres_accelerate(h._h, int(L), int(m), _ptr(U, torch.float64, m * L, "U"),
                                    _ptr(G, torch.float64, m * L, "G"),
                                    _ptr(u_bar, torch.float64, L, "u_bar"),
                                    _ptr(g_bar, torch.float64, L, "g_bar"), float(eps),
                                    _ptr(u_hat_out, torch.float64, L, "u_hat_out"),
                                    _ptr(gTd_out, torch.float64, 1, "gTd_out"),
                                    _ptr(alpha_out, torch.float64, m, "alpha_out"), _stream()))
    return u_hat_out, alpha_out, gTd_out


def cp_init_uniform(h: Handle, L: int, seed: int, u_out=None, device="cuda"):
    """The seeded uniform initial guess (Philox-4x64-10 stream of `seed`)."""
    if u_out is None:
        u_out = torch.empty(int(L), dtype=torch.float64, device=device)
    h.check(lib().cp_init_uniform(h._h, int(L), C.c_uint64(int(seed) & (2**64 - 1)),
                                  _ptr(u_out, torch.float64, int(L), "u_out"), _stream()))
    return u_out


def options(**kw):
    o = cp_options()
    lib().cp_options_default(C.byref(o))
    for k, v in kw.items():
        if k in ("precision", "final_precision") and isinstance(v, str):
            v = PREC[v]
        if k == "method" and isinstance(v, str):
            v = {"ngmres": CP_METHOD_NGMRES, "als": CP_METHOD_ALS, "ncg": CP_METHOD_NCG,
                 "ngmres_sd": CP_METHOD_NGMRES_SD}[v]
        if k == "init" and isinstance(v, str):
            v = {"given": CP_INIT_GIVEN, "seeded": CP_INIT_SEEDED}[v]
        setattr(o, k, v)
    return o


class NGMRESState:
    """Stateful N-GMRES iteration (cp_ngmres_create / ngmres_step / cp_ngmres_get)."""

    def __init__(self, h: Handle, T: Tensor, R: int, u0, **opts):
        """u0: device initial guess, or None with init="seeded" and a seed."""
        self.h, self.T, self.R = h, T, R
        self.opt = options(**opts)
        self._s = C.c_void_p()
        h.check(lib().cp_ngmres_create(h._h, C.byref(T.c), int(R), C.byref(self.opt),
                                       _ptr(u0, torch.float64, iterate_length(T.dims, R), "u0"),
                                       _stream(), C.byref(self._s)))

    def save(self, device="cuda"):
        """Checkpoint: (meta dict, U, G, u, g, d) with U, G the window, oldest first."""
        L = iterate_length(self.T.dims, self.R)
        w = max(1, int(self.opt.window))
        U = torch.empty((w, L), dtype=torch.float64, device=device)
        G = torch.empty((w, L), dtype=torch.float64, device=device)
        u, g, d = (torch.empty(L, dtype=torch.float64, device=device) for _ in range(3))
        meta = cp_ngmres_meta()
        self.h.check(lib().cp_ngmres_save(self.h._h, self._s, _ptr(U), _ptr(G), _ptr(u), _ptr(g),
                                          _ptr(d), C.byref(meta)))
        torch.cuda.synchronize()
        md = {k: getattr(meta, k) for k, _ in cp_ngmres_meta._fields_}
        return md, U[:md["m"]].clone(), G[:md["m"]].clone(), u, g, d

    def load(self, meta, U, G, u, g, d=None):
        """Resume from a checkpoint (or teacher-force the state: window, iterate, gradient)."""
        m = cp_ngmres_meta()
        for k, _ in cp_ngmres_meta._fields_:
            if k in meta:
                setattr(m, k, meta[k])
        L = iterate_length(self.T.dims, self.R)
        nU = 0 if U is None else U.shape[0] * L
        self.h.check(lib().cp_ngmres_load(self.h._h, self._s, _ptr(U, torch.float64, nU, "U"),
                                          _ptr(G, torch.float64, nU, "G"),
                                          _ptr(u, torch.float64, L, "u"),
                                          _ptr(g, torch.float64, L, "g"),
                                          _ptr(d, torch.float64, L, "d"), C.byref(m)))

    def last_step(self, device="cuda"):
        """(u_bar, g_bar, u_hat, d, f_bar, slope) of the last N-GMRES iteration."""
        L = iterate_length(self.T.dims, self.R)
        vs = [torch.empty(L, dtype=torch.float64, device=device) for _ in range(4)]
        fb, sl = C.c_double(), C.c_double()
        self.h.check(lib().cp_ngmres_last_step(self.h._h, self._s, *[_ptr(v) for v in vs],
                                               C.byref(fb), C.byref(sl)))
        torch.cuda.synchronize()
        return (*vs, fb.value, sl.value)

    def step(self):
        info = cp_iter_info()
        rc = self.h.check(lib().ngmres_step(self.h._h, self._s, C.byref(info)),
                          allow=(CP_OK, CP_LS_FALLBACK))
        return _info_dict(info) | {"rc": rc}

    def scalars(self):
        """(f, rho) of the current iterate (no device copies)."""
        f, rho = C.c_double(), C.c_double()
        self.h.check(lib().cp_ngmres_get(self.h._h, self._s, None, None, C.byref(f), C.byref(rho)))
        return f.value, rho.value

    def get(self, device="cuda"):
        L = iterate_length(self.T.dims, self.R)
        u = torch.empty(L, dtype=torch.float64, device=device)
        g = torch.empty(L, dtype=torch.float64, device=device)
        f, rho = C.c_double(), C.c_double()
        self.h.check(lib().cp_ngmres_get(self.h._h, self._s, _ptr(u), _ptr(g), C.byref(f), C.byref(rho)))
        torch.cuda.synchronize()
        return u, g, f.value, rho.value

    def close(self):
        if self._s:
            lib().cp_ngmres_destroy(self.h._h, self._s)
            self._s = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CP_KERNEL_DENSE_MTTKRP, CP_KERNEL_SPARSE_MTTKRP, CP_KERNEL_STREAM_READ, CP_KERNEL_GROUP_MTTKRP = 0, 1, 2, 3
CP_KERNEL_DENSE_MTTKRP_F64, CP_KERNEL_SPARSE_GATHER = 4, 5
CP_KERNEL_DENSE_TWOSIDED, CP_KERNEL_DENSE_TWOSIDED_F64 = 6, 7


def cp_stream_read(h: Handle, buf):
    """Streaming-read reference kernel over a device tensor (measurement only)."""
    nbytes = buf.numel() * buf.element_size()
    h.check(lib().cp_stream_read(h._h, buf.data_ptr(), nbytes, _stream()))


def cp_sparse_gather_read(h: Handle, T: Tensor, u, R: int, mode: int):
    """The sparse FP32 MTTKRP's factor-row gathers alone (measurement only)."""
    h.check(lib().cp_sparse_gather_read(h._h, C.byref(T.c),
                                        _ptr(u, torch.float64, iterate_length(T.dims, R), "u"),
                                        int(R), int(mode), _stream()))


def cp_profile(h: Handle, enable: bool):
    h.check(lib().cp_profile(h._h, int(bool(enable))))


def cp_profile_select(h: Handle, kernel_mask: int):
    """Time only the kernel ids whose bits are set in kernel_mask."""
    h.check(lib().cp_profile_select(h._h, int(kernel_mask)))


def cp_profile_read(h: Handle, kernel: int):
    n, ms = C.c_int64(), C.c_double()
    h.check(lib().cp_profile_read(h._h, int(kernel), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def ngmres_step(state: NGMRESState):
    return state.step()


def _info_dict(r: cp_iter_info):
    return {"it": r.it, "f": r.f, "rho": r.rho, "beta": r.beta, "restart": bool(r.restart),
            "nfev": r.nfev, "ls_status": LS_STATUS.get(r.ls_status, str(r.ls_status)), "m": r.m,
            "precision": r.precision, "t_passes": r.t_passes, "nfev_pre": r.nfev_pre}


def cp_decompose(h: Handle, T: Tensor, R: int, tol: float, u_inout, trace_cap=0, **opts):
    """Run the method; u_inout holds the initial guess and receives the result
    (None: the seeded guess of opts["seed"], result described by the report only)."""
    o = options(**opts)
    buf = None
    if trace_cap > 0:
        buf = (cp_iter_info * trace_cap)()
        o.trace = C.cast(buf, C.POINTER(cp_iter_info))
        o.trace_cap = trace_cap
    rep = cp_report()
    rc = h.check(lib().cp_decompose(h._h, C.byref(T.c), int(R), float(tol), C.byref(o),
                                    _ptr(u_inout, torch.float64, iterate_length(T.dims, R), "u"),
                                    C.byref(rep), _stream()),
                 allow=(CP_OK, CP_MAXITER))
    trace = [_info_dict(buf[i]) for i in range(rep.n_trace)] if buf is not None else []
    return {"rc": rc, "iters": rep.iters, "converged": bool(rep.converged), "f": rep.f,
            "rho": rep.rho, "n_fg": rep.n_fg, "n_restarts": rep.n_restarts,
            "n_ls_fallback": rep.n_ls_fallback, "switch_iter": rep.switch_iter,
            "seconds": rep.seconds, "trace": trace}


def _report_dict(rep):
    return {"iters": rep.iters, "converged": bool(rep.converged), "f": rep.f, "rho": rep.rho,
            "n_fg": rep.n_fg, "n_restarts": rep.n_restarts, "n_ls_fallback": rep.n_ls_fallback,
            "switch_iter": rep.switch_iter, "seconds": rep.seconds}


def cp_batch_decompose(h: Handle, tensors, ranks, tol, us, trace_cap=0, **opts):
    """Batched N-GMRES of several small dense requests (one launch per step
    over all of them); us[k] holds request k's initial guess and receives its
    result.  Returns one dict per request (status, report, trace)."""
    n = len(tensors)
    o = options(**opts)
    reqs = (cp_batch_request * max(1, n))()
    bufs = []
    for k, (T, R, u) in enumerate(zip(tensors, ranks, us)):
        r = reqs[k]
        r.T = C.pointer(T.c)
        r.R = int(R)
        r.tol = float(tol[k] if isinstance(tol, (list, tuple)) else tol)
        r.u_inout = _ptr(u, torch.float64, iterate_length(T.dims, R), "u")
        if trace_cap > 0:
            buf = (cp_iter_info * trace_cap)()
            bufs.append(buf)
            r.trace = C.cast(buf, C.POINTER(cp_iter_info))
            r.trace_cap = trace_cap
        else:
            bufs.append(None)
    h.check(lib().cp_batch_decompose(h._h, n, reqs, C.byref(o), _stream()))
    out = []
    for k in range(n):
        r = reqs[k]
        tr = [_info_dict(bufs[k][i]) for i in range(r.report.n_trace)] if bufs[k] is not None else []
        out.append({"status": r.status, **_report_dict(r.report), "trace": tr})
    return out


class Server:
    """Continuous-batching decomposition server (cp_server_* in the C ABI).

    submit() hands a device tensor and initial guess to the native scheduler;
    the caller's objects are kept alive here until their result is polled."""

    def __init__(self, device=0, slots=4, hbm_budget=0, batch_elems=0, batch_capacity=256,
                 **opts):
        o = cp_server_opts()
        o.slots = int(slots)
        o.hbm_budget = int(hbm_budget)
        o.decompose = options(**opts)
        o.batch_elems = int(batch_elems)
        o.batch_capacity = int(batch_capacity)
        self._s = C.c_void_p()
        rc = lib().cp_server_create(int(device), C.byref(o), C.byref(self._s))
        if rc != CP_OK:
            raise CpError(rc, "cp_server_create failed")
        self._keep = {}

    def submit(self, T: Tensor, R: int, tol: float, u_inout, tag: int = 0):
        rid = C.c_int64()
        rc = lib().cp_server_submit(self._s, C.byref(T.c), int(R), float(tol),
                                    _ptr(u_inout, torch.float64, iterate_length(T.dims, R), "u"),
                                    C.c_uint64(tag), C.byref(rid))
        if rc != CP_OK:
            raise CpError(rc, "cp_server_submit failed")
        self._keep[rid.value] = (T, u_inout)
        return rid.value

    def poll(self, wait_for=0, max_out=256):
        buf = (cp_result * max_out)()
        n = C.c_int32()
        rc = lib().cp_server_poll(self._s, int(wait_for), buf, int(max_out), C.byref(n))
        if rc != CP_OK:
            raise CpError(rc, "cp_server_poll failed")
        out = []
        for i in range(n.value):
            r = buf[i]
            d = {k: getattr(r, k) for k, _ in cp_result._fields_}
            d["converged"] = bool(d["converged"])
            self._keep.pop(r.req_id, None)
            out.append(d)
        return out

    def stats(self):
        q, a = C.c_int32(), C.c_int32()
        used, budget = C.c_size_t(), C.c_size_t()
        lib().cp_server_stats(self._s, C.byref(q), C.byref(a), C.byref(used), C.byref(budget))
        return {"queued": q.value, "active": a.value, "in_use": used.value, "budget": budget.value}

    def close(self):
        if self._s:
            lib().cp_server_destroy(self._s)
            self._s = C.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

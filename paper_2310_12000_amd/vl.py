"""Python binding of the C ABI in include/vl.h (argument marshalling only).

Every computation runs in the HIP library libvl.so built from csrc/; this
module converts torch tensors to device pointers and checks status codes.  It
raises if the library is missing: there is no fallback.

Device memory and streams come from PyTorch: inputs and outputs are CUDA
(HIP) float64 tensors on the model's device, and calls are enqueued on the
current torch stream at model creation.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvl.so")

VL_OK = 0
VL_ERR_INVALID_ARG = -1
VL_ERR_NOT_SPD = -2
VL_ERR_NO_CONVERGENCE = -3
VL_ERR_OOM = -4
VL_ERR_NONFINITE = -5
VL_ERR_HIP = -6
VL_ERR_STATE = -7
VL_ERR_TIMEOUT = -8

VL_COV_EXPONENTIAL = 0
VL_COV_MATERN32 = 1
VL_LIK_BERNOULLI_LOGIT = 0
VL_LIK_POISSON_LOG = 1
VL_LIK_GAUSSIAN = 2
VL_LIK_GAMMA = 3
VL_PREC_VADU = 0
VL_PREC_LRAC = 1
VL_PREC_LVA = 2
VL_PREC_DIAG = 3
VL_FP64 = 0
VL_MIXED = 1
VL_PRED_SIMULATION = 0
VL_PRED_LANCZOS_L1 = 1
VL_PRED_LANCZOS_L2 = 2

EXPORT = {
    "nbr": (0, torch.int32), "bval": (1, torch.float64), "D": (2, torch.float64),
    "mode": (3, torch.float64), "W": (4, torch.float64),
    "dbval_sigma2": (5, torch.float64), "dbval_rho": (6, torch.float64),
    "dD_sigma2": (7, torch.float64), "dD_rho": (8, torch.float64),
    "block_iters": (9, torch.int32), "newton_cg_iters": (10, torch.int32),
    "slq_quad": (11, torch.float64), "slq_r0z0": (12, torch.float64),
    "pred_nbr": (13, torch.int32), "pred_bval": (14, torch.float64),
    "pred_D": (15, torch.float64),
    "lrac_L": (16, torch.float64), "lrac_piv": (17, torch.int32),
    "lrac_chol": (18, torch.float64), "newton_halvings": (19, torch.int32),
    "lanczos_alpha": (20, torch.float64), "lanczos_beta": (21, torch.float64),
}


class vl_opts(ctypes.Structure):
    _fields_ = [
        ("max_newton", ctypes.c_int), ("newton_tol", ctypes.c_double),
        ("max_cg", ctypes.c_int), ("cg_tol", ctypes.c_double),
        ("pred_cg_tol", ctypes.c_double), ("num_probes", ctypes.c_int),
        ("num_pred_samples", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("precond", ctypes.c_int), ("lrac_rank", ctypes.c_int),
        ("precision", ctypes.c_int), ("pred_tile", ctypes.c_int),
        ("replay_cg_iters", ctypes.POINTER(ctypes.c_int)), ("replay_len", ctypes.c_int),
        ("pred_method", ctypes.c_int), ("lanczos_rank", ctypes.c_int),
    ]

    def __copy__(self):
        o = vl_opts()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(self), ctypes.sizeof(vl_opts))
        o._replay = getattr(self, "_replay", None)  # keeps the replayed counts alive
        return o

    def set_replay(self, counts):
        """Fix the CG iteration counts (see vl_opts.replay_cg_iters); None clears."""
        if counts is None:
            self._replay = None
            self.replay_cg_iters = None
            self.replay_len = 0
            return
        self._replay = (ctypes.c_int * len(counts))(*[int(c) for c in counts])
        self.replay_cg_iters = ctypes.cast(self._replay, ctypes.POINTER(ctypes.c_int))
        self.replay_len = len(counts)


class vl_stats(ctypes.Structure):
    _fields_ = [
        ("newton_iters", ctypes.c_int), ("cg_iters_total", ctypes.c_int),
        ("cg_iters_max", ctypes.c_int), ("hit_cap", ctypes.c_int),
        ("t_ms", ctypes.c_double), ("t_build_us", ctypes.c_double),
        ("t_mode_us", ctypes.c_double), ("t_slq_us", ctypes.c_double),
        ("t_pred_us", ctypes.c_double), ("err_vs_fp64_est", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vl_problem(ctypes.Structure):
    _fields_ = [
        ("coords", ctypes.c_void_p), ("n", ctypes.c_int64), ("m", ctypes.c_int),
        ("cov", ctypes.c_int), ("theta", ctypes.c_double * 2), ("y", ctypes.c_void_p),
        ("F", ctypes.c_void_p), ("seed", ctypes.c_uint64),
    ]


class vl_request(ctypes.Structure):
    _fields_ = [
        ("coords", ctypes.c_void_p), ("n", ctypes.c_int64), ("m", ctypes.c_int),
        ("cov", ctypes.c_int), ("theta", ctypes.c_double * 2), ("y", ctypes.c_void_p),
        ("F", ctypes.c_void_p), ("lik", ctypes.c_int), ("aux", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("coords_p", ctypes.c_void_p), ("n_p", ctypes.c_int64),
        ("Fp", ctypes.c_void_p), ("mean_out", ctypes.c_void_p), ("var_out", ctypes.c_void_p),
    ]


# void* alloc(size_t bytes, void* stream, void* ctx); void release(void* p, void* stream, void* ctx)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class VLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libvl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2310_12000_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I, I64, S = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                       ctypes.c_size_t)
    L.vl_default_opts.argtypes = [ctypes.POINTER(vl_opts)]
    L.vl_default_opts.restype = None
    L.vl_status_string.argtypes = [I]
    L.vl_status_string.restype = ctypes.c_char_p
    L.vl_last_error.argtypes = []
    L.vl_last_error.restype = ctypes.c_char_p
    L.vl_build_vecchia.argtypes = [P, I64, I, I, ctypes.POINTER(D), P, I, ctypes.POINTER(P)]
    L.vl_set_theta.argtypes = [P, ctypes.POINTER(D)]
    L.vl_find_mode.argtypes = [P, P, P, I, ctypes.POINTER(D), ctypes.POINTER(vl_opts), P,
                               ctypes.POINTER(vl_stats)]
    L.vl_neg_log_marglik.argtypes = [P, ctypes.POINTER(vl_opts), ctypes.POINTER(D),
                                     ctypes.POINTER(D), ctypes.POINTER(vl_stats)]
    L.vl_predict.argtypes = [P, P, I64, P, ctypes.POINTER(vl_opts), P, P,
                             ctypes.POINTER(vl_stats)]
    L.vl_export.argtypes = [P, I, P, S]
    L.vl_grad_offset.argtypes = [P, P]
    L.vl_estimate.argtypes = [P, P, P, I, ctypes.POINTER(D), ctypes.POINTER(vl_opts),
                              ctypes.POINTER(D), I, D, ctypes.POINTER(D), ctypes.POINTER(I),
                              ctypes.POINTER(I)]
    L.vl_grad_beta.argtypes = [P, P, I, ctypes.POINTER(D)]
    L.vl_estimate_glm.argtypes = [P, P, P, I, I, ctypes.POINTER(vl_opts), ctypes.POINTER(D), I,
                                  D, ctypes.POINTER(D), ctypes.POINTER(I), ctypes.POINTER(I)]
    L.vl_grad_aux.argtypes = [P, ctypes.POINTER(D)]
    L.vl_export_count.argtypes = [P, I]
    L.vl_export_count.restype = I64
    L.vl_spmm.argtypes = [P, I, P, P, I]
    L.vl_trsm.argtypes = [P, I, P, P, I]
    L.vl_trsm_noalloc.argtypes = [P, I, P, P, I]
    L.vl_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
    L.vl_timing_enable.argtypes = [P, I]
    L.vl_timing_read.argtypes = [P, I, ctypes.POINTER(D), ctypes.POINTER(I64), ctypes.POINTER(D)]
    L.vl_free.argtypes = [P]
    L.vl_free.restype = None
    L.vl_batch_create.argtypes = [ctypes.POINTER(vl_problem), I, I, ctypes.POINTER(D), P,
                                  ctypes.POINTER(P)]
    L.vl_batch_fit.argtypes = [P, ctypes.POINTER(vl_opts), ctypes.POINTER(D)]
    L.vl_batch_mode.argtypes = [P, I, P]
    L.vl_batch_stats.argtypes = [P, I, ctypes.POINTER(vl_stats)]
    L.vl_batch_tuned_path.argtypes = [P, I]
    L.vl_batch_tuned_path.restype = I
    L.vl_batch_free.argtypes = [P]
    L.vl_batch_free.restype = None
    L.vl_server_create.argtypes = [I, D, ctypes.POINTER(vl_opts), ctypes.POINTER(P)]
    L.vl_server_submit.argtypes = [P, ctypes.POINTER(vl_request), ctypes.POINTER(I64)]
    L.vl_server_wait.argtypes = [P, I64, ctypes.POINTER(D), ctypes.POINTER(vl_stats),
                                 ctypes.POINTER(D)]
    L.vl_server_info.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I)]
    L.vl_request_bytes.argtypes = [ctypes.POINTER(vl_request), ctypes.POINTER(vl_opts)]
    L.vl_request_bytes.restype = D
    L.vl_server_free.argtypes = [P]
    L.vl_server_free.restype = None
    for f in ("vl_build_vecchia", "vl_set_theta", "vl_find_mode", "vl_neg_log_marglik",
              "vl_predict", "vl_export", "vl_spmm", "vl_trsm", "vl_trsm_noalloc",
              "vl_set_allocator", "vl_grad_offset", "vl_grad_beta", "vl_grad_aux", "vl_estimate", "vl_estimate_glm",
              "vl_timing_enable",
              "vl_timing_read", "vl_batch_create", "vl_batch_fit", "vl_batch_mode",
              "vl_batch_stats", "vl_server_create", "vl_server_submit", "vl_server_wait",
              "vl_server_info"):
        getattr(L, f).restype = I
    _lib = L
    return L


def _check(code, allow=()):
    if code != VL_OK and code not in allow:
        raise VLError(code, lib().vl_last_error().decode() or
                      lib().vl_status_string(code).decode())
    return code


def _ptr(t, dtype=torch.float64, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def vl_default_opts(**kw):
    o = vl_opts()
    lib().vl_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def vl_build_vecchia(coords, m, cov, theta, want_deriv=False, stream=None):
    """Handle of the Vecchia approximation at locations `coords` (n x 2)."""
    n = coords.shape[0]
    _ptr(coords, shape=(n, 2))
    th = (ctypes.c_double * 2)(*[float(x) for x in theta])
    s = stream if stream is not None else torch.cuda.current_stream(coords.device).cuda_stream
    h = ctypes.c_void_p()
    _check(lib().vl_build_vecchia(ctypes.c_void_p(coords.data_ptr()), n, int(m), int(cov), th,
                                  ctypes.c_void_p(s), 1 if want_deriv else 0, ctypes.byref(h)))
    return h


def vl_set_theta(h, theta):
    th = (ctypes.c_double * 2)(*[float(x) for x in theta])
    _check(lib().vl_set_theta(h, th))


def vl_find_mode(h, y, F, lik, aux=None, opts=None, mode_out=None, allow_no_conv=False):
    opts = opts or vl_default_opts()
    st = vl_stats()
    a = (ctypes.c_double * 1)(float(aux)) if aux is not None else None
    code = lib().vl_find_mode(h, _ptr(y), _ptr(F), int(lik), a, ctypes.byref(opts),
                              _ptr(mode_out), ctypes.byref(st))
    _check(code, allow=(VL_ERR_NO_CONVERGENCE,) if allow_no_conv else ())
    return st, code


def vl_neg_log_marglik(h, opts=None, want_grad=False, allow_no_conv=False):
    opts = opts or vl_default_opts()
    nll = ctypes.c_double()
    grad = (ctypes.c_double * 2)()
    st = vl_stats()
    code = lib().vl_neg_log_marglik(h, ctypes.byref(opts), ctypes.byref(nll),
                                    grad if want_grad else None, ctypes.byref(st))
    _check(code, allow=(VL_ERR_NO_CONVERGENCE,) if allow_no_conv else ())
    return nll.value, (list(grad) if want_grad else None), st


def vl_predict(h, coords_p, Fp, opts, mean_out, var_out=None, allow_no_conv=False):
    npred = coords_p.shape[0]
    st = vl_stats()
    code = lib().vl_predict(h, _ptr(coords_p, shape=(npred, 2)), npred, _ptr(Fp),
                            ctypes.byref(opts), _ptr(mean_out), _ptr(var_out), ctypes.byref(st))
    _check(code, allow=(VL_ERR_NO_CONVERGENCE,) if allow_no_conv else ())
    return st


def vl_export(h, name, device="cuda"):
    which, dtype = EXPORT[name]
    cnt = lib().vl_export_count(h, which)
    if cnt < 0:
        raise VLError(VL_ERR_STATE, f"{name} not available")
    out = torch.empty(max(int(cnt), 0), dtype=dtype, device=device)
    _check(lib().vl_export(h, which, ctypes.c_void_p(out.data_ptr()) if cnt else None,
                           out.numel() * out.element_size()))
    return out


_allocator_keep = None  # the installed callbacks must outlive their use


def vl_set_allocator(alloc=None, release=None):
    """Install Python callables alloc(bytes, stream) -> int device pointer
    and release(ptr, stream) as the library's device allocator (both None:
    the library's default, hipMallocAsync)."""
    global _allocator_keep
    if alloc is None and release is None:
        _check(lib().vl_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator_keep = None
        return

    def _a(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0)))
        except Exception:  # out of memory or a failing hook: the call fails with VL_ERR_OOM
            return None

    def _f(ptr, stream, ctx):
        release(int(ptr), int(stream or 0))

    keep = (ALLOC_FN(_a), FREE_FN(_f))
    _check(lib().vl_set_allocator(keep[0], keep[1], None))
    _allocator_keep = keep


def use_torch_allocator(enable=True):
    """Back every device buffer of the library with PyTorch's caching
    allocator (on the stream of the library call), or restore the default."""
    if not enable:
        vl_set_allocator(None, None)
        return
    vl_set_allocator(
        lambda nbytes, stream: torch.cuda.caching_allocator_alloc(nbytes, stream=stream),
        lambda ptr, stream: torch.cuda.caching_allocator_delete(ptr))


def vl_trsm_noalloc(h, X, Y, transpose=False):
    """vl_trsm for at most 64 columns with no device allocation (fixed
    per-GPU scratch)."""
    t = 1 if X.dim() == 1 else X.shape[1]
    _ptr(X), _ptr(Y)
    _check(lib().vl_trsm_noalloc(h, 1 if transpose else 0, ctypes.c_void_p(X.data_ptr()),
                                 ctypes.c_void_p(Y.data_ptr()), t))


def vl_spmm(h, X, Y, transpose=False):
    t = 1 if X.dim() == 1 else X.shape[1]
    _ptr(X), _ptr(Y)
    _check(lib().vl_spmm(h, 1 if transpose else 0, ctypes.c_void_p(X.data_ptr()),
                         ctypes.c_void_p(Y.data_ptr()), t))


def vl_trsm(h, X, Y, transpose=False):
    t = 1 if X.dim() == 1 else X.shape[1]
    _ptr(X), _ptr(Y)
    _check(lib().vl_trsm(h, 1 if transpose else 0, ctypes.c_void_p(X.data_ptr()),
                         ctypes.c_void_p(Y.data_ptr()), t))


TIMED_KINDS = {"spmm_b": 0, "spmm_bt": 1, "trsm_lower": 2, "trsm_upper": 3,
               "dense_lower": 4, "dense_upper": 5, "level_lower": 6, "level_upper": 7,
               "level_upper_split": 8, "level_upper_fold": 9,
               "dense_wide": 10}


def vl_timing_enable(h, enable=True, kinds=None):
    """Record kernel classes `kinds` (names of TIMED_KINDS; None = all)."""
    mask = 0
    if enable:
        mask = -1 if kinds is None else sum(1 << TIMED_KINDS[k] for k in kinds)
    _check(lib().vl_timing_enable(h, mask))


def vl_timing_read(h, kind):
    """(total kernel ms, launches, algorithmic bytes) of one kernel class."""
    ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().vl_timing_read(h, TIMED_KINDS[kind], ctypes.byref(ms), ctypes.byref(n),
                                ctypes.byref(by)))
    return ms.value, n.value, by.value


def vl_free(h):
    if h:
        lib().vl_free(h)


class VecchiaLaplace:
    """Convenience wrapper owning one model handle."""

    def __init__(self, coords, m, cov, theta, want_deriv=False):
        self.coords = coords
        self.n = coords.shape[0]
        self.m = m
        self.h = vl_build_vecchia(coords, m, cov, theta, want_deriv)

    def set_theta(self, theta):
        vl_set_theta(self.h, theta)

    def find_mode(self, y, F=None, lik=VL_LIK_BERNOULLI_LOGIT, aux=None, opts=None,
                  allow_no_conv=False):
        mode = torch.empty(self.n, dtype=torch.float64, device=y.device)
        st, code = vl_find_mode(self.h, y, F, lik, aux, opts, mode, allow_no_conv)
        return mode, st

    def neg_log_marglik(self, opts=None, want_grad=False, allow_no_conv=False):
        nll, grad, st = vl_neg_log_marglik(self.h, opts, want_grad, allow_no_conv)
        return nll, grad, st

    def predict(self, coords_p, Fp=None, opts=None, want_var=True, allow_no_conv=False):
        opts = opts or vl_default_opts()
        npred = coords_p.shape[0]
        mean = torch.empty(npred, dtype=torch.float64, device=coords_p.device)
        var = torch.empty(npred, dtype=torch.float64, device=coords_p.device) if want_var else None
        st = vl_predict(self.h, coords_p, Fp, opts, mean, var, allow_no_conv)
        return mean, var, st

    def estimate(self, y, F, lik, theta0, aux=None, opts=None, max_iter=50, grad_tol=1e-6,
                 allow_no_conv=False):
        """L-BFGS estimate of theta (vl_estimate); returns (theta, nll, iters, evals)."""
        opts = opts or vl_default_opts()
        th = (ctypes.c_double * 2)(*[float(v) for v in theta0])
        nll, it, ev = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        a = (ctypes.c_double * 1)(float(aux)) if aux is not None else None
        code = lib().vl_estimate(self.h, _ptr(y), _ptr(F), int(lik), a, ctypes.byref(opts), th,
                                 int(max_iter), float(grad_tol), ctypes.byref(nll),
                                 ctypes.byref(it), ctypes.byref(ev))
        _check(code, allow=(VL_ERR_NO_CONVERGENCE,) if allow_no_conv else ())
        return (th[0], th[1]), nll.value, it.value, ev.value

    def estimate_glm(self, y, X, lik, params0, opts=None, max_iter=100, grad_tol=1e-6,
                     allow_no_conv=False):
        """Joint L-BFGS estimate (vl_estimate_glm) of {sigma2, rho, [xi], beta}
        with F = X beta (X: device n x p float64, or None for p = 0); returns
        (params, nll, iters, evals)."""
        opts = opts or vl_default_opts()
        p = 0 if X is None else (1 if X.dim() == 1 else X.shape[1])
        prm = (ctypes.c_double * len(params0))(*[float(v) for v in params0])
        nll, it, ev = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        code = lib().vl_estimate_glm(self.h, _ptr(y), _ptr(X) if X is not None else None, p,
                                     int(lik), ctypes.byref(opts), prm, int(max_iter),
                                     float(grad_tol), ctypes.byref(nll), ctypes.byref(it),
                                     ctypes.byref(ev))
        _check(code, allow=(VL_ERR_NO_CONVERGENCE,) if allow_no_conv else ())
        return list(prm), nll.value, it.value, ev.value

    def grad_offset(self):
        """dL/dF (device tensor, n) from the last neg_log_marglik with a gradient."""
        out = torch.empty(self.n, dtype=torch.float64, device=self.coords.device)
        _check(lib().vl_grad_offset(self.h, _ptr(out)))
        return out

    def grad_beta(self, X):
        """X^T dL/dF for F = X beta (X: device n x p float64)."""
        p = 1 if X.dim() == 1 else X.shape[1]
        out = (ctypes.c_double * p)()
        _check(lib().vl_grad_beta(self.h, _ptr(X), p, out))
        return list(out)

    def grad_aux(self):
        """dL/dxi (Gaussian tau^2 or Gamma shape) from the last neg_log_marglik
        with a gradient."""
        out = ctypes.c_double()
        _check(lib().vl_grad_aux(self.h, ctypes.byref(out)))
        return out.value

    def export(self, name):
        return vl_export(self.h, name, self.coords.device)

    def close(self):
        if self.h:
            vl_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VecchiaLaplaceBatch:
    """Many problems fitted together (vl_batch_*).  `problems`: list of dicts
    with coords (n x 2), y, F (or None), m, cov, theta, seed -- device tensors
    or arrays convertible to them."""

    def __init__(self, problems, lik=VL_LIK_BERNOULLI_LOGIT, aux=None, device="cuda"):
        self._keep = []
        arr = (vl_problem * len(problems))()
        for k, p in enumerate(problems):
            c = torch.as_tensor(p["coords"], dtype=torch.float64, device=device).contiguous()
            y = torch.as_tensor(p["y"], dtype=torch.float64, device=device).contiguous()
            F = p.get("F")
            F = None if F is None else torch.as_tensor(F, dtype=torch.float64,
                                                       device=device).contiguous()
            self._keep += [c, y, F]
            arr[k].coords = c.data_ptr()
            arr[k].n = c.shape[0]
            arr[k].m = int(p["m"])
            arr[k].cov = int(p["cov"])
            arr[k].theta[0], arr[k].theta[1] = float(p["theta"][0]), float(p["theta"][1])
            arr[k].y = y.data_ptr()
            arr[k].F = F.data_ptr() if F is not None else None
            arr[k].seed = int(p.get("seed", 0))
        self.sizes = [int(arr[k].n) for k in range(len(problems))]
        self.device = device
        h = ctypes.c_void_p()
        a = (ctypes.c_double * 1)(float(aux)) if aux is not None else None
        _check(lib().vl_batch_create(arr, len(problems), lik, a, None, ctypes.byref(h)))
        self.h = h
        self._keep = []

    def fit(self, opts=None):
        opts = opts or vl_default_opts()
        out = (ctypes.c_double * len(self.sizes))()
        _check(lib().vl_batch_fit(self.h, ctypes.byref(opts), out))
        return list(out)

    def mode(self, p):
        out = torch.empty(self.sizes[p], dtype=torch.float64, device=self.device)
        _check(lib().vl_batch_mode(self.h, p, ctypes.c_void_p(out.data_ptr())))
        return out

    def stats(self, p):
        st = vl_stats()
        _check(lib().vl_batch_stats(self.h, p, ctypes.byref(st)))
        return st

    def tuned_path(self, width_class):
        return lib().vl_batch_tuned_path(self.h, width_class)

    def close(self):
        if self.h:
            lib().vl_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (vl_server_*).  submit() takes a dict
    with coords, y, F, m, cov, theta, lik, seed and optionally coords_p, Fp;
    it returns a ticket; wait(ticket) returns (nll, mean, var, stats,
    queue_ms) with mean/var as device tensors."""

    def __init__(self, slots, hbm_budget_bytes, opts=None, device="cuda"):
        self.opts = opts or vl_default_opts()
        h = ctypes.c_void_p()
        _check(lib().vl_server_create(int(slots), float(hbm_budget_bytes),
                                      ctypes.byref(self.opts), ctypes.byref(h)))
        self.h = h
        self.device = device
        self._live = {}

    def _request(self, r):
        t = lambda x: (None if x is None else
                       torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous())
        keep = dict(coords=t(r["coords"]), y=t(r["y"]), F=t(r.get("F")),
                    coords_p=t(r.get("coords_p")), Fp=t(r.get("Fp")))
        n_p = 0 if keep["coords_p"] is None else keep["coords_p"].shape[0]
        keep["mean"] = torch.empty(n_p, dtype=torch.float64, device=self.device)
        keep["var"] = torch.empty(n_p, dtype=torch.float64, device=self.device)
        q = vl_request()
        ptr = lambda x: None if x is None else x.data_ptr()
        q.coords, q.n, q.m, q.cov = ptr(keep["coords"]), keep["coords"].shape[0], int(r["m"]), \
            int(r["cov"])
        q.theta[0], q.theta[1] = float(r["theta"][0]), float(r["theta"][1])
        q.y, q.F, q.lik, q.aux = ptr(keep["y"]), ptr(keep["F"]), int(r["lik"]), \
            float(r.get("aux", 0.0))
        q.seed = int(r.get("seed", 0))
        q.coords_p, q.n_p, q.Fp = ptr(keep["coords_p"]), n_p, ptr(keep["Fp"])
        q.mean_out = ptr(keep["mean"]) if n_p else None
        q.var_out = ptr(keep["var"]) if n_p else None
        return q, keep

    def request_bytes(self, r):
        q, _ = self._request(r)
        return lib().vl_request_bytes(ctypes.byref(q), ctypes.byref(self.opts))

    def submit(self, r):
        q, keep = self._request(r)
        torch.cuda.synchronize()
        tk = ctypes.c_int64()
        _check(lib().vl_server_submit(self.h, ctypes.byref(q), ctypes.byref(tk)))
        self._live[tk.value] = keep
        return tk.value

    def wait(self, ticket):
        nll, st, qms = ctypes.c_double(), vl_stats(), ctypes.c_double()
        code = lib().vl_server_wait(self.h, ticket, ctypes.byref(nll), ctypes.byref(st),
                                    ctypes.byref(qms))
        keep = self._live.pop(ticket)
        _check(code, allow=(VL_ERR_NO_CONVERGENCE,))
        return nll.value, keep["mean"], keep["var"], st.as_dict(), qms.value

    def info(self):
        b, r = ctypes.c_double(), ctypes.c_int()
        _check(lib().vl_server_info(self.h, ctypes.byref(b), ctypes.byref(r)))
        return b.value, r.value

    def close(self):
        if self.h:
            lib().vl_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of libnpga (see include/npga.h for the semantics).

Every function takes CUDA/HIP torch tensors already resident on the device
and enqueues on ``torch.cuda.current_stream()``.  Matrices are passed as
C-contiguous (cols, n) float32 tensors: row t is column t of the n x cols
matrix, i.e. the column-major layout with leading dimension n.  When n is
not a multiple of 4 the binding copies into a padded buffer (ld = 4
ceil(n/4)) because the kernels load float4.
"""
import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libnpga.so")

NPGA_OK = 0
STATUS_NAMES = {
    0: "OK", 1: "INVALID", 2: "INFEASIBLE", 3: "NOT_CONVERGED", 4: "BRACKET",
    5: "NUMERIC", 6: "WORKSPACE", 7: "HIP", 8: "UNSUPPORTED",
}
PATHS = {"auto": 0, "gemv": 1, "syrk": 2}


class NpgaError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({status_string(code)})")


class _Factor(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cols", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("L", ctypes.c_void_p), ("mu", ctypes.c_void_p), ("gamma", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("proj_tol", ctypes.c_double),
                ("power_iters", ctypes.c_int32), ("step_safety", ctypes.c_double),
                ("refine", ctypes.c_int32), ("path", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("warm_start", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("refine_max_iter", ctypes.c_int32),
                ("momentum", ctypes.c_int32), ("step_estimator", ctypes.c_int32),
                ("batch_config", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("projection", ctypes.c_int32), ("dykstra_iters", ctypes.c_int32),
                ("backtrack_rho", ctypes.c_double), ("refine_method", ctypes.c_int32),
                ("refine_plain_cg", ctypes.c_int32)]


class _StrOptions(ctypes.Structure):
    _fields_ = [("sketch", ctypes.c_int32), ("ell_rule", ctypes.c_int32), ("k", ctypes.c_int64),
                ("ell", ctypes.c_int64), ("ridge_coef", ctypes.c_double), ("kappa_tar", ctypes.c_double),
                ("knee_tau", ctypes.c_double), ("knee_rho", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("S", ctypes.c_void_p), ("lds", ctypes.c_int64), ("cs_bucket", ctypes.c_void_p),
                ("cs_sign", ctypes.c_void_p)]


class _BackwardResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("support", ctypes.c_int32),
                ("return_active", ctypes.c_int32), ("degenerate", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nu", ctypes.c_double), ("lambda_", ctypes.c_double), ("dl_dr", ctypes.c_double),
                ("dl_dgamma", ctypes.c_double), ("residual", ctypes.c_double), ("time_ms", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("support", ctypes.c_int32),
                ("return_active", ctypes.c_int32), ("refined", ctypes.c_int32),
                ("path_used", ctypes.c_int32), ("step_sweeps", ctypes.c_int32),
                ("residual", ctypes.c_double), ("final_residual", ctypes.c_double),
                ("objective", ctypes.c_double), ("nu", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("alpha", ctypes.c_double),
                ("lipschitz", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("time_to_tol_ms", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("sweep_samples", ctypes.c_int32),
                ("dykstra_used", ctypes.c_int32), ("backtracks", ctypes.c_int32),
                ("refine_fallback", ctypes.c_int32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build it with `python paper_2604_02917_amd/build.py` "
            "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    u64 = ctypes.c_uint64
    sig = {
        "npga_default_options": (None, [ctypes.POINTER(_Options)]),
        "npga_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "npga_struct_size": (sz, [i32]),
        "npga_solve_workspace_size": (sz, [i64, i64, ctypes.POINTER(_Options)]),
        "npga_auto_path": (ctypes.c_int, [i64, i64, i32]),
        "npga_solve": (ctypes.c_int, [ctypes.POINTER(_Factor), dbl, ctypes.POINTER(_Options), vp,
                                      ctypes.POINTER(_Result), vp, sz, vp]),
        "npga_project": (ctypes.c_int, [vp, vp, i64, dbl, vp, vp, vp, sz, vp]),
        "npga_project_dykstra": (ctypes.c_int, [vp, vp, i64, dbl, i32, dbl, vp, vp, vp, vp, sz, vp]),
        "npga_gradient": (ctypes.c_int, [ctypes.POINTER(_Factor), vp, vp, vp, vp, sz, vp]),
        "npga_spectral_norm_sq": (ctypes.c_int, [ctypes.POINTER(_Factor), i32, u64, i32, vp, vp, vp, sz, vp]),
        "npga_syrk": (ctypes.c_int, [vp, i64, i64, i64, vp, i64, vp]),
        "npga_syrk_split_workspace_size": (sz, [i64, i64]),
        "npga_syrk_split": (ctypes.c_int, [vp, i64, i64, i64, vp, i64, vp, sz, vp]),
        "npga_to_bf16": (ctypes.c_int, [vp, i64, i64, i64, vp, i64, vp]),
        "npga_build_factor_workspace_size": (sz, [i64, i64]),
        "npga_build_factor": (ctypes.c_int, [vp, i64, i64, i64, vp, i64, vp, vp, sz, vp]),
        "npga_sketch_workspace_size": (sz, [i64, i64, i64, i64]),
        "npga_sketch_str": (ctypes.c_int, [vp, i64, i64, i64, i64, i64, dbl, u64, vp, i64, vp, i64, vp,
                                           vp, vp, sz, vp]),
        "npga_batched_workspace_size": (sz, [i64, i64, i32, ctypes.POINTER(_Options)]),
        "npga_solve_batched": (ctypes.c_int, [ctypes.POINTER(_Factor), vp, i32, ctypes.POINTER(_Options),
                                              vp, i64, ctypes.POINTER(_Result), vp, sz, vp]),
        "npga_gradient_batched": (ctypes.c_int, [ctypes.POINTER(_Factor), vp, i64, i32, vp, i64, vp, i32,
                                                 vp, sz, vp]),
        "npga_batched_tune": (ctypes.c_int, [ctypes.POINTER(_Factor), i32, i32, vp, vp, vp, sz, vp]),
        "npga_default_str_options": (None, [ctypes.POINTER(_StrOptions)]),
        "npga_sketch_ex_workspace_size": (sz, [i64, i64, ctypes.POINTER(_StrOptions)]),
        "npga_sketch_str_ex": (ctypes.c_int, [vp, i64, i64, i64, ctypes.POINTER(_StrOptions), vp, i64, vp,
                                              ctypes.POINTER(i64), ctypes.POINTER(dbl), vp, sz, vp]),
        "npga_philox_sketch": (ctypes.c_int, [u64, i64, i64, vp, i64, vp, vp]),
        "npga_gradient_noalloc_max_bytes": (sz, []),
        "npga_gradient_noalloc": (ctypes.c_int, [ctypes.POINTER(_Factor), vp, vp, vp, vp]),
        "npga_backward_workspace_size": (sz, [i64, i64]),
        "npga_backward": (ctypes.c_int, [ctypes.POINTER(_Factor), dbl, vp, vp, vp, vp, i64,
                                         ctypes.POINTER(_BackwardResult), vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib_path():
    return _LIB_PATH


def status_string(code):
    return _lib.npga_status_string(int(code)).decode()


@dataclasses.dataclass
class Options:
    tol: float = 1e-6
    check_every: int = 5
    max_iter: int = 200000
    proj_tol: float = 1e-12
    power_iters: int = 20
    step_safety: float = 1.05
    refine: bool = True
    path: str = "auto"
    seed: int = 1
    warm_start: bool = False
    restart: bool = False
    refine_tol: float = 1e-9
    refine_max_iter: int = 20000
    batch_config: int = -1
    momentum: str = "fista"   # "fista" (Algorithm 1) or "constant" (strongly convex, gamma > 0)
    step_estimator: str = "lanczos"   # or "power" (the paper's Remark)
    alpha: float = 0.0   # > 0: the caller's fixed step (no estimate)
    projection: str = "exact"   # or "dykstra" (alternating projections only)
    dykstra_iters: int = 5000
    backtrack_rho: float = 0.0   # in (0, 1): adaptive backtracking from the trial step
    refine_method: str = "auto"   # "auto", "pdas" (primal-dual active set) or "cg" (blocking face CG)
    refine_precond: bool = True   # Nystrom-preconditioned face CG of the active-set method (n >= 2048)

    def _c(self):
        o = _Options()
        _lib.npga_default_options(ctypes.byref(o))
        o.tol, o.check_every, o.max_iter = self.tol, self.check_every, self.max_iter
        o.proj_tol, o.power_iters, o.step_safety = self.proj_tol, self.power_iters, self.step_safety
        o.refine, o.path, o.seed = int(self.refine), PATHS[self.path], self.seed
        o.warm_start, o.restart = int(self.warm_start), int(self.restart)
        o.refine_tol, o.refine_max_iter = self.refine_tol, self.refine_max_iter
        o.batch_config = self.batch_config
        o.momentum = {"fista": 0, "constant": 1}[self.momentum]
        o.step_estimator = {"lanczos": 0, "power": 1}[self.step_estimator]
        o.alpha = self.alpha
        o.projection = {"exact": 0, "dykstra": 1}[self.projection]
        o.dykstra_iters = self.dykstra_iters
        o.backtrack_rho = self.backtrack_rho
        o.refine_method = {"auto": 0, "pdas": 1, "cg": 2}[self.refine_method]
        o.refine_plain_cg = 0 if self.refine_precond else 1
        return o


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(code, where):
    if code != NPGA_OK:
        raise NpgaError(code, where)


def _as_colmajor(M):
    """(cols, n) float32 or bfloat16 CUDA tensor -> (tensor with row stride ld, n, cols, ld)."""
    if M.dim() != 2 or M.dtype not in (torch.float32, torch.bfloat16) or not M.is_cuda:
        raise ValueError("expected a 2-D float32 or bfloat16 CUDA tensor of shape (cols, n)")
    cols, n = M.shape
    # float32: float4 loads; bfloat16: 8 entries (16 bytes) per load
    q = 4 if M.dtype == torch.float32 else 8
    ld = (n + q - 1) // q * q
    align = 16
    if M.is_contiguous() and ld == n and M.data_ptr() % align == 0:
        return M, n, cols, ld
    buf = torch.zeros((cols, ld), dtype=M.dtype, device=M.device)
    buf[:, :n].copy_(M)
    return buf, n, cols, ld


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _factor(Lb, n, cols, ld, mu, gamma):
    dtype = 1 if Lb.dtype == torch.bfloat16 else 0
    return _Factor(n, cols, ld, Lb.data_ptr(), mu.data_ptr(), float(gamma), dtype, 0)


def build_factor(R_TxN):
    """mu = R 1/T, L = (R - mu 1^T)/sqrt(T-1) on the GPU (Sec. 2.1).

    R_TxN: (T, n) float32 CUDA tensor.  Returns (L (T, n) float32, mu (n,) float64).
    """
    Rb, n, T, ld = _as_colmajor(R_TxN)
    L = torch.empty((T, ld), dtype=torch.float32, device=Rb.device)
    mu = torch.empty(n, dtype=torch.float64, device=Rb.device)
    ws = _workspace(_lib.npga_build_factor_workspace_size(n, T), Rb.device)
    _check(_lib.npga_build_factor(_ptr(Rb), n, T, ld, _ptr(L), ld, _ptr(mu), _ptr(ws), ws.numel(),
                                  _stream()), "npga_build_factor")
    return (L if ld == n else L[:, :n]), mu


def auto_path(n, cols, dtype="f32"):
    """The path npga_solve's AUTO runs for this shape: "gemv" or "syrk"."""
    code = _lib.npga_auto_path(int(n), int(cols), {"f32": 0, "bf16": 1}[dtype])
    if code < 0:
        raise ValueError("invalid shape or dtype")
    return {1: "gemv", 2: "syrk"}[code]


def solve(L_TxN, mu, r, gamma=0.0, x0=None, options=None, **kw):
    """NPGA solve (Algorithm 1).  Returns (x (n,) float32 tensor, info dict)."""
    opts = options or Options(**kw)
    if x0 is not None:
        opts = dataclasses.replace(opts, warm_start=True)
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    mu = mu.to(dtype=torch.float64).contiguous()
    co = opts._c()
    ws = _workspace(_lib.npga_solve_workspace_size(n, cols, ctypes.byref(co)), Lb.device)
    x = torch.empty(n, dtype=torch.float32, device=Lb.device)
    if x0 is not None:
        x.copy_(x0.to(torch.float32))
    res = _Result()
    f = _factor(Lb, n, cols, ld, mu, gamma)
    code = _lib.npga_solve(ctypes.byref(f), float(r), ctypes.byref(co), _ptr(x), ctypes.byref(res),
                           _ptr(ws), ws.numel(), _stream())
    info = {k: getattr(res, k) for k, _ in _Result._fields_}
    info["lambda"] = info.pop("lambda_")
    info["status_name"] = STATUS_NAMES.get(code, str(code))
    if code not in (NPGA_OK, 3):
        raise NpgaError(code, "npga_solve")
    return x, info


def _info(res, code):
    info = {k: getattr(res, k) for k, _ in _Result._fields_}
    info["lambda"] = info.pop("lambda_")
    info["status_name"] = STATUS_NAMES.get(code, str(code))
    return info


BATCH_CONFIGS = 12


def solve_batched(L_TxN, mu, r_targets, gamma=0.0, X0=None, options=None, **kw):
    """m solves on one factor, target r_j per solve (an efficient frontier).

    r_targets: sequence of m floats.  X0: optional (m, n) warm starts.
    Returns (X (m, n) float32 tensor, row j = x_j; list of m info dicts).
    """
    opts = options or Options(**kw)
    if X0 is not None:
        opts = dataclasses.replace(opts, warm_start=True)
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    mu = mu.to(dtype=torch.float64).contiguous()
    r = [float(v) for v in r_targets]
    m = len(r)
    co = opts._c()
    ws = _workspace(_lib.npga_batched_workspace_size(n, cols, m, ctypes.byref(co)), Lb.device)
    X = torch.empty((m, n), dtype=torch.float32, device=Lb.device)
    if X0 is not None:
        X.copy_(X0.to(torch.float32))
    res = (_Result * m)()
    rt = (ctypes.c_double * m)(*r)
    f = _factor(Lb, n, cols, ld, mu, gamma)
    code = _lib.npga_solve_batched(ctypes.byref(f), rt, m, ctypes.byref(co), _ptr(X), n, res, _ptr(ws),
                                   ws.numel(), _stream())
    infos = [_info(res[j], res[j].status) for j in range(m)]
    if code not in (NPGA_OK, 3):
        raise NpgaError(code, "npga_solve_batched")
    return X, infos


def gradient_batched(L_TxN, X, gamma=0.0, config=-1):
    """G[j] = 2 L (L^T x_j) + 2 gamma x_j and f_j for the rows x_j of X (m, n),
    by the batched matrix-core GEMMs.  Returns (G (m, n) float64, f list)."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    X = X.to(torch.float32).contiguous()
    m = X.shape[0]
    mu = torch.zeros(n, dtype=torch.float64, device=Lb.device)
    G = torch.empty((m, n), dtype=torch.float64, device=Lb.device)
    ws = _workspace(_lib.npga_batched_workspace_size(n, cols, m, None), Lb.device)
    fo = (ctypes.c_double * m)()
    f = _factor(Lb, n, cols, ld, mu, gamma)
    _check(_lib.npga_gradient_batched(ctypes.byref(f), _ptr(X), n, m, _ptr(G), n, fo, int(config), _ptr(ws),
                                      ws.numel(), _stream()), "npga_gradient_batched")
    return G, list(fo)


def batched_tune(L_TxN, m, reps=5):
    """Times every batched tile configuration on this factor and batch size;
    returns (best config id, list of ms per U+G GEMM pair)."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    mu = torch.zeros(n, dtype=torch.float64, device=Lb.device)
    ws = _workspace(_lib.npga_batched_workspace_size(n, cols, m, None), Lb.device)
    best = ctypes.c_int32(-1)
    ms = (ctypes.c_float * BATCH_CONFIGS)()
    f = _factor(Lb, n, cols, ld, mu, 0.0)
    _check(_lib.npga_batched_tune(ctypes.byref(f), int(m), int(reps), ctypes.byref(best), ms, _ptr(ws),
                                  ws.numel(), _stream()), "npga_batched_tune")
    return best.value, list(ms)


def sketch_str_ex(L_TxN, k, ell, sketch="gaussian", S_kxT=None, seed=3, h=None, sgn=None, ell_rule="fixed",
                  tau=1e-3, rho=0.9, ridge_coef=1e-4, kappa_tar=0.0):
    """STR build with the App. D options.  sketch: "gaussian" (S_kxT given,
    or drawn on the device from Philox with `seed`) or "count" (h: (T,)
    int32 buckets, sgn: (T,) float32 signs, CUDA tensors).  ell_rule:
    "fixed" or "knee" (ell is then the cap).  kappa_tar > 1 selects the
    kappa_tar ridge.  Returns (Leff (ell_used, n), sigma (ell_used,), gamma,
    ell_used)."""
    Lb, n, T, ld = _as_colmajor(L_TxN)
    if Lb.dtype != torch.float32:
        raise ValueError("sketch_str_ex expects a float32 factor")
    so = _StrOptions()
    _lib.npga_default_str_options(ctypes.byref(so))
    so.sketch = {"gaussian": 0, "count": 1}[sketch]
    so.ell_rule = {"fixed": 0, "knee": 1}[ell_rule]
    so.k, so.ell, so.ridge_coef, so.kappa_tar = int(k), int(ell), float(ridge_coef), float(kappa_tar)
    so.knee_tau, so.knee_rho, so.seed = float(tau), float(rho), int(seed)
    keep = []
    if S_kxT is not None:
        Sb = S_kxT.to(torch.float32).contiguous()
        keep.append(Sb)
        so.S, so.lds = Sb.data_ptr(), Sb.shape[1]
    if sketch == "count":
        hb = h.to(torch.int32).contiguous()
        sb = sgn.to(torch.float32).contiguous()
        keep += [hb, sb]
        so.cs_bucket, so.cs_sign = hb.data_ptr(), sb.data_ptr()
    ldle = ld
    Leff = torch.zeros((ell, ldle), dtype=torch.float32, device=Lb.device)
    sigma = torch.empty(ell, dtype=torch.float32, device=Lb.device)
    ws = _workspace(_lib.npga_sketch_ex_workspace_size(n, T, ctypes.byref(so)), Lb.device)
    g = ctypes.c_double(0.0)
    eo = ctypes.c_int64(0)
    _check(_lib.npga_sketch_str_ex(_ptr(Lb), n, T, ld, ctypes.byref(so), _ptr(Leff), ldle, _ptr(sigma),
                                   ctypes.byref(eo), ctypes.byref(g), _ptr(ws), ws.numel(), _stream()),
           "npga_sketch_str_ex")
    e = int(eo.value)
    return Leff[:e, :n], sigma[:e], g.value, e


def philox_sketch(T, k, seed, raw=False, device="cuda:0"):
    """The on-device Gaussian sketch: returns S as a (k, T) float32 tensor
    (column-major T x k) and, if raw, the (k, T, 2) uint32 output words."""
    S = torch.empty((k, T), dtype=torch.float32, device=device)
    R = torch.empty((k, T, 2), dtype=torch.int32, device=device) if raw else None
    _check(_lib.npga_philox_sketch(int(seed), int(T), int(k), _ptr(S), int(T), _ptr(R), _stream()),
           "npga_philox_sketch")
    return (S, R) if raw else S


def backward(L_TxN, mu, r, x_star, dl_dx, gamma=0.0, want_dL=True):
    """Adjoint of the solution map (implicit differentiation of the KKT
    system on the face of x*).  Returns (dl_dmu (n,) float64, dl_dL (T, n)
    float32 or None, info dict with dl_dr, dl_dgamma, nu, support, ...)."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    mu = mu.to(dtype=torch.float64).contiguous()
    xs = x_star.to(torch.float32).contiguous()
    gx = dl_dx.to(torch.float32).contiguous()
    dmu = torch.empty(n, dtype=torch.float64, device=Lb.device)
    dL = torch.empty((cols, n), dtype=torch.float32, device=Lb.device) if want_dL else None
    ws = _workspace(_lib.npga_backward_workspace_size(n, cols), Lb.device)
    res = _BackwardResult()
    f = _factor(Lb, n, cols, ld, mu, gamma)
    code = _lib.npga_backward(ctypes.byref(f), float(r), _ptr(xs), _ptr(gx), _ptr(dmu), _ptr(dL), n,
                              ctypes.byref(res), _ptr(ws), ws.numel(), _stream())
    info = {k: getattr(res, k) for k, _ in _BackwardResult._fields_}
    info["lambda"] = info.pop("lambda_")
    info["status_name"] = STATUS_NAMES.get(code, str(code))
    if code not in (NPGA_OK, 3):
        raise NpgaError(code, "npga_backward")
    return dmu, dL, info


class NPGAFunction(torch.autograd.Function):
    """x* = argmin_{x in F} ||L^T x||^2 + gamma ||x||^2 as a differentiable
    map of (mu, L): forward by npga_solve, backward by npga_backward.
    Usage: x = NPGAFunction.apply(mu, L_TxN, r[, gamma])."""

    @staticmethod
    def forward(ctx, mu, L_TxN, r, gamma=0.0):
        x, info = solve(L_TxN.detach(), mu.detach(), float(r), gamma=gamma)
        ctx.save_for_backward(mu, L_TxN, x)
        ctx.r, ctx.gamma = float(r), float(gamma)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        mu, L_TxN, x = ctx.saved_tensors
        dmu, dL, _ = backward(L_TxN.detach(), mu.detach(), ctx.r, x, gx, gamma=ctx.gamma,
                              want_dL=ctx.needs_input_grad[1])
        return dmu.to(mu.dtype), (dL.to(L_TxN.dtype) if dL is not None else None), None, None


def project(v, mu, r):
    """Pi_F(v) (Sec. 3.1).  v, mu: (n,) float64 CUDA.  Returns (x, nu, tau)."""
    v = v.to(torch.float64).contiguous()
    mu = mu.to(torch.float64).contiguous()
    n = v.numel()
    x = torch.empty_like(v)
    ws = _workspace(_lib.npga_solve_workspace_size(n, 1, None), v.device)
    nt = (ctypes.c_double * 2)()
    _check(_lib.npga_project(_ptr(v), _ptr(mu), n, float(r), _ptr(x), nt, _ptr(ws), ws.numel(),
                             _stream()), "npga_project")
    return x, nt[0], nt[1]


def project_dykstra(v, mu, r, max_iter=5000, tol=1e-14):
    """Pi_F(v) by Dykstra's alternating projections (the Sec. 3.1 fallback).
    Returns (x, nu, tau, sweeps, converged)."""
    v = v.to(torch.float64).contiguous()
    mu = mu.to(torch.float64).contiguous()
    n = v.numel()
    x = torch.empty_like(v)
    ws = _workspace(_lib.npga_solve_workspace_size(n, 1, None), v.device)
    nt = (ctypes.c_double * 2)()
    it = ctypes.c_int32(0)
    code = _lib.npga_project_dykstra(_ptr(v), _ptr(mu), n, float(r), int(max_iter), float(tol), _ptr(x), nt,
                                     ctypes.byref(it), _ptr(ws), ws.numel(), _stream())
    if code not in (NPGA_OK, 3):
        raise NpgaError(code, "npga_project_dykstra")
    return x, nt[0], nt[1], it.value, code == NPGA_OK


def gradient(L_TxN, x, gamma=0.0):
    """g = 2 L(L^T x) + 2 gamma x and f(x) (eq. npga-unified-grad) by the fused sweep."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    x = x.to(torch.float32).contiguous()
    mu = torch.zeros(n, dtype=torch.float64, device=Lb.device)
    g = torch.empty(n, dtype=torch.float64, device=Lb.device)
    ws = _workspace(_lib.npga_solve_workspace_size(n, cols, None), Lb.device)
    fv = ctypes.c_double(0.0)
    f = _factor(Lb, n, cols, ld, mu, gamma)
    _check(_lib.npga_gradient(ctypes.byref(f), _ptr(x), _ptr(g), ctypes.byref(fv), _ptr(ws),
                              ws.numel(), _stream()), "npga_gradient")
    return g, fv.value


def gradient_noalloc(L_TxN, x, gamma=0.0, want_f=True):
    """npga_gradient_noalloc: the same gradient as ``gradient`` with the
    library's own per-device scratch array (no workspace).  With want_f =
    False the call does not synchronise and f is None."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    x = x.to(torch.float32).contiguous()
    mu = torch.zeros(n, dtype=torch.float64, device=Lb.device)
    g = torch.empty(n, dtype=torch.float64, device=Lb.device)
    fv = ctypes.c_double(0.0)
    f = _factor(Lb, n, cols, ld, mu, gamma)
    _check(_lib.npga_gradient_noalloc(ctypes.byref(f), _ptr(x), _ptr(g), ctypes.byref(fv) if want_f else None,
                                      _stream()), "npga_gradient_noalloc")
    return g, (fv.value if want_f else None)


def spectral_norm_sq(L_TxN, iters=30, seed=1, method="power", return_steps=False):
    """||L||_2^2 estimate (Sec. 3.1 Remark): method "power" (iters steps) or
    "lanczos" (at most min(iters, 64) steps, stopped on convergence)."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    mu = torch.zeros(n, dtype=torch.float64, device=Lb.device)
    ws = _workspace(_lib.npga_solve_workspace_size(n, cols, None), Lb.device)
    out = ctypes.c_double(0.0)
    st = ctypes.c_int32(0)
    f = _factor(Lb, n, cols, ld, mu, 0.0)
    _check(_lib.npga_spectral_norm_sq(ctypes.byref(f), int(iters), int(seed), {"lanczos": 0, "power": 1}[method],
                                      ctypes.byref(out), ctypes.byref(st), _ptr(ws), ws.numel(), _stream()),
           "npga_spectral_norm_sq")
    return (out.value, st.value) if return_steps else out.value


def sketch_str(L_TxN, S_kxT, ell, ridge_coef=1e-4, seed=0):
    """Sketch-truncate-ridge (Sec. 2.5, App. D) on the GPU.

    L_TxN: (T, n) float32 factor; S_kxT: (k, T) float32 sketch (row j is
    column j of the T x k sketch).  Returns (L_eff as an (ell, n) float32
    tensor, i.e. the n x ell factor column-major, sigma (ell,) float32,
    gamma).
    """
    Lb, n, T, ld = _as_colmajor(L_TxN)
    if S_kxT.dim() != 2 or S_kxT.shape[1] != T or S_kxT.dtype != torch.float32:
        raise ValueError("S must be a (k, T) float32 CUDA tensor")
    S = S_kxT.contiguous()
    k = S.shape[0]
    ldle = (n + 3) // 4 * 4
    Leff = torch.empty((ell, ldle), dtype=torch.float32, device=Lb.device)
    sigma = torch.empty(ell, dtype=torch.float32, device=Lb.device)
    ws = _workspace(_lib.npga_sketch_workspace_size(n, T, k, ell), Lb.device)
    gam = ctypes.c_double(0.0)
    _check(_lib.npga_sketch_str(_ptr(Lb), n, T, ld, k, int(ell), float(ridge_coef), int(seed), _ptr(S), T,
                                _ptr(Leff), ldle, _ptr(sigma), ctypes.byref(gam), _ptr(ws), ws.numel(),
                                _stream()), "npga_sketch_str")
    return (Leff if ldle == n else Leff[:, :n]), sigma, gam.value


def to_bf16(L_TxN):
    """bfloat16 copy of a (T, n) float32 factor, rounded to nearest even by
    the library's conversion kernel.  Returns a (T, n) torch.bfloat16 tensor."""
    Lb, n, T, ld = _as_colmajor(L_TxN)
    if Lb.dtype != torch.float32:
        raise ValueError("to_bf16 expects a float32 factor")
    ldb = (n + 7) // 8 * 8
    out = torch.empty((T, ldb), dtype=torch.bfloat16, device=Lb.device)
    _check(_lib.npga_to_bf16(_ptr(Lb), n, T, ld, _ptr(out), ldb, _stream()), "npga_to_bf16")
    return out if ldb == n else out[:, :n]


def syrk(L_TxN, method="fp32"):
    """Sigma = L L^T (n x n float32, symmetric, both triangles).

    method "fp32": float32 matrix cores; "split": bfloat16 matrix cores on
    three-plane operands (npga_syrk_split)."""
    Lb, n, cols, ld = _as_colmajor(L_TxN)
    lds = ld
    S = torch.empty((n, lds), dtype=torch.float32, device=Lb.device)
    if method == "fp32":
        _check(_lib.npga_syrk(_ptr(Lb), n, cols, ld, _ptr(S), lds, _stream()), "npga_syrk")
    elif method == "split":
        ws = _workspace(_lib.npga_syrk_split_workspace_size(n, cols), Lb.device)
        _check(_lib.npga_syrk_split(_ptr(Lb), n, cols, ld, _ptr(S), lds, _ptr(ws), ws.numel(), _stream()),
               "npga_syrk_split")
    else:
        raise ValueError(method)
    return S[:, :n]

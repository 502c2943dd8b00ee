"""ctypes binding of libgp2s (the C ABI declared in include/gp2s.h).

Argument marshalling only: every step of the computation runs in the library's HIP
kernels. Torch supplies device memory (through the library's allocator callbacks,
which forward to torch's caching allocator) and the current stream. The functions
keep the C names: gp2s_assemble, gp2s_spmv, gp2s_solve, gp2s_lml, gp2s_lml_grad.
If the shared library is missing this module raises ImportError: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgp2s.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_06143_amd.build`")

# torch is loaded first: it brings its own HIP runtime, which has to be in the process
# before libgp2s's (loaded the other way round, the library's device queries have
# failed with "no ROCm-capable device" once torch initialised the GPU)
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

GP2S_OK, GP2S_E_INVALID, GP2S_E_HIP, GP2S_E_OOM, GP2S_E_CAPACITY = 0, 1, 2, 3, 4
GP2S_E_NOT_SPD, GP2S_E_NOCONV, GP2S_E_NONFINITE = 5, 6, 7
GP2S_FP64, GP2S_MIXED = 0, 1
PRECISIONS = {"fp64": GP2S_FP64, "mixed": GP2S_MIXED}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_bumps", ctypes.c_int32), ("radius", ctypes.c_double),
                ("bump_width", ctypes.c_double), ("noise_var", ctypes.c_double),
                ("centers", ctypes.POINTER(ctypes.c_double)), ("weights", ctypes.POINTER(ctypes.c_double)),
                ("kernel", ctypes.c_int32), ("radii", ctypes.POINTER(ctypes.c_double)),
                ("ls_weights", ctypes.POINTER(ctypes.c_double)), ("ff_groups", ctypes.POINTER(ctypes.c_int32))]


WENDLAND = {"c2": 0, "c6": 1}  # Wendland member: C^2, or the printed C^6 of Eq. wendland


class SolveOpts(ctypes.Structure):
    _fields_ = [("n_probes", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("max_ir", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("seed", ctypes.c_uint64), ("tol", ctypes.c_double),
                ("probe_tol", ctypes.c_double), ("precond", ctypes.c_int32)]


PRECOND = {"jacobi": 0, "block": 1, "block64": 2}  # preconditioner of the CG solves (include/gp2s.h)


NUM_TIMERS = 16
TIMER_NAMES = ["asm_prep", "asm_count", "asm_fill", "cg_matvec1", "cg_matvec_block", "cg_update1", "cg_pupdate1",
               "spmv", "spmm", "slq", "backward", "grad_reduce", "cg_update_block", "cg_pupdate_block"]


class Stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NUM_TIMERS), ("count", ctypes.c_int64 * NUM_TIMERS)]

    def as_dict(self):
        return {name: (self.ms[k], int(self.count[k])) for k, name in enumerate(TIMER_NAMES)}


class Report(ctypes.Structure):
    _fields_ = [("lml", ctypes.c_double), ("logdet", ctypes.c_double), ("yTa", ctypes.c_double),
                ("resid", ctypes.c_double), ("logdet_stderr", ctypes.c_double), ("iters", ctypes.c_int32),
                ("probe_iters", ctypes.c_int32), ("ir_steps", ctypes.c_int32), ("n_probes", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PredictReport(ctypes.Structure):
    _fields_ = [("nnz_cross", ctypes.c_int64), ("var_blocks", ctypes.c_int32), ("var_iters", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_SIGS = {
    "gp2s_abi_version": (_i32, []),
    "gp2s_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
    "gp2s_status_string": (ctypes.c_char_p, [_i32]),
    "gp2s_create": (_i32, [ctypes.POINTER(_vp), _vp, ALLOC_FN, FREE_FN, _vp]),
    "gp2s_destroy": (_i32, [_vp]),
    "gp2s_last_error": (ctypes.c_char_p, [_vp]),
    "gp2s_check_params": (_i32, [_vp, _i64, ctypes.POINTER(Params)]),
    "gp2s_set_timing": (_i32, [_vp, _i32]),
    "gp2s_set_timing_mask": (_i32, [_vp, ctypes.c_uint32]),
    "gp2s_set_progress": (_i32, [_vp, PROGRESS_FN, _vp]),
    "gp2s_get_stats": (_i32, [_vp, ctypes.POINTER(Stats)]),
    "gp2s_assemble": (_i32, [_vp, _i64, _vp, ctypes.POINTER(Params), _i32, ctypes.POINTER(_vp)]),
    "gp2s_matrix_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "gp2s_matrix_export": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "gp2s_matrix_import": (_i32, [_vp, _i64, _i64, _vp, _vp, _vp, _i32, ctypes.POINTER(_vp)]),
    "gp2s_matrix_free": (_i32, [_vp]),
    "gp2s_matrix_refill": (_i32, [_vp, _vp, ctypes.POINTER(Params)]),
    "gp2s_matrix_set_block_product": (_i32, [_vp, _i32, _i32]),
    "gp2s_matrix_get_block_product": (_i32, [_vp, _i32, ctypes.POINTER(_i32)]),
    "gp2s_spmv": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "gp2s_spmv_noalloc": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "gp2s_solve": (_i32, [_vp, _vp, _vp, _vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(Report)]),
    "gp2s_lml": (_i32, [_vp, _vp, _vp, ctypes.POINTER(SolveOpts), _vp, ctypes.POINTER(Report)]),
    "gp2s_lml_grad": (_i32, [_vp, _vp, _vp, ctypes.POINTER(SolveOpts), _vp, ctypes.POINTER(Report),
                             ctypes.POINTER(ctypes.c_double)]),
    "gp2s_predict": (_i32, [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(SolveOpts), _vp, _vp,
                            ctypes.POINTER(PredictReport)]),
    "gp2s_batch_plan": (_i32, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_vp), ctypes.POINTER(Params), _i32,
                               ctypes.POINTER(SolveOpts), ctypes.POINTER(_vp)]),
    "gp2s_batch_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                               ctypes.POINTER(_i32)]),
    "gp2s_batch_run": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), ctypes.POINTER(Report)]),
    "gp2s_batch_free": (_i32, [_vp]),
}
EXPORTED = tuple(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class GP2SError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib.gp2s_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib.gp2s_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solver option {k}")
        if k == "precond" and isinstance(v, str):
            v = PRECOND[v]
        setattr(o, k, v)
    return o


@dataclass
class HostParams:
    """Kernel hyperparameters (host values)."""
    dim: int
    radius: float
    bump_width: float
    noise_var: float
    centers: np.ndarray
    weights: np.ndarray
    kernel: int | str = 0  # 0 / "c2" or 1 / "c6"
    radii: np.ndarray | None = None       # per-axis radii (axis-anisotropic W), or None
    ls_weights: np.ndarray | None = None  # c_q of the length-scale field (Eq. wendconv), or None
    ff_groups: np.ndarray | None = None   # group of each bump for the far-field kernel (Eq. bump_kernel), or None

    def n_grad(self) -> int:
        """Length of the gradient: (r | r_1..r_d, a_1..a_P, [c_1..c_P], sigma^2)."""
        P = int(np.asarray(self.weights).reshape(-1).shape[0])
        return (self.dim if self.radii is not None else 1) + P + (P if self.ls_weights is not None else 0) + 1

    def to_c(self):
        dp = ctypes.POINTER(ctypes.c_double)
        c = np.ascontiguousarray(self.centers, dtype=np.float64).reshape(-1)
        w = np.ascontiguousarray(self.weights, dtype=np.float64).reshape(-1)
        r = None if self.radii is None else np.ascontiguousarray(self.radii, dtype=np.float64).reshape(-1)
        ls = None if self.ls_weights is None else np.ascontiguousarray(self.ls_weights, dtype=np.float64).reshape(-1)
        grp = None if self.ff_groups is None else np.ascontiguousarray(self.ff_groups, dtype=np.int32).reshape(-1)
        ip = ctypes.POINTER(ctypes.c_int32)
        kern = WENDLAND[self.kernel] if isinstance(self.kernel, str) else int(self.kernel)
        p = Params(int(self.dim), int(w.shape[0]), float(self.radius), float(self.bump_width),
                   float(self.noise_var), c.ctypes.data_as(dp), w.ctypes.data_as(dp), kern,
                   r.ctypes.data_as(dp) if r is not None else dp(), ls.ctypes.data_as(dp) if ls is not None else dp(),
                   grp.ctypes.data_as(ip) if grp is not None else ip())
        return p, (c, w, r, ls, grp)  # keep the arrays alive while p is used


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Context:
    """A library context bound to a HIP stream (default: torch's current stream) whose
    device allocations go through torch's caching allocator."""

    def __init__(self, stream=None, use_torch_allocator=True, alloc=None, free=None):
        """alloc(nbytes) -> device pointer or None, free(ptr): custom device allocator
        callbacks (both or neither); otherwise torch's caching allocator (or hipMalloc)."""
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if torch.cuda.is_available() else None
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        if alloc is not None and free is not None:
            self._alloc = ALLOC_FN(lambda nbytes, user: alloc(int(nbytes)))
            self._free = FREE_FN(lambda ptr, user: free(int(ptr)))
        elif use_torch_allocator and torch.cuda.is_available():
            dev = self.device.index
            tstream = stream

            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, tstream)
                except Exception:
                    return None

            def _free(ptr, user):
                try:
                    torch.cuda.caching_allocator_delete(int(ptr))
                except Exception:
                    pass

            self._alloc, self._free = ALLOC_FN(_alloc), FREE_FN(_free)
        else:
            self._alloc, self._free = ALLOC_FN(), FREE_FN()
        ctx = ctypes.c_void_p()
        st = lib.gp2s_create(ctypes.byref(ctx), handle, self._alloc, self._free, None)
        if st != GP2S_OK:
            raise GP2SError(st, "gp2s_create failed")
        self.ptr = ctx

    def check(self, st, allow_noconv=False):
        if st == GP2S_E_NOCONV and allow_noconv:
            return st
        if st != GP2S_OK:
            raise GP2SError(st, lib.gp2s_last_error(self.ptr).decode())
        return st

    def set_timing(self, enable=True, only=None):
        """Per-kernel event timing (resets the totals). `only`: a list of category names
        (TIMER_NAMES) to time, the others running without event records."""
        if only is None:
            self.check(lib.gp2s_set_timing(self.ptr, 1 if enable else 0))
        else:
            mask = 0
            for name in only:
                mask |= 1 << TIMER_NAMES.index(name)
            self.check(lib.gp2s_set_timing_mask(self.ptr, mask if enable else 0))

    def set_progress(self, fn=None):
        """fn(label: str, iters: int, open_cols: int, max_rel_resid: float) or None."""
        if fn is None:
            self._progress = PROGRESS_FN()
        else:
            self._progress = PROGRESS_FN(lambda lab, it, op, res, user: fn(lab.decode(), it, op, res))
        self.check(lib.gp2s_set_progress(self.ptr, self._progress, None))

    def stats(self) -> dict:
        st = Stats()
        self.check(lib.gp2s_get_stats(self.ptr, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "ptr", None):
            lib.gp2s_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = None


def default_context() -> Context:
    global _default_ctx
    import torch
    if _default_ctx is None or (torch.cuda.is_available() and
                                _default_ctx.stream != torch.cuda.current_stream()):
        _default_ctx = Context()
    return _default_ctx


class Matrix:
    """Handle to an assembled (or imported) covariance matrix."""

    def __init__(self, ctx: Context, handle, params: HostParams | None, precision: int):
        self.ctx, self.handle, self.params, self.precision = ctx, handle, params, precision
        n, nnz, pr = _i64(), _i64(), _i32()
        lib.gp2s_matrix_info(handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(pr))
        self.n, self.nnz = n.value, nnz.value

    def refill(self, params: "HostParams"):
        """New weights / noise / Wendland member on the same pattern (see gp2s_matrix_refill)."""
        p, keep = params.to_c()
        self.ctx.check(lib.gp2s_matrix_refill(self.ctx.ptr, self.handle, ctypes.byref(p)))
        self.params = params

    def set_block_product(self, nrhs: int, variant: int):
        """Pin the block-product kernel for `nrhs` columns (see include/gp2s.h); -1 retunes."""
        st = lib.gp2s_matrix_set_block_product(self.handle, int(nrhs), int(variant))
        if st != GP2S_OK:
            raise GP2SError(st, f"block-product variant {variant} does not apply to {nrhs} columns")

    def block_product(self, nrhs: int) -> int:
        """The block-product variant in use for `nrhs` columns (-1 before the first solve)."""
        v = _i32()
        st = lib.gp2s_matrix_get_block_product(self.handle, int(nrhs), ctypes.byref(v))
        if st != GP2S_OK:
            raise GP2SError(st, f"no block product for {nrhs} columns")
        return v.value

    def free(self):
        if self.handle:
            lib.gp2s_matrix_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def export(self):
        """(row_ptr, col, val, perm) as device tensors, internal order."""
        torch = self.ctx._torch
        dev = self.ctx.device
        rp = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        val = torch.empty(self.nnz, dtype=torch.float32 if self.precision == GP2S_MIXED else torch.float64,
                          device=dev)
        perm = torch.empty(self.n, dtype=torch.int32, device=dev) if self.params is not None else None
        self.ctx.check(lib.gp2s_matrix_export(self.ctx.ptr, self.handle, _ptr(rp), _ptr(col), _ptr(val),
                                              _ptr(perm)))
        return rp, col, val, perm


def _as_dev64(t, ctx):
    torch = ctx._torch
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    return t.to(device=ctx.device, dtype=torch.float64).contiguous()


def gp2s_assemble(x, params: HostParams, precision="mixed", ctx: Context | None = None) -> Matrix:
    ctx = ctx or default_context()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    xd = _as_dev64(x, ctx)
    p, keep = params.to_c()
    h = ctypes.c_void_p()
    ctx.check(lib.gp2s_assemble(ctx.ptr, int(xd.shape[0]), _ptr(xd), ctypes.byref(p), prec, ctypes.byref(h)))
    return Matrix(ctx, h, params, prec)


def gp2s_matrix_import(row_ptr, col, val, precision="fp64", ctx: Context | None = None) -> Matrix:
    ctx = ctx or default_context()
    torch = ctx._torch
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    rp = torch.as_tensor(row_ptr, dtype=torch.int64).to(ctx.device).contiguous()
    cl = torch.as_tensor(col, dtype=torch.int32).to(ctx.device).contiguous()
    vt = torch.float32 if prec == GP2S_MIXED else torch.float64
    vl = torch.as_tensor(val).to(device=ctx.device, dtype=vt).contiguous()
    h = ctypes.c_void_p()
    ctx.check(lib.gp2s_matrix_import(ctx.ptr, rp.numel() - 1, cl.numel(), _ptr(rp), _ptr(cl), _ptr(vl), prec,
                                     ctypes.byref(h)))
    return Matrix(ctx, h, None, prec)


def gp2s_spmv(m: Matrix, X):
    ctx = m.ctx
    Xd = _as_dev64(X, ctx)
    nrhs = 1 if Xd.dim() == 1 else int(Xd.shape[1])
    Y = ctx._torch.empty_like(Xd)
    ctx.check(lib.gp2s_spmv(ctx.ptr, m.handle, nrhs, _ptr(Xd), _ptr(Y)))
    return Y


def gp2s_spmv_noalloc(m: Matrix, X, Y):
    """Y = K X into the caller's Y (DEVICE float64, X's shape) through the allocation-free
    entry point: the library allocates nothing (see gp2s_spmv_noalloc in gp2s.h)."""
    ctx = m.ctx
    nrhs = 1 if X.dim() == 1 else int(X.shape[1])
    for t in (X, Y):
        if not (t.is_cuda and t.dtype == ctx._torch.float64 and t.is_contiguous()):
            raise ValueError("X and Y must be contiguous float64 device tensors")
    if tuple(Y.shape) != tuple(X.shape) or int(X.shape[0]) != m.n:
        raise ValueError("X and Y must both have n rows and the same shape")
    ctx.check(lib.gp2s_spmv_noalloc(ctx.ptr, m.handle, nrhs, _ptr(X), _ptr(Y)))
    return Y


def gp2s_solve(m: Matrix, y, opts: SolveOpts | None = None, allow_noconv=False):
    """a = K^-1 y. With allow_noconv, a CG that hits max_iter returns the last iterate
    (rep.status == GP2S_E_NOCONV) instead of raising."""
    ctx = m.ctx
    yd = _as_dev64(y, ctx)
    a = ctx._torch.empty_like(yd)
    rep = Report()
    o = opts or default_opts()
    st = lib.gp2s_solve(ctx.ptr, m.handle, _ptr(yd), _ptr(a), ctypes.byref(o), ctypes.byref(rep))
    rep.status = ctx.check(st, allow_noconv)
    return a, rep


def gp2s_predict(m: Matrix, x_test, a, opts: SolveOpts | None = None, want_var=True, allow_noconv=False):
    """Posterior mean (and variance) of the latent function at the rows of x_test, given
    a = K^-1 y from gp2s_solve / gp2s_lml. Returns (mean, var or None, report)."""
    ctx = m.ctx
    xd = _as_dev64(x_test, ctx)
    nt = int(xd.shape[0]) if xd.dim() > 1 else 0
    ad = _as_dev64(a, ctx)
    mean = ctx._torch.empty(nt, dtype=ctx._torch.float64, device=ad.device)
    var = ctx._torch.empty(nt, dtype=ctx._torch.float64, device=ad.device) if want_var else None
    rep = PredictReport()
    o = opts or default_opts()
    rep.status = ctx.check(lib.gp2s_predict(ctx.ptr, m.handle, nt, _ptr(xd), _ptr(ad), ctypes.byref(o), _ptr(mean),
                                            _ptr(var), ctypes.byref(rep)), allow_noconv)
    return mean, var, rep


def gp2s_lml(m: Matrix, y, opts: SolveOpts | None = None, want_a=True, allow_noconv=False):
    ctx = m.ctx
    yd = _as_dev64(y, ctx)
    a = ctx._torch.empty_like(yd) if want_a else None
    rep = Report()
    o = opts or default_opts()
    rep.status = ctx.check(lib.gp2s_lml(ctx.ptr, m.handle, _ptr(yd), ctypes.byref(o), _ptr(a),
                                        ctypes.byref(rep)), allow_noconv)
    return rep, a


def gp2s_lml_grad(m: Matrix, y, opts: SolveOpts | None = None, want_a=True, allow_noconv=False):
    ctx = m.ctx
    yd = _as_dev64(y, ctx)
    a = ctx._torch.empty_like(yd) if want_a else None
    rep = Report()
    o = opts or default_opts()
    ng = m.params.n_grad() if m.params is not None else 2
    grad = (ctypes.c_double * ng)()
    rep.status = ctx.check(lib.gp2s_lml_grad(ctx.ptr, m.handle, _ptr(yd), ctypes.byref(o), _ptr(a),
                                             ctypes.byref(rep), grad), allow_noconv)
    return rep, np.array(grad[:], dtype=np.float64), a


class Batch:
    """Many instances planned together (gp2s_batch_plan) and evaluated together
    (gp2s_batch_run). `xs` are (n_i, d_i) arrays or tensors, `params` HostParams."""

    def __init__(self, xs, params, precision="mixed", opts: SolveOpts | None = None, ctx: Context | None = None):
        self.ctx = ctx or default_context()
        self.prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.opts = opts or default_opts(n_probes=16)
        self.M = len(xs)
        self._xs = [_as_dev64(x, self.ctx) for x in xs]
        self.n = [int(x.shape[0]) for x in self._xs]
        self.params = list(params)
        self.P = [int(np.asarray(p.weights).reshape(-1).shape[0]) for p in self.params]
        n_arr = (_i64 * self.M)(*self.n)
        x_arr = (_vp * self.M)(*[_ptr(x) for x in self._xs])
        p_arr, self._keep = self._params_array(self.params)
        h = ctypes.c_void_p()
        self.ctx.check(lib.gp2s_batch_plan(self.ctx.ptr, self.M, n_arr, x_arr, p_arr, self.prec,
                                           ctypes.byref(self.opts), ctypes.byref(h)))
        self.handle = h

    def _params_array(self, params):
        arr = (Params * len(params))()
        keep = []
        for i, p in enumerate(params):
            c, k = p.to_c()
            arr[i] = c
            keep.append(k)
        return arr, keep

    def info(self):
        nt, nnz, cap = _i64(), _i64(), _i64()
        tuned = (_i32 * 3)()
        self.ctx.check(lib.gp2s_batch_info(self.handle, ctypes.byref(nt), ctypes.byref(nnz), ctypes.byref(cap),
                                           tuned))
        return dict(n_total=nt.value, nnz=nnz.value, capacity=cap.value, bin_refinement=tuned[0],
                    spmv_lanes=tuned[1], spmm_lanes=tuned[2])

    def run(self, ys, params=None, want_grad=True, allow_noconv=False):
        """Returns (lml [M], list of gradients or None, list of report dicts)."""
        yd = [_as_dev64(y, self.ctx) for y in ys]
        y_arr = (_vp * self.M)(*[_ptr(y) for y in yd])
        p_arr, keep = (self._params_array(params) if params is not None else (None, None))
        lml = (ctypes.c_double * self.M)()
        grads = [(ctypes.c_double * (p + 2))() for p in self.P] if want_grad else None
        g_arr = ((ctypes.POINTER(ctypes.c_double) * self.M)(*[ctypes.cast(g, ctypes.POINTER(ctypes.c_double))
                                                               for g in grads]) if want_grad else None)
        reps = (Report * self.M)()
        st = lib.gp2s_batch_run(self.handle, y_arr, p_arr, lml, g_arr, reps)
        self.ctx.check(st, allow_noconv)
        return (np.array(lml[:]), [np.array(g[:]) for g in grads] if want_grad else None,
                [r.as_dict() for r in reps])

    def free(self):
        if getattr(self, "handle", None):
            lib.gp2s_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

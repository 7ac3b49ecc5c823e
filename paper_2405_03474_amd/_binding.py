"""ctypes binding of liblogdet (include/logdet.h).

Argument marshalling only: torch supplies device memory and the stream, the
library does every step of the computation.  Importing this module loads the
shared library and raises if it has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblogdet.so")

LD_OK, LD_EINVAL, LD_ENOTSPD, LD_ENOCONV, LD_EHIP, LD_ENOMEM = 0, -1, -2, -3, -4, -5
LD_RBF, LD_MATERN52 = 0, 1
LD_F64, LD_F32, LD_BF16 = 0, 1, 2
LD_ROW_MAJOR, LD_TILED = 0, 1
LD_BATCH_GRAPH, LD_BATCH_RETUNE, LD_BATCH_PRECOND_ONLY, LD_BATCH_NO_SYMMETRIC = 1, 2, 4, 8
LD_SUR_FEATURES, LD_SUR_WIDTH, LD_SUR_BINS = 38, 256, 32
LD_LANCZOS_MAX = 128
(LD_PRECOND_RSVD, LD_PRECOND_IDENTITY, LD_PRECOND_DIAGONAL, LD_PRECOND_RANK_ONE,
 LD_PRECOND_PCHOL) = 0, 1, 2, 3, 4
LD_PRECOND_SCALED = 1
LD_PROBE_RADEMACHER, LD_PROBE_GAUSSIAN, LD_PROBE_ORTHOGONAL = 0, 1, 2
LD_SYM_F32, LD_SYM_BF16 = 1, 2

STATUS_NAMES = {0: "LD_OK", -1: "LD_EINVAL", -2: "LD_ENOTSPD", -3: "LD_ENOCONV", -4: "LD_EHIP",
                -5: "LD_ENOMEM"}

EXPORTED = (
    "ld_ctx_create", "ld_ctx_destroy", "ld_last_error", "ld_ctx_set_timing", "ld_ctx_read_timing",
    "ld_ctx_set_probes", "ld_ctx_set_graphs", "ld_ctx_set_symmetric", "ld_workspace_bytes", "ld_set_workspace",
    "ld_stored_elements", "ld_rational_coeffs", "ld_fill_probes",
    "ld_fill_gaussian", "kernel_matmat", "kernel_matmat_noalloc", "kernel_materialize",
    "logdet_precond_build",
    "logdet_precond_build_kind", "ld_precond_info", "ld_precond_export",
    "ld_precond_apply_inverse", "ld_precond_free",
    "logdet_estimate", "logdet_estimate_orders", "logdet_estimate_lanczos",
    "logdet_estimate_lanczos_orders", "logdet_gradient",
    "logdet_estimate_batched",
    "ld_surrogate_param_count",
    "ld_surrogate_features", "ld_surrogate_create", "ld_surrogate_free", "ld_surrogate_set_scaling",
    "ld_surrogate_train_step", "ld_surrogate_gradient", "ld_surrogate_params",
    "ld_surrogate_predict",
)


class LogdetError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Operator(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
        ("kind", ctypes.c_int32), ("lengthscale", ctypes.c_double), ("variance", ctypes.c_double),
        ("noise", ctypes.c_double), ("precision", ctypes.c_int32), ("M_stored", ctypes.c_void_p),
        ("layout", ctypes.c_int32),
    ]


class Instance(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
        ("kind", ctypes.c_int32), ("lengthscale", ctypes.c_double), ("variance", ctypes.c_double),
        ("noise", ctypes.c_double), ("rank", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("precond_seed", ctypes.c_uint64), ("probe_seed", ctypes.c_uint64),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("logdet", ctypes.c_double), ("logdet_P", ctypes.c_double), ("trace_term", ctypes.c_double),
        ("std_err", ctypes.c_double), ("rel_resid", ctypes.c_double),
        ("seconds_precond", ctypes.c_double), ("seconds_solve", ctypes.c_double),
        ("iterations", ctypes.c_int32),
        ("converged_cols", ctypes.c_int32), ("k", ctypes.c_int32), ("num_probes", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load():
    """Load liblogdet.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ld_ctx_create": (i32, [ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "ld_ctx_destroy": (None, [vp]),
        "ld_last_error": (ctypes.c_char_p, []),
        "ld_ctx_set_timing": (i32, [vp, i32]),
        "ld_ctx_read_timing": (i32, [vp, pd, ctypes.POINTER(i64), pd, pd]),
        "ld_ctx_set_probes": (i32, [vp, i32]),
        "ld_ctx_set_graphs": (i32, [vp, i32]),
        "ld_ctx_set_symmetric": (i32, [vp, i32]),
        "ld_stored_elements": (i64, [i64, i32]),
        "ld_rational_coeffs": (i32, [i32, pd, pd, pd]),
        "ld_fill_probes": (i32, [vp, u64, i64, i64, i32, vp]),
        "ld_fill_gaussian": (i32, [vp, u64, i32, i64, i64, vp]),
        "kernel_matmat": (i32, [vp, ctypes.POINTER(Operator), vp, i64, vp]),
        "kernel_matmat_noalloc": (i32, [vp, ctypes.POINTER(Operator), vp, i64, vp]),
        "kernel_materialize": (i32, [vp, ctypes.POINTER(Operator), vp]),
        "ld_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Operator), i64, i32, i32, i32]),
        "ld_set_workspace": (i32, [vp, vp, ctypes.c_size_t]),
        "logdet_precond_build": (i32, [vp, ctypes.POINTER(Operator), i32, i32, i32, u64,
                                       ctypes.POINTER(vp)]),
        "logdet_precond_build_kind": (i32, [vp, ctypes.POINTER(Operator), i32, i32, i32, i32, u64,
                                            i32, ctypes.POINTER(vp)]),
        "ld_precond_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), pd]),
        "ld_precond_export": (i32, [vp, vp, vp, vp, vp]),
        "ld_precond_apply_inverse": (i32, [vp, vp, vp, i64, i32, vp]),
        "ld_precond_free": (None, [vp]),
        "logdet_estimate": (i32, [vp, ctypes.POINTER(Operator), vp, i32, i32, u64, dbl, i32,
                                  ctypes.POINTER(Result), pd]),
        "logdet_estimate_orders": (i32, [vp, ctypes.POINTER(Operator), vp, i32,
                                         ctypes.POINTER(i32), i32, u64, dbl, i32,
                                         ctypes.POINTER(Result), pd]),
        "logdet_estimate_lanczos_orders": (i32, [vp, ctypes.POINTER(Operator), vp, i32,
                                                 ctypes.POINTER(i32), i32, u64, i32,
                                                 ctypes.POINTER(Result), pd]),
        "logdet_estimate_lanczos": (i32, [vp, ctypes.POINTER(Operator), vp, i32, i32, u64, i32,
                                          ctypes.POINTER(Result), pd]),
        "logdet_gradient": (i32, [vp, ctypes.POINTER(Operator), vp, i32, u64, dbl, i32, pd, pd, pd,
                                  ctypes.POINTER(Result)]),
        "logdet_estimate_batched": (i32, [vp, i32, ctypes.POINTER(Instance), i32, i32, i32, i32,
                                          dbl, i32, i32, ctypes.POINTER(Result), pd, pd, i32]),
        "ld_surrogate_param_count": (i64, []),
        "ld_surrogate_features": (i32, [pd, i32, i32, dbl, dbl, dbl, i64, i32, pd,
                                        ctypes.POINTER(ctypes.c_float)]),
        "ld_surrogate_create": (i32, [vp, i32, u64, ctypes.POINTER(vp)]),
        "ld_surrogate_free": (None, [vp]),
        "ld_surrogate_set_scaling": (i32, [vp, vp, ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(ctypes.c_float), dbl, dbl]),
        "ld_surrogate_train_step": (i32, [vp, vp, vp, vp, i32, ctypes.c_float, pd]),
        "ld_surrogate_gradient": (i32, [vp, vp, i32, vp, vp, i32, vp, pd]),
        "ld_surrogate_params": (i32, [vp, vp, i32, vp, vp]),
        "ld_surrogate_predict": (i32, [vp, vp, vp, i64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, allow=()):
    if status != LD_OK and status not in allow:
        raise LogdetError(status, load().ld_last_error().decode())
    return status


def rational_coeffs(k: int):
    """(b, a, c) of r_k from the library (host-only query)."""
    lib = load()
    b = ctypes.c_double()
    a = (ctypes.c_double * k)()
    c = (ctypes.c_double * k)()
    _check(lib.ld_rational_coeffs(k, ctypes.byref(b), a, c))
    return b.value, np.array(a[:]), np.array(c[:])


def _torch():
    import torch
    return torch


class Context:
    """A library context on one device, enqueueing on a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        self.torch_stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        _check(load().ld_ctx_create(device, ctypes.c_void_p(self.torch_stream.cuda_stream),
                                    ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().ld_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self.torch_stream.synchronize()

    def set_timing(self, on: bool = True):
        _check(load().ld_ctx_set_timing(self.handle, 1 if on else 0))

    def set_workspace(self, buf=None):
        """Use a caller-owned device tensor (or None: library scratch again) as
        the context's scratch; the tensor must outlive its use here."""
        if buf is None:
            _check(load().ld_set_workspace(self.handle, None, 0))
            self._workspace = None
            return
        assert buf.is_cuda and buf.is_contiguous()
        nbytes = buf.numel() * buf.element_size()
        _check(load().ld_set_workspace(self.handle, ctypes.c_void_p(buf.data_ptr()), nbytes))
        self._workspace = buf   # kept alive with the context

    def set_graphs(self, on: bool = True):
        """Replay the solver's iterations from captured HIP graphs."""
        _check(load().ld_ctx_set_graphs(self.handle, 1 if on else 0))

    def set_symmetric(self, f32: bool = True, bf16: bool = False):
        """Generate each off-diagonal kernel entry once in the on-the-fly
        products of 33..64 columns of these forms (default: FP32 only)."""
        forms = (LD_SYM_F32 if f32 else 0) | (LD_SYM_BF16 if bf16 else 0)
        _check(load().ld_ctx_set_symmetric(self.handle, forms))

    def set_probes(self, kind: int):
        """Probe distribution (LD_PROBE_*) of later single-problem estimates."""
        _check(load().ld_ctx_set_probes(self.handle, kind))

    def read_timing(self):
        """(total ms, launches, algorithmic flops, algorithmic bytes) of the
        solver's kernel-matrix product launches since set_timing."""
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        calls = ctypes.c_int64()
        _check(load().ld_ctx_read_timing(self.handle, ctypes.byref(ms), ctypes.byref(calls),
                                         ctypes.byref(fl), ctypes.byref(by)))
        return ms.value, calls.value, fl.value, by.value


def _dtype(precision: int):
    torch = _torch()
    return torch.float64 if precision == LD_F64 else torch.float32


@dataclass
class GPOperator:
    """M = K(X, X) + noise I (caller-owned device tensors)."""
    X: object                 # torch cuda float64 (n, d)
    kind: int
    lengthscale: float
    variance: float
    noise: float
    precision: int = LD_F64
    M: object = None          # optional stored matrix in the operator's dtype and layout
    layout: int = LD_ROW_MAJOR
    _keep: list = field(default_factory=list, repr=False)

    @property
    def n(self):
        return int(self.X.shape[0])

    @property
    def d(self):
        return int(self.X.shape[1])

    def c_struct(self) -> Operator:
        torch = _torch()
        assert self.X.is_cuda and self.X.dtype == torch.float64 and self.X.is_contiguous()
        if self.M is not None:
            assert self.M.is_cuda and self.M.dtype == _dtype(self.precision) and self.M.is_contiguous()
            assert self.M.numel() == stored_elements(self.n, self.layout)
        return Operator(X=self.X.data_ptr(), n=self.n, d=self.d, kind=self.kind,
                        lengthscale=self.lengthscale, variance=self.variance, noise=self.noise,
                        precision=self.precision,
                        M_stored=self.M.data_ptr() if self.M is not None else None,
                        layout=self.layout)


def workspace_bytes(op: GPOperator, s: int, rank: int, oversample: int = 10, k: int = 5) -> int:
    """Scratch bytes covering the single-problem calls on op (ld_workspace_bytes)."""
    cop = op.c_struct()
    v = load().ld_workspace_bytes(ctypes.byref(cop), s, rank, oversample, k)
    if v == 0:
        raise LogdetError(LD_EINVAL, load().ld_last_error().decode())
    return int(v)


def fill_probes(ctx: Context, seed: int, n: int, s: int, precision: int = LD_F64):
    torch = _torch()
    Z = torch.empty((n, s), dtype=_dtype(precision), device=f"cuda:{ctx.device}")
    _check(load().ld_fill_probes(ctx.handle, seed, n, s, precision, ctypes.c_void_p(Z.data_ptr())))
    return Z


def fill_gaussian(ctx: Context, seed: int, stream: int, rows: int, cols: int):
    torch = _torch()
    G = torch.empty((rows, cols), dtype=torch.float64, device=f"cuda:{ctx.device}")
    _check(load().ld_fill_gaussian(ctx.handle, seed, stream, rows, cols, ctypes.c_void_p(G.data_ptr())))
    return G


def kernel_matmat(ctx: Context, op: GPOperator, V):
    torch = _torch()
    assert V.is_cuda and V.dtype == _dtype(op.precision) and V.is_contiguous() and V.shape[0] == op.n
    V2 = V if V.dim() == 2 else V.reshape(op.n, 1)
    Y = torch.empty_like(V2)
    cop = op.c_struct()
    _check(load().kernel_matmat(ctx.handle, ctypes.byref(cop), ctypes.c_void_p(V2.data_ptr()),
                                V2.shape[1], ctypes.c_void_p(Y.data_ptr())))
    return Y.reshape(V.shape)


def kernel_matmat_noalloc(ctx: Context, op: GPOperator, V, Y=None):
    """kernel_matmat with the library's static device scratch (no allocation
    inside the library); Y may be passed in (n x s, V's dtype)."""
    torch = _torch()
    assert V.is_cuda and V.dtype == _dtype(op.precision) and V.is_contiguous() and V.shape[0] == op.n
    V2 = V if V.dim() == 2 else V.reshape(op.n, 1)
    if Y is None:
        Y = torch.empty_like(V2)
    assert Y.shape == V2.shape and Y.dtype == V2.dtype and Y.is_contiguous()
    cop = op.c_struct()
    _check(load().kernel_matmat_noalloc(ctx.handle, ctypes.byref(cop),
                                        ctypes.c_void_p(V2.data_ptr()), V2.shape[1],
                                        ctypes.c_void_p(Y.data_ptr())))
    return Y.reshape(V.shape)


def stored_elements(n: int, layout: int) -> int:
    v = load().ld_stored_elements(n, layout)
    if v < 0:
        raise LogdetError(LD_EINVAL, "bad stored-matrix size query")
    return int(v)


def kernel_materialize(ctx: Context, op: GPOperator, out=None):
    """Stored M in op.layout (row-major: shape (n, n); tiled: a flat buffer)."""
    torch = _torch()
    count = stored_elements(op.n, op.layout)
    if out is None:
        shape = (op.n, op.n) if op.layout == LD_ROW_MAJOR else (count,)
        out = torch.empty(shape, dtype=_dtype(op.precision), device=f"cuda:{ctx.device}")
    M = out
    assert M.is_cuda and M.dtype == _dtype(op.precision) and M.is_contiguous()
    assert M.numel() == count
    cop = op.c_struct()
    _check(load().kernel_materialize(ctx.handle, ctypes.byref(cop), ctypes.c_void_p(M.data_ptr())))
    return M


class Precond:
    """Library-owned preconditioner: the randomized truncated SVD by default,
    or any kind of the Appendix's list (LD_PRECOND_*), optionally "plus
    scaling" (D = noise I)."""

    def __init__(self, ctx: Context, op: GPOperator, rank: int, oversample: int = 10,
                 power_iters: int = 2, seed: int = 0, kind: int = LD_PRECOND_RSVD,
                 scaled: bool = False):
        self.ctx = ctx
        h = ctypes.c_void_p()
        cop = op.c_struct()
        if kind == LD_PRECOND_RSVD and not scaled:
            _check(load().logdet_precond_build(ctx.handle, ctypes.byref(cop), rank, oversample,
                                               power_iters, seed, ctypes.byref(h)))
        else:
            _check(load().logdet_precond_build_kind(ctx.handle, ctypes.byref(cop), kind, rank,
                                                    oversample, power_iters, seed,
                                                    LD_PRECOND_SCALED if scaled else 0,
                                                    ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        r = ctypes.c_int32()
        ld = ctypes.c_double()
        _check(load().ld_precond_info(h, ctypes.byref(n), ctypes.byref(r), ctypes.byref(ld)))
        self.n, self.rank, self.logdet = n.value, r.value, ld.value

    def export(self):
        torch = _torch()
        dev = f"cuda:{self.ctx.device}"
        U = torch.empty((self.n, self.rank), dtype=torch.float64, device=dev)
        lam = torch.empty((self.rank,), dtype=torch.float64, device=dev)
        D = torch.empty((self.n,), dtype=torch.float64, device=dev)
        _check(load().ld_precond_export(self.ctx.handle, self.handle, ctypes.c_void_p(U.data_ptr()),
                                        ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(D.data_ptr())))
        self.ctx.synchronize()
        return U, lam, D

    def apply_inverse(self, R, precision: int = LD_F64):
        torch = _torch()
        R2 = R if R.dim() == 2 else R.reshape(self.n, 1)
        assert R2.is_cuda and R2.dtype == _dtype(precision) and R2.is_contiguous()
        out = torch.empty_like(R2)
        _check(load().ld_precond_apply_inverse(self.ctx.handle, self.handle,
                                               ctypes.c_void_p(R2.data_ptr()), R2.shape[1], precision,
                                               ctypes.c_void_p(out.data_ptr())))
        return out.reshape(R.shape)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().ld_precond_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def logdet_estimate(ctx: Context, op: GPOperator, P: Precond | None, k: int, num_probes: int,
                    probe_seed: int, tol: float, max_iters: int = 5000, allow_noconv: bool = False):
    """Returns (result dict, per-probe values as a numpy array)."""
    res = Result()
    per = np.zeros(num_probes, dtype=np.float64)
    cop = op.c_struct()
    st = load().logdet_estimate(ctx.handle, ctypes.byref(cop), P.handle if P is not None else None, k,
                                num_probes, probe_seed, tol, max_iters, ctypes.byref(res),
                                per.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(st, allow=(LD_ENOCONV,) if allow_noconv else ())
    out = res.as_dict()
    out["status"] = STATUS_NAMES.get(st, st)
    return out, per


def logdet_estimate_orders(ctx: Context, op: GPOperator, P: Precond | None, ks, num_probes: int,
                           probe_seed: int, tol: float, max_iters: int = 5000,
                           allow_noconv: bool = False):
    """Estimates for every k in ks from one multi-shift solve over the union
    of their poles, with one shared probe block.  Returns (list of result
    dicts, per-probe values (len(ks), s))."""
    m = len(ks)
    res = (Result * m)()
    karr = (ctypes.c_int32 * m)(*ks)
    per = np.zeros((m, num_probes), dtype=np.float64)
    cop = op.c_struct()
    st = load().logdet_estimate_orders(ctx.handle, ctypes.byref(cop),
                                       P.handle if P is not None else None, m, karr, num_probes,
                                       probe_seed, tol, max_iters, res,
                                       per.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(st, allow=(LD_ENOCONV,) if allow_noconv else ())
    out = []
    for r in res:
        d = r.as_dict()
        d["status"] = STATUS_NAMES.get(st, st)
        out.append(d)
    return out, per


def logdet_estimate_lanczos_orders(ctx: Context, op: GPOperator, P: Precond | None, ks,
                                   num_probes: int, probe_seed: int, steps: int = 20):
    """Algorithm 1 for every k in ks from one Lanczos recurrence per probe.
    Returns (list of result dicts, per-probe values (len(ks), s))."""
    m = len(ks)
    res = (Result * m)()
    karr = (ctypes.c_int32 * m)(*ks)
    per = np.zeros((m, num_probes), dtype=np.float64)
    cop = op.c_struct()
    st = load().logdet_estimate_lanczos_orders(ctx.handle, ctypes.byref(cop),
                                               P.handle if P is not None else None, m, karr,
                                               num_probes, probe_seed, steps, res,
                                               per.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(st)
    out = []
    for r in res:
        d = r.as_dict()
        d["status"] = STATUS_NAMES.get(st, st)
        out.append(d)
    return out, per


def logdet_estimate_lanczos(ctx: Context, op: GPOperator, P: Precond | None, k: int,
                            num_probes: int, probe_seed: int, steps: int = 20):
    """Algorithm 1 as printed (t = steps Lanczos steps per probe, tridiagonal
    solves per pole).  Returns (result dict, per-probe values)."""
    res = Result()
    per = np.zeros(num_probes, dtype=np.float64)
    cop = op.c_struct()
    st = load().logdet_estimate_lanczos(ctx.handle, ctypes.byref(cop),
                                        P.handle if P is not None else None, k, num_probes,
                                        probe_seed, steps, ctypes.byref(res),
                                        per.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(st)
    out = res.as_dict()
    out["status"] = STATUS_NAMES.get(st, st)
    return out, per


def logdet_gradient(ctx: Context, op: GPOperator, P: Precond | None, num_probes: int,
                    probe_seed: int, tol: float, max_iters: int = 5000, allow_noconv: bool = False):
    """d log det M / d (lengthscale, variance, noise).  Returns (grad (3,),
    standard errors (3,), per-probe values (3, s), result dict)."""
    res = Result()
    grad = np.zeros(3)
    se = np.zeros(3)
    per = np.zeros((3, num_probes))
    cop = op.c_struct()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    st = load().logdet_gradient(ctx.handle, ctypes.byref(cop), P.handle if P is not None else None,
                                num_probes, probe_seed, tol, max_iters, dp(grad), dp(se), dp(per),
                                ctypes.byref(res))
    _check(st, allow=(LD_ENOCONV,) if allow_noconv else ())
    out = res.as_dict()
    out["status"] = STATUS_NAMES.get(st, st)
    return grad, se, per, out


@dataclass
class BatchItem:
    """One problem of a batch (caller-owned device points, FP64 (n, d))."""
    X: object
    kind: int
    lengthscale: float
    variance: float
    noise: float
    rank: int
    precond_seed: int
    probe_seed: int


def logdet_estimate_batched(ctx: Context, items, k: int, num_probes: int, oversample: int = 10,
                            power_iters: int = 2, tol: float = 1e-6, max_iters: int = 5000,
                            graph: bool = False, retune: bool = False, allow_noconv: bool = False,
                            precond_only: bool = False, want_lambda: bool = False,
                            allow_breakdown: bool = False, symmetric: bool = True):
    """Returns (list of result dicts, per-probe values (count, num_probes), status name), and
    with want_lambda also the kept eigenvalues (count, max rank), zero-padded.  With
    allow_breakdown a solver breakdown (LD_ENOTSPD: the results are still filled, the broken
    probes counted as not converged) is returned instead of raised."""
    torch = _torch()
    count = len(items)
    arr = (Instance * count)()
    for i, it in enumerate(items):
        assert it.X.is_cuda and it.X.dtype == torch.float64 and it.X.is_contiguous()
        arr[i] = Instance(X=it.X.data_ptr(), n=int(it.X.shape[0]), d=int(it.X.shape[1]),
                          kind=it.kind, lengthscale=it.lengthscale, variance=it.variance,
                          noise=it.noise, rank=it.rank, reserved=0,
                          precond_seed=it.precond_seed, probe_seed=it.probe_seed)
    res = (Result * max(count, 1))()
    per = np.zeros((max(count, 1), num_probes), dtype=np.float64)
    flags = ((LD_BATCH_GRAPH if graph else 0) | (LD_BATCH_RETUNE if retune else 0)
             | (LD_BATCH_PRECOND_ONLY if precond_only else 0)
             | (0 if symmetric else LD_BATCH_NO_SYMMETRIC))
    stride = max([it.rank for it in items] + [1])
    lam = np.zeros((max(count, 1), stride), dtype=np.float64) if want_lambda else None
    pd = ctypes.POINTER(ctypes.c_double)
    st = load().logdet_estimate_batched(ctx.handle, count, arr, k, num_probes, oversample,
                                        power_iters, tol, max_iters, flags, res,
                                        per.ctypes.data_as(pd),
                                        lam.ctypes.data_as(pd) if want_lambda else None, stride)
    allow = ((LD_ENOCONV,) if allow_noconv else ()) + ((LD_ENOTSPD,) if allow_breakdown else ())
    _check(st, allow=allow)
    out = ([r.as_dict() for r in res[:count]], per[:count], STATUS_NAMES.get(st, st))
    return out + (lam[:count],) if want_lambda else out


def surrogate_param_count() -> int:
    return int(load().ld_surrogate_param_count())


def surrogate_features(lam, kind: int, lengthscale: float, variance: float, noise: float, n: int,
                       d: int, edges) -> np.ndarray:
    """The 38 features of one problem (host computation in the library)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    edges = np.ascontiguousarray(edges, dtype=np.float64)
    out = np.zeros(LD_SUR_FEATURES, dtype=np.float32)
    _check(load().ld_surrogate_features(lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        len(lam), kind, lengthscale, variance, noise, n, d,
                                        edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


class Surrogate:
    """Ensemble MLP surrogate (library-owned parameters on the context's device)."""

    def __init__(self, ctx: Context, members: int = 5, seed: int = 0):
        self.ctx = ctx
        self.members = members
        h = ctypes.c_void_p()
        _check(load().ld_surrogate_create(ctx.handle, members, seed, ctypes.byref(h)))
        self.handle = h

    def set_scaling(self, x_mean, x_std, y_mean: float, y_std: float):
        fp = ctypes.POINTER(ctypes.c_float)
        xm = np.ascontiguousarray(x_mean, dtype=np.float32)
        xs = np.ascontiguousarray(x_std, dtype=np.float32)
        _check(load().ld_surrogate_set_scaling(self.ctx.handle, self.handle, xm.ctypes.data_as(fp),
                                               xs.ctypes.data_as(fp), float(y_mean), float(y_std)))

    def train_step(self, X, y, lr: float = 1e-3, want_loss: bool = True):
        loss = np.zeros(self.members, dtype=np.float64)
        _check(load().ld_surrogate_train_step(
            self.ctx.handle, self.handle, X.data_ptr(), y.data_ptr(), int(X.shape[0]), lr,
            loss.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_loss else None))
        return loss if want_loss else None

    def gradient(self, member: int, X, y):
        torch = _torch()
        g = torch.empty(surrogate_param_count(), dtype=torch.float32, device=X.device)
        loss = ctypes.c_double()
        _check(load().ld_surrogate_gradient(self.ctx.handle, self.handle, member, X.data_ptr(),
                                            y.data_ptr(), int(X.shape[0]), g.data_ptr(),
                                            ctypes.byref(loss)))
        return g, loss.value

    def get_params(self, member: int):
        torch = _torch()
        out = torch.empty(surrogate_param_count(), dtype=torch.float32, device="cuda")
        _check(load().ld_surrogate_params(self.ctx.handle, self.handle, member, out.data_ptr(), None))
        self.ctx.synchronize()
        return out

    def set_params(self, member: int, p):
        _check(load().ld_surrogate_params(self.ctx.handle, self.handle, member, None, p.data_ptr()))
        self.ctx.synchronize()

    def predict(self, X):
        torch = _torch()
        N = int(X.shape[0])
        mean = torch.empty(N, dtype=torch.float32, device=X.device)
        sd = torch.empty(N, dtype=torch.float32, device=X.device)
        _check(load().ld_surrogate_predict(self.ctx.handle, self.handle, X.data_ptr(), N,
                                           mean.data_ptr(), sd.data_ptr()))
        return mean, sd

    def close(self):
        if getattr(self, "handle", None):
            load().ld_surrogate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""MI355X pairwise-perturbation CP-ALS: Python binding of libppals.so.

This module only marshals arguments: device buffers are PyTorch tensors
(memory and streams), every computation runs in the library's HIP kernels.
The function names mirror the C ABI declared in include/ppals.h:
cp_als_sweep, pp_build_operators, pp_sweep, gram_solve, plus the auxiliary
entry points (norm, bf16 cast, MTTKRP, first-level contraction, PP right-hand
side, operators, exact residual and the native decomposition driver), the
batched engine and the Tucker path of orders 3 to 8 (TuckerPlan: tucker_ttmc,
tucker_factor_update, tucker_hosvd, tucker_hosvd_interlaced, tucker_als_sweep,
tucker_pp_build, tucker_pp_rhs, tucker_pp_sweep, tucker_run).
"""
from __future__ import annotations

import collections.abc
import ctypes
import json
import operator

import torch

from . import _lib
from ._lib import (PPALS_BF16, PPALS_FP32, PPALS_FP64, RECORD_BYTES, SWEEP_ALS,  # noqa: F401
                   SWEEP_PP_APPROX, SWEEP_PP_INIT, PPALSError, SweepRecord)

_DTYPES = {"f64": PPALS_FP64, "f32": PPALS_FP32, "bf16": PPALS_BF16}
KIND_NAMES = {SWEEP_ALS: "als", SWEEP_PP_INIT: "pp_init", SWEEP_PP_APPROX: "pp_approx"}
KIND_CODES = {v: k for k, v in KIND_NAMES.items()}


def lib():
    return _lib.load()


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, name, dtype=None, numel=None, min_bytes=None):
    if t is None:
        raise ValueError(f"{name} is None")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if min_bytes is not None and t.numel() * t.element_size() < min_bytes:
        raise ValueError(f"{name} must hold at least {min_bytes} bytes")
    return t


def _factor_array(plan, A):
    if len(A) != plan.order:
        raise ValueError(f"expected {plan.order} factors")
    for n, a in enumerate(A):
        _dev(a, f"A[{n}]", torch.float64, plan.dims[n] * plan.rank)
    return (ctypes.c_void_p * len(A))(*[a.data_ptr() for a in A])


class Plan:
    """Host plan: dimension-tree schedules and the workspace layout."""

    def __init__(self, dims, rank, tensor_dtype="f64", level1_dtype=None, second_order=True,
                 step_size=1.0, pp_build="tree"):
        dims = [int(d) for d in dims]
        if level1_dtype is None:
            level1_dtype = tensor_dtype
        d = _lib.Desc()
        d.order = len(dims)
        d.rank = int(rank)
        for i, s in enumerate(dims[:_lib.MAX_ORDER]):
            d.dims[i] = s
        d.tensor_dtype = _DTYPES[tensor_dtype]
        d.level1_dtype = _DTYPES[level1_dtype]
        d.use_second_order = 1 if second_order else 0
        d.step_size = float(step_size)
        # "tree", "direct" (every operator from X), "auto" (the plan's cost model) or the
        # number of leading tree levels to combine
        if pp_build == "tree":
            d.pp_build_levels = 0
        elif pp_build == "direct":
            d.pp_build_levels = max(1, len(dims) - 2)
        elif pp_build == "auto":
            d.pp_build_levels = -1
        elif isinstance(pp_build, int) and pp_build >= 0:
            d.pp_build_levels = pp_build
        else:
            raise ValueError("pp_build must be 'tree', 'direct', 'auto' or a level count")
        h = ctypes.c_void_p()
        _lib.check(lib().ppals_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.dims = dims
        self.order = len(dims)
        self.rank = int(rank)
        self.tensor_dtype = tensor_dtype
        self.level1_dtype = level1_dtype
        self.second_order = bool(second_order)
        self.step_size = float(step_size)
        self.pp_build = pp_build
        self.torch_dtype = torch.float64 if tensor_dtype == "f64" else torch.float32

    @property
    def handle(self):
        return self._h

    @property
    def workspace_bytes(self):
        return int(lib().ppals_workspace_bytes(self._h))

    def describe(self):
        buf = ctypes.create_string_buffer(1 << 20)
        _lib.check(lib().ppals_plan_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def workspace(self, device="cuda"):
        return torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ppals_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _x(self, X, Xb):
        n = 1
        for s in self.dims:
            n *= s
        _dev(X, "X", self.torch_dtype, n)
        if self.level1_dtype == "bf16":
            _dev(Xb, "X_bf16", None, n)
            if Xb.element_size() != 2:
                raise ValueError("X_bf16 must hold 2-byte bfloat16 bit patterns")
            return _p(X), _p(Xb)
        return _p(X), None


def set_profiling(plan, enable=True):
    _lib.check(lib().ppals_set_profiling(plan.handle, 1 if enable else 0))


def get_profile(plan, reset=False):
    """Per-kernel-class statistics: {name: {launches, total_ms, avg_ms, flops, bytes}}."""
    arr = (_lib.KernelStat * _lib.PROF_CLASSES)()
    n = ctypes.c_int32(0)
    _lib.check(lib().ppals_get_profile(plan.handle, arr, _lib.PROF_CLASSES, ctypes.byref(n),
                                       1 if reset else 0))
    out = {}
    for i in range(n.value):
        e = arr[i]
        out[e.name.decode()] = {
            "launches": int(e.launches), "total_ms": e.total_ms,
            "avg_ms": e.total_ms / e.launches if e.launches else 0.0,
            "flops": e.flops, "bytes": e.bytes,
        }
    return out


def new_record(device="cuda"):
    return torch.zeros(RECORD_BYTES, dtype=torch.uint8, device=device)


def read_record(rec):
    raw = bytes(rec.detach().to("cpu").numpy().tobytes())
    r = SweepRecord.from_buffer_copy(raw[:RECORD_BYTES])
    return record_dict(r)


def record_dict(r, order=None):
    n = _lib.MAX_ORDER if order is None else order
    return {
        "fit_est": r.fit_est,
        "grad_norm": r.grad_norm[:n],
        "rel_change": r.rel_change[:n],
        "chol_status": r.chol_status[:n],
        "kind": KIND_NAMES.get(r.sweep_kind, str(r.sweep_kind)),
        "ctrl_pred": r.ctrl_pred,
        "ctrl_true_err": r.ctrl_true_err,
        "ctrl_leave": r.ctrl_leave,
        "ctrl_fallback": r.ctrl_fallback,
        "chol_pivot": r.chol_pivot[:n],
        "nonfinite": r.nonfinite[:n],
    }


def cp_als_sweep(plan, X, X_bf16, A, S, normX2, ws, rec, stream=None):
    x, xb = plan._x(X, X_bf16)
    _dev(S, "S", torch.float64, plan.order * plan.rank * plan.rank)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _dev(rec, "rec", min_bytes=RECORD_BYTES)
    _lib.check(lib().cp_als_sweep(plan.handle, x, xb, _factor_array(plan, A), _p(S), float(normX2),
                                  _p(ws), _p(rec), _stream(stream)))


def pp_build_operators(plan, X, X_bf16, A, ws, stream=None):
    x, xb = plan._x(X, X_bf16)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _lib.check(lib().pp_build_operators(plan.handle, x, xb, _factor_array(plan, A), _p(ws),
                                        _stream(stream)))


def pp_sweep(plan, A, S, normX2, ws, rec, stream=None):
    _dev(S, "S", torch.float64, plan.order * plan.rank * plan.rank)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _dev(rec, "rec", min_bytes=RECORD_BYTES)
    _lib.check(lib().pp_sweep(plan.handle, _factor_array(plan, A), _p(S), float(normX2), _p(ws),
                              _p(rec), _stream(stream)))


def gram_solve_workspace_bytes(R, rows):
    return int(lib().ppals_gram_solve_workspace_bytes(int(R), int(rows)))


def gram_solve(R, rows, Gamma, M, A, grad_out, status_out, ws, stream=None):
    _dev(Gamma, "Gamma", torch.float64, R * R)
    if M.dtype not in (torch.float64, torch.float32):
        raise ValueError("M must be float64 or float32")
    _dev(M, "M", None, rows * R)
    _dev(A, "A", torch.float64, rows * R)
    _dev(grad_out, "grad_out", torch.float64)
    _dev(status_out, "status_out", torch.int32)
    _dev(ws, "ws", min_bytes=gram_solve_workspace_bytes(R, rows))
    mdt = PPALS_FP64 if M.dtype == torch.float64 else PPALS_FP32
    _lib.check(lib().gram_solve(int(R), int(rows), _p(Gamma), _p(M), mdt, _p(A), _p(grad_out),
                                _p(status_out), _p(ws), _stream(stream)))


GRAM_SOLVE_NOALLOC_MAX_ROWS = 65536


def gram_solve_noalloc(R, rows, Gamma, M, A, grad_out, status_out, stream=None):
    """gram_solve with the library's fixed scratch array instead of a workspace (no
    device allocation; calls on one GPU must not overlap)."""
    _dev(Gamma, "Gamma", torch.float64, R * R)
    if M.dtype not in (torch.float64, torch.float32):
        raise ValueError("M must be float64 or float32")
    _dev(M, "M", None, rows * R)
    _dev(A, "A", torch.float64, rows * R)
    _dev(grad_out, "grad_out", torch.float64)
    _dev(status_out, "status_out", torch.int32)
    mdt = PPALS_FP64 if M.dtype == torch.float64 else PPALS_FP32
    _lib.check(lib().gram_solve_noalloc(int(R), int(rows), _p(Gamma), _p(M), mdt, _p(A),
                                        _p(grad_out), _p(status_out), _stream(stream)))


def tensor_norm2(X, out, ws=None, stream=None):
    if X.dtype not in (torch.float64, torch.float32):
        raise ValueError("X must be float64 or float32")
    _dev(X, "X")
    _dev(out, "out", torch.float64)
    nb = int(lib().ppals_norm2_workspace_bytes())
    if ws is None:
        ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    _dev(ws, "ws", min_bytes=nb)
    dt = PPALS_FP64 if X.dtype == torch.float64 else PPALS_FP32
    _lib.check(lib().ppals_tensor_norm2(_p(X), dt, X.numel(), _p(out), _p(ws), _stream(stream)))


def cast_bf16(X32, out, stream=None):
    _dev(X32, "X", torch.float32)
    _dev(out, "out", None, X32.numel())
    if out.element_size() != 2:
        raise ValueError("out must have 2-byte elements")
    _lib.check(lib().ppals_cast_bf16(_p(X32), _p(out), X32.numel(), _stream(stream)))


def mttkrp(plan, X, X_bf16, A, mode, out, ws, stream=None):
    x, xb = plan._x(X, X_bf16)
    _dev(out, "out", torch.float64, plan.dims[mode] * plan.rank)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _lib.check(lib().ppals_mttkrp(plan.handle, x, xb, _factor_array(plan, A), int(mode), _p(out),
                                  _p(ws), _stream(stream)))


def level1(plan, X, X_bf16, A, contract_modes, out, ws, stream=None):
    x, xb = plan._x(X, X_bf16)
    mask = 0
    for m in contract_modes:
        mask |= 1 << int(m)
    n = plan.rank
    for i in range(plan.order):
        if i not in contract_modes:
            n *= plan.dims[i]
    _dev(out, "out", plan.torch_dtype, n)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _lib.check(lib().ppals_level1(plan.handle, x, xb, _factor_array(plan, A), mask, _p(out),
                                  _p(ws), _stream(stream)))


def pp_rhs(plan, A, S, mode, out, ws, stream=None):
    _dev(S, "S", torch.float64, plan.order * plan.rank * plan.rank)
    _dev(out, "out", torch.float64, plan.dims[mode] * plan.rank)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _lib.check(lib().ppals_pp_rhs(plan.handle, _factor_array(plan, A), _p(S), int(mode), _p(out),
                                  _p(ws), _stream(stream)))


def get_operator(plan, ws, i, j, out, stream=None):
    _dev(out, "out", plan.torch_dtype, plan.dims[i] * plan.dims[j] * plan.rank)
    _lib.check(lib().ppals_get_operator(plan.handle, _p(ws), int(i), int(j), _p(out),
                                        _stream(stream)))


def exact_residual2(plan, X, A, out, ws, stream=None):
    x, _ = plan._x(X, None) if plan.level1_dtype != "bf16" else (_p(X), None)
    _dev(out, "out", torch.float64)
    _lib.check(lib().ppals_exact_residual2(plan.handle, x, _factor_array(plan, A), _p(out), _p(ws),
                                           _stream(stream)))


class Records(collections.abc.Sequence):
    """The sweep records of a run, each turned into a dict (record_dict) when read."""

    def __init__(self, raw, count, order):
        self._raw, self._n, self._order = raw, count, order

    def __len__(self):
        return self._n

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[k] for k in range(*i.indices(self._n))]
        i = operator.index(i)
        if i < 0:
            i += self._n
        if not 0 <= i < self._n:
            raise IndexError(i)
        return record_dict(self._raw[i], self._order)


def run(plan, X, X_bf16, A, S, normX2, ws, rec, eps, max_sweeps, delta=0.0, replay=None,
        timing=True, stream=None):
    """Native decomposition driver (Algorithm 3 control; eps <= 0 gives plain ALS).

    Returns (records, sweep_ms): a sequence of one dict per sweep (Records) and the device
    time of each.
    """
    x, xb = plan._x(X, X_bf16)
    _dev(S, "S", torch.float64, plan.order * plan.rank * plan.rank)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _dev(rec, "rec", min_bytes=RECORD_BYTES)
    n = int(max_sweeps)
    recs = (SweepRecord * max(1, n))()
    ms = (ctypes.c_float * max(1, n))() if timing else None
    done = ctypes.c_int32(0)
    rp = None
    if replay is not None:
        codes = [KIND_CODES[k] if isinstance(k, str) else int(k) for k in replay]
        if len(codes) < n:
            raise ValueError("replay shorter than max_sweeps")
        rp = (ctypes.c_int32 * len(codes))(*codes)
    _lib.check(lib().ppals_run(plan.handle, x, xb, _factor_array(plan, A), _p(S), float(normX2),
                               _p(ws), _p(rec), float(eps), float(delta), n, rp, recs,
                               ms, ctypes.byref(done), _stream(stream)))
    return Records(recs, done.value, plan.order), (ms[:done.value] if timing else None)


# ---- learned PP controller --------------------------------------------------

def mlp_n_params(d, hidden):
    return hidden * d + 2 * hidden + 1


def mlp_forward(params, d, hidden, X, y, hcache=None, stream=None):
    B = X.shape[0]
    _dev(params, "params", torch.float32, mlp_n_params(d, hidden))
    _dev(X, "X", torch.float32, B * d)
    _dev(y, "y", torch.float32, B)
    if hcache is not None:
        _dev(hcache, "hcache", torch.float32, B * hidden)
    _lib.check(lib().ppals_mlp_forward(_p(params), int(d), int(hidden), _p(X), int(B), _p(y),
                                       _p(hcache), _stream(stream)))


def mlp_backward(params, d, hidden, X, hcache, y, t, grad, loss=None, stream=None):
    B = X.shape[0]
    _dev(params, "params", torch.float32, mlp_n_params(d, hidden))
    _dev(X, "X", torch.float32, B * d)
    _dev(hcache, "hcache", torch.float32, B * hidden)
    _dev(y, "y", torch.float32, B)
    _dev(t, "t", torch.float32, B)
    _dev(grad, "grad", torch.float32, mlp_n_params(d, hidden))
    if loss is not None:
        _dev(loss, "loss", torch.float32, 1)
    _lib.check(lib().ppals_mlp_backward(_p(params), int(d), int(hidden), _p(X), _p(hcache), _p(y),
                                        _p(t), int(B), _p(grad), _p(loss), _stream(stream)))


def mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    P = params.numel()
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _dev(t, name, torch.float32, P)
    _lib.check(lib().ppals_mlp_adam(_p(params), _p(grad), _p(m), _p(v), int(P), int(step),
                                    float(lr), float(beta1), float(beta2), float(eps),
                                    _stream(stream)))


def pp_rhs_error(plan, X, X_bf16, A, S, ws, err, stream=None):
    """Device double err := max_n ||M~^(n) - M^(n)|| / ||M^(n)|| at the current factors."""
    x, xb = plan._x(X, X_bf16)
    _dev(S, "S", torch.float64, plan.order * plan.rank * plan.rank)
    _dev(ws, "ws", min_bytes=plan.workspace_bytes)
    _dev(err, "err", torch.float64)
    _lib.check(lib().ppals_pp_rhs_error(plan.handle, x, xb, _factor_array(plan, A), _p(S), _p(ws),
                                        _p(err), _stream(stream)))


def set_controller(plan, params=None, hidden=64, log10_tau=-2.0, rho_cap=0.3, check_period=0,
                   fallback_factor=10.0):
    """Attach a learned controller to the plan's native driver (params=None detaches).
    The parameter tensor must stay alive while attached."""
    if params is None:
        _lib.check(lib().ppals_set_controller(plan.handle, None))
        plan._ctl_params = None
        return
    _dev(params, "params", torch.float32, mlp_n_params(plan.order + 2, hidden))
    c = _lib.Controller(params=params.data_ptr(), hidden=int(hidden), check_period=int(check_period),
                        log10_tau=float(log10_tau), rho_cap=float(rho_cap),
                        fallback_factor=float(fallback_factor))
    _lib.check(lib().ppals_set_controller(plan.handle, ctypes.byref(c)))
    plan._ctl_params = params


# ---- batched execution ------------------------------------------------------

class Batch:
    """Many independent order-3 problems (FP32 tensors, FP64 factors) advanced by the
    library's grouped kernels with per-problem device state machines."""

    def __init__(self, problems, max_sweeps):
        arr = (_lib.BatchProblem * len(problems))()
        for i, (dims, rank) in enumerate(problems):
            if len(dims) != 3:
                raise ValueError("batched problems are order 3")
            arr[i].dims[:] = [int(d) for d in dims]
            arr[i].rank = int(rank)
        h = ctypes.c_void_p()
        _lib.check(lib().ppals_batch_create(arr, len(problems), int(max_sweeps), ctypes.byref(h)))
        self._h = h
        self.problems = [(tuple(int(d) for d in dims), int(rank)) for dims, rank in problems]
        self.count = len(problems)
        self.max_sweeps = int(max_sweeps)
        self._bound = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().ppals_batch_destroy(h)
            self._h = None

    @property
    def workspace_bytes(self):
        return int(lib().ppals_batch_workspace_bytes(self._h))

    def workspace(self, device="cuda"):
        return torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=device)

    def bind(self, X, A, ws, eps, tol, second_order=True, stream=None):
        if len(X) != self.count or len(A) != self.count:
            raise ValueError("need one tensor and three factors per problem")
        for p, ((dims, R), x, fs) in enumerate(zip(self.problems, X, A)):
            _dev(x, f"X[{p}]", torch.float32, dims[0] * dims[1] * dims[2])
            for n in range(3):
                _dev(fs[n], f"A[{p}][{n}]", torch.float64, dims[n] * R)
        _dev(ws, "ws", min_bytes=self.workspace_bytes)
        xs = (ctypes.c_void_p * self.count)(*[x.data_ptr() for x in X])
        As = (ctypes.c_void_p * (3 * self.count))(*[f.data_ptr() for fs in A for f in fs])
        _lib.check(lib().ppals_batch_bind(self._h, xs, As, _p(ws), float(eps), float(tol),
                                          1 if second_order else 0, _stream(stream)))
        self._bound = (X, A, ws)

    def autotune(self, ws, reps=3, stream=None):
        _lib.check(lib().ppals_batch_autotune(self._h, _p(ws), int(reps), _stream(stream)))

    def sweep(self, ws, stream=None):
        _lib.check(lib().ppals_batch_sweep(self._h, _p(ws), _stream(stream)))

    def run(self, ws, sweeps, use_graph=True, stream=None):
        _lib.check(lib().ppals_batch_run(self._h, _p(ws), int(sweeps), 1 if use_graph else 0,
                                         _stream(stream)))

    def results(self, ws, stream=None):
        out = (_lib.BatchResult * self.count)()
        _lib.check(lib().ppals_batch_results(self._h, _p(ws), out, _stream(stream)))
        return [{
            "sweeps": r.sweeps, "converged_sweep": r.converged_sweep, "n_als": r.n_als,
            "n_pp_init": r.n_pp_init, "n_pp_approx": r.n_pp_approx, "done": r.done,
            "chol_status": list(r.chol_status), "fit": r.fit, "normX2": r.normX2,
            "rel_change": list(r.rel_change), "time_to_converge_ms": r.time_to_converge_ms,
        } for r in out]

    def kind_log(self, ws, stream=None):
        import numpy as np
        buf = (ctypes.c_uint8 * (self.count * self.max_sweeps))()
        _lib.check(lib().ppals_batch_kind_log(self._h, _p(ws), buf, _stream(stream)))
        return np.frombuffer(bytes(buf), dtype=np.uint8).reshape(self.count, self.max_sweeps)

    def describe(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _lib.check(lib().ppals_batch_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())


BATCH_KIND_NAMES = {1: "als", 2: "pp_init", 3: "pp_approx"}


# ---- Tucker (order 3) -----------------------------------------------------------

TUCKER_RECORD_FIELDS = ("iters", "converged", "rr_status", "fit", "core_norm", "f_norm",
                        "rel_change", "ritz_residual", "ms")


def tucker_record_dict(r, order=3):
    d = {"kind": KIND_NAMES.get(r.kind, str(r.kind))}
    for f in TUCKER_RECORD_FIELDS:
        v = getattr(r, f)
        d[f] = list(v)[:order] if hasattr(v, "__len__") else v
    return d


class TuckerPlan:
    """Tucker plan of order 3 to 8 (HOOI and PP-Tucker-ALS, FP64): sizes, solver limits
    and the workspace layout.  Tensors and factors are float64 device tensors."""

    def __init__(self, dims, rank, tol=None, max_iters=None, hosvd_max_iters=None):
        dims = [int(d) for d in dims]
        arr = (ctypes.c_int64 * len(dims))(*dims)
        h = ctypes.c_void_p()
        _lib.check(lib().tucker_plan_create(len(dims), arr, int(rank), ctypes.byref(h)))
        self._h = h
        self.dims = dims
        self.order = len(dims)
        self.rank = int(rank)
        if tol is not None or max_iters is not None or hosvd_max_iters is not None:
            self.set_solver(1e-12 if tol is None else tol, 500 if max_iters is None else max_iters,
                            5000 if hosvd_max_iters is None else hosvd_max_iters)

    def set_solver(self, tol, max_iters, hosvd_max_iters):
        _lib.check(lib().tucker_set_solver(self._h, float(tol), int(max_iters),
                                           int(hosvd_max_iters)))

    @property
    def workspace_bytes(self):
        return int(lib().tucker_workspace_bytes(self._h))

    def workspace(self, device="cuda"):
        return torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=device)

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and h.value:
                lib().tucker_plan_destroy(h)
                self._h = None
        except Exception:
            pass

    def _X(self, X):
        n = 1
        for s in self.dims:
            n *= s
        return _dev(X, "X", torch.float64, n)

    def _A(self, A, name="A"):
        if len(A) != self.order:
            raise ValueError(f"{name} needs {self.order} factors")
        for n, a in enumerate(A):
            _dev(a, f"{name}[{n}]", torch.float64, self.dims[n] * self.rank)
        return (ctypes.c_void_p * self.order)(*[a.data_ptr() for a in A])

    def _ws(self, ws):
        return _dev(ws, "ws", min_bytes=self.workspace_bytes)

    def _G(self, G):
        return _dev(G, "G", torch.float64, self.rank ** self.order)

    def _Y(self, Y, mode):
        return _dev(Y, "Y", torch.float64, self.dims[mode] * self.rank ** (self.order - 1))


def tucker_ttmc(plan, ws, X, A, mode, Y, stream=None):
    _lib.check(lib().tucker_ttmc(plan._h, _p(plan._ws(ws)), _p(plan._X(X)), plan._A(A), int(mode),
                                 _p(plan._Y(Y, mode)), _stream(stream)))


def tucker_factor_update(plan, ws, Y, mode, A_prev, A_out, stream=None):
    """Returns {iterations, converged, rr_status, residual}."""
    _dev(A_prev, "A_prev", torch.float64, plan.dims[mode] * plan.rank)
    _dev(A_out, "A_out", torch.float64, plan.dims[mode] * plan.rank)
    info = (ctypes.c_int32 * 3)()
    res = ctypes.c_double()
    _lib.check(lib().tucker_factor_update(plan._h, _p(plan._ws(ws)), _p(plan._Y(Y, mode)),
                                          int(mode), _p(A_prev), _p(A_out), info,
                                          ctypes.byref(res), _stream(stream)))
    return {"iterations": info[0], "converged": info[1], "rr_status": info[2],
            "residual": res.value}


def tucker_hosvd(plan, ws, X, V0, A, G, stream=None):
    """Returns the per-mode [iterations, converged, rr_status]."""
    info = (ctypes.c_int32 * (3 * plan.order))()
    _lib.check(lib().tucker_hosvd(plan._h, _p(plan._ws(ws)), _p(plan._X(X)), plan._A(V0, "V0"),
                                  plan._A(A), _p(plan._G(G)), info, _stream(stream)))
    return [list(info[3 * n:3 * n + 3]) for n in range(plan.order)]


def tucker_hosvd_interlaced(plan, ws, X, V0, A, G, stream=None):
    """Returns the per-mode [iterations, converged, rr_status]."""
    info = (ctypes.c_int32 * (3 * plan.order))()
    _lib.check(lib().tucker_hosvd_interlaced(plan._h, _p(plan._ws(ws)), _p(plan._X(X)),
                                             plan._A(V0, "V0"), plan._A(A), _p(plan._G(G)),
                                             info, _stream(stream)))
    return [list(info[3 * n:3 * n + 3]) for n in range(plan.order)]


def tucker_als_sweep(plan, ws, X, A, G, normX2, stream=None):
    rec = _lib.TuckerRecord()
    _lib.check(lib().tucker_als_sweep(plan._h, _p(plan._ws(ws)), _p(plan._X(X)), plan._A(A),
                                      _p(plan._G(G)), float(normX2), ctypes.byref(rec),
                                      _stream(stream)))
    return tucker_record_dict(rec, plan.order)


def tucker_pp_build(plan, ws, X, A, stream=None):
    _lib.check(lib().tucker_pp_build(plan._h, _p(plan._ws(ws)), _p(plan._X(X)), plan._A(A),
                                     _stream(stream)))


def tucker_pp_rhs(plan, ws, mode, Y, stream=None):
    _lib.check(lib().tucker_pp_rhs(plan._h, _p(plan._ws(ws)), int(mode), _p(plan._Y(Y, mode)),
                                   _stream(stream)))


def tucker_pp_sweep(plan, ws, A, G, normX2, kind="pp_approx", stream=None):
    rec = _lib.TuckerRecord()
    _lib.check(lib().tucker_pp_sweep(plan._h, _p(plan._ws(ws)), plan._A(A), _p(plan._G(G)),
                                     float(normX2), KIND_CODES[kind], ctypes.byref(rec),
                                     _stream(stream)))
    return tucker_record_dict(rec, plan.order)


def tucker_run(plan, ws, X, A, G, eps, sweeps, delta=0.0, replay=None, stream=None):
    """PP-Tucker-ALS control (eps = 0: plain Tucker-ALS); returns the list of records."""
    recs = (_lib.TuckerRecord * max(1, int(sweeps)))()
    n_out = ctypes.c_int32()
    if replay is not None:
        codes = [KIND_CODES[k] for k in replay]
        rp = (ctypes.c_int32 * max(1, len(codes)))(*codes)
        rlen = len(codes)
    else:
        rp, rlen = None, 0
    _lib.check(lib().tucker_run(plan._h, _p(plan._ws(ws)), _p(plan._X(X)), plan._A(A),
                                _p(plan._G(G)), float(eps), int(sweeps), float(delta), rp, rlen,
                                recs, ctypes.byref(n_out), _stream(stream)))
    return [tucker_record_dict(recs[i], plan.order) for i in range(n_out.value)]

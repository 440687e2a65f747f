"""Python binding of the MI355X Leja phi-action library (libleja.so).

Argument marshalling only: every step of phi_l(hJ)v -- power iteration,
divided differences, the fused Newton recurrence, substepping, the stage
driver -- runs in the HIP kernels behind the C ABI of include/leja.h.  PyTorch
supplies device memory (float64 CUDA tensors) and streams.

The functions carry the C names.  Tensors are checked (device, dtype, shape,
contiguity) before their pointers cross the ABI.
"""
from __future__ import annotations

import contextlib
import ctypes as C
from dataclasses import dataclass
from typing import Sequence

from . import _lib
from ._lib import (  # noqa: F401
    LJ_EHIP, LJ_EINVAL, LJ_ENOMEM, LJ_ENOTCONV, LJ_EPIRK4S3, LJ_EPIRK4S3_LEKRY, LJ_EPIRK4S3A, LJ_EPIRK4S3A_LEKRY, LJ_EXPRB2, LJ_EXPRB43, LJ_EXPRB43_U3,
    LJ_MAX_K, LJ_MAX_L, LJ_OK, LJ_OP_ADR2D, LJ_OP_ADVDIFF2D, LJ_OP_ALLENCAHN2D, LJ_OP_BRUSSELATOR2D, LJ_OP_BURGERS2D,
    LJ_NOALLOC_SCRATCH_BYTES, LJ_OP_DIAG, LJ_OP_GRAYSCOTT2D, LJ_PROPOSAL_MARGIN, LejaLibraryError, lj_integrate_stats, lj_operator, lj_options, lj_stats, lj_step_record,
    lj_timing,
)

KIND_CODES = {
    "diag": LJ_OP_DIAG, "advdiff": LJ_OP_ADVDIFF2D, "allencahn": LJ_OP_ALLENCAHN2D,
    "brusselator": LJ_OP_BRUSSELATOR2D, "burgers": LJ_OP_BURGERS2D, "grayscott": LJ_OP_GRAYSCOTT2D,
    "adr": LJ_OP_ADR2D,
}
SCHEMES = {"EXPRB2": LJ_EXPRB2, "EXPRB43_U3": LJ_EXPRB43_U3, "EXPRB43": LJ_EXPRB43, "EPIRK4S3": LJ_EPIRK4S3,
           "EPIRK4S3_LEKRY": LJ_EPIRK4S3_LEKRY, "EPIRK4S3A": LJ_EPIRK4S3A, "EPIRK4S3A_LEKRY": LJ_EPIRK4S3A_LEKRY}


class LejaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"leja error {code}: {msg}")
        self.code = code


def lib():
    return _lib.load()


def _stream_ptr(stream) -> C.c_void_p:
    import torch
    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:  # the current stream's handle without building a Stream object
            return C.c_void_p(raw(torch.cuda.current_device()))
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _tensor_ptr(t, n: int, what: str) -> C.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} entries, expected {n}")
    return C.c_void_p(t.data_ptr())


@dataclass
class Operator:
    """An lj_operator plus the tensor that keeps its state alive."""

    kind: str
    nx: int
    ny: int
    ncomp: int
    dx: float
    dy: float
    coef: Sequence[float]
    state: object = None  # float64 CUDA tensor or None

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.ncomp

    def c_struct(self) -> lj_operator:
        # rebuilt only when a field or the state tensor's storage changed
        key = (self.kind, self.nx, self.ny, self.ncomp, self.dx, self.dy, tuple(self.coef),
               None if self.state is None else (self.state.data_ptr(), self.state.numel(), self.state.dtype,
                                                self.state.is_contiguous(), self.state.device))
        cached = self.__dict__.get("_c_cache")
        if cached is not None and cached[0] == key:
            return cached[1]
        op = self._build_c_struct()
        self.__dict__["_c_cache"] = (key, op)
        return op

    def _build_c_struct(self) -> lj_operator:
        op = lj_operator()
        op.kind = KIND_CODES[self.kind]
        op.nx, op.ny, op.ncomp = self.nx, self.ny, self.ncomp
        op.dx, op.dy = float(self.dx), float(self.dy)
        for i in range(8):
            op.coef[i] = float(self.coef[i]) if i < len(self.coef) else 0.0
        op.state = _tensor_ptr(self.state, self.n, "operator state").value if self.state is not None else None
        return op


def lj_default_options(**overrides) -> lj_options:
    o = lj_options()
    lib().lj_default_options(C.byref(o))
    for k, v in overrides.items():
        if k == "pi_start":
            v = C.c_void_p(v.data_ptr()) if v is not None else None
        if k == "bound_device" and v is not None and not isinstance(v, int):
            v = v.data_ptr()  # a float64 device tensor holding the bound
        setattr(o, k, v)
    return o


def lj_leja_points(count: int = 101):
    buf = (C.c_double * count)()
    rc = lib().lj_leja_points(buf, count)
    if rc != LJ_OK:
        raise LejaError(rc, "lj_leja_points")
    return list(buf)


def lj_version() -> str:
    return lib().lj_version().decode()


class Context:
    """Owns an lj_context on one HIP device."""

    def __init__(self, device: int = 0):
        self._lib = lib()
        h = C.c_void_p()
        rc = self._lib.lj_create(C.byref(h), int(device))
        if rc != LJ_OK:
            raise LejaError(rc, self._lib.lj_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self._lib.lj_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, allow_notconv: bool = True) -> int:
        if rc < 0 or (rc == LJ_ENOTCONV and not allow_notconv):
            raise LejaError(rc, self._lib.lj_last_error(self.handle).decode())
        return rc

    def last_error(self) -> str:
        return self._lib.lj_last_error(self.handle).decode()


def lj_create(device: int = 0) -> Context:
    return Context(device)


def lj_spectral_bound(ctx: Context, J: Operator, iters: int = 20, seed: int = 0x5EED, start=None,
                      stream=None) -> float:
    op = J.c_struct()
    out = C.c_double()
    sp = _tensor_ptr(start, J.n, "start") if start is not None else None
    ctx._check(ctx._lib.lj_spectral_bound(ctx.handle, C.byref(op), int(iters), C.c_uint64(seed), sp,
                                          C.byref(out), _stream_ptr(stream)), False)
    return out.value


def lj_divided_differences(ctx: Context, l: int, s: float, c: float, gamma: float, npts: int = 101,
                           stream=None):
    buf = (C.c_double * npts)()
    ctx._check(ctx._lib.lj_divided_differences(ctx.handle, int(l), float(s), float(c), float(gamma),
                                               int(npts), buf, _stream_ptr(stream)), False)
    return list(buf)


def lj_rhs(ctx: Context, J: Operator, u, f, stream=None) -> None:
    op = J.c_struct()
    ctx._check(ctx._lib.lj_rhs(ctx.handle, C.byref(op), _tensor_ptr(u, J.n, "u"), _tensor_ptr(f, J.n, "f"),
                               _stream_ptr(stream)), False)


def lj_jv(ctx: Context, J: Operator, x, y, stream=None) -> None:
    """y = J(J.state) x for a built-in family."""
    op = J.c_struct()
    ctx._check(ctx._lib.lj_jv(ctx.handle, C.byref(op), _tensor_ptr(x, J.n, "x"), _tensor_ptr(y, J.n, "y"),
                              _stream_ptr(stream)), False)


class _DeviceVector:
    """n float64 values at a device address, exposed to torch.as_tensor through
    the CUDA array interface (no copy)."""

    def __init__(self, ptr: int, n: int):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def device_view(ptr: int, n: int):
    """A torch tensor viewing n float64 values at device address ptr."""
    import torch
    return torch.as_tensor(_DeviceVector(ptr, n), device=torch.device("cuda", torch.cuda.current_device()))


class UserOperator:
    """An operator u' = f(u) of n unknowns given by Python callables on torch
    tensors (lj_user_operator):

        rhs(x, out):     out[:] = f(x)
        jv(u, x, out):   out[:] = J(u) x

    Either may be None (jv None: the library forms finite-difference products
    from rhs; rhs None: actions only).  The callables run on the library's
    stream, which is made torch's current stream for their duration.  An
    exception raised in a callable makes the library call fail; it is re-raised
    by the wrapper."""

    def __init__(self, n: int, state, rhs=None, jv=None):
        self.n = int(n)
        self.state = state
        self.errors: list = []
        n_ = self.n

        def on_stream(stream):
            import torch
            cur = torch.cuda.current_stream()
            if stream is None or int(stream) == int(cur.cuda_stream):
                return contextlib.nullcontext()
            return torch.cuda.stream(torch.cuda.ExternalStream(int(stream)))

        def rhs_c(user, x, fx, stream):
            try:
                with on_stream(stream):
                    rhs(device_view(x, n_), device_view(fx, n_))
                return 0
            except BaseException as e:  # reported after the library call returns
                self.errors.append(e)
                return 1

        def jv_c(user, u, x, jx, stream):
            try:
                with on_stream(stream):
                    jv(device_view(u, n_), device_view(x, n_), device_view(jx, n_))
                return 0
            except BaseException as e:
                self.errors.append(e)
                return 1

        self._rhs_c = _lib.lj_rhs_fn(rhs_c) if rhs is not None else _lib.lj_rhs_fn()
        self._jv_c = _lib.lj_jv_fn(jv_c) if jv is not None else _lib.lj_jv_fn()

    def c_struct(self) -> "_lib.lj_user_operator":
        op = _lib.lj_user_operator()
        op.n = self.n
        op.rhs = self._rhs_c
        op.jv = self._jv_c
        op.user = None
        op.state = _tensor_ptr(self.state, self.n, "user operator state").value
        return op



def _user_call(ctx: Context, U: UserOperator, rc: int):
    """Raises for a failed call; a callback's own exception is chained."""
    if U.errors:
        e = U.errors[0]
        U.errors.clear()
        raise LejaError(rc, ctx.last_error()) from e
    ctx._check(rc)


def lj_user_phi_action(ctx: Context, U: UserOperator, v, w, l: int, h: float, tol: float,
                       opt: lj_options | None = None, stream=None):
    """w = phi_l(h J) v for a user operator.  Returns (rc, stats dict)."""
    op = U.c_struct()
    st = lj_stats()
    rc = ctx._lib.lj_user_phi_action(ctx.handle, C.byref(op), _tensor_ptr(v, U.n, "v"), _tensor_ptr(w, U.n, "w"),
                                     int(l), float(h), float(tol), C.byref(opt) if opt is not None else None,
                                     C.byref(st), _stream_ptr(stream))
    _user_call(ctx, U, rc)
    return rc, st.as_dict(1)


def lj_user_phi_vertical(ctx: Context, U: UserOperator, v, ls: Sequence[int], As: Sequence[float], h: float,
                         tol: float, ws: Sequence, opt: lj_options | None = None, stream=None):
    K = len(ls)
    if len(As) != K or len(ws) != K:
        raise ValueError("ls, As and ws must have the same length")
    op = U.c_struct()
    st = lj_stats()
    larr = (C.c_int * K)(*[int(x) for x in ls])
    aarr = (C.c_double * K)(*[float(x) for x in As])
    warr = (C.c_void_p * K)(*[_tensor_ptr(w, U.n, f"w[{k}]").value for k, w in enumerate(ws)])
    rc = ctx._lib.lj_user_phi_vertical(ctx.handle, C.byref(op), _tensor_ptr(v, U.n, "v"), K, larr, aarr,
                                       float(h), float(tol), warr, C.byref(opt) if opt is not None else None,
                                       C.byref(st), _stream_ptr(stream))
    _user_call(ctx, U, rc)
    return rc, st.as_dict(K)


def lj_user_step(ctx: Context, scheme: str, U: UserOperator, h: float, tol: float, u_out, err=None,
                 opt: lj_options | None = None, stream=None):
    """One exponential-integrator step from U.state.  Returns (rc, list of stats dicts)."""
    op = U.c_struct()
    stats = (lj_stats * 4)()
    ncalls = C.c_int()
    rc = ctx._lib.lj_user_step(ctx.handle, SCHEMES[scheme], C.byref(op), float(h), float(tol),
                               _tensor_ptr(u_out, U.n, "u_out"),
                               _tensor_ptr(err, U.n, "err") if err is not None else None,
                               C.byref(opt) if opt is not None else None, stats, 4, C.byref(ncalls),
                               _stream_ptr(stream))
    _user_call(ctx, U, rc)
    return rc, [stats[i].as_dict() for i in range(ncalls.value)]


def lj_measure_bandwidth(nbytes: int = 1 << 30) -> dict:
    """Attainable HBM bandwidth (GB/s) of the current device: copy, read-only
    and the Newton-step access pattern (3 reads + 2 writes)."""
    out = (C.c_double * 3)()
    rc = lib().lj_measure_bandwidth(int(nbytes), out)
    if rc != LJ_OK:
        raise LejaError(rc, "lj_measure_bandwidth")
    return {"copy": out[0], "read": out[1], "newton_step": out[2]}


def lj_measure_bandwidth_shape(nbytes: int, blocks: int, threads: int, unroll: int = 1,
                               nontemporal: bool = False) -> dict:
    """The same patterns at a chosen launch shape, accesses in flight per
    thread and load/store flavour (non-temporal or ordinary)."""
    out = (C.c_double * 3)()
    rc = lib().lj_measure_bandwidth_shape(int(nbytes), int(blocks), int(threads), int(unroll),
                                          1 if nontemporal else 0, out)
    if rc != LJ_OK:
        raise LejaError(rc, "lj_measure_bandwidth_shape")
    return {"copy": out[0], "read": out[1], "newton_step": out[2]}


def lj_default_krylov_options(**overrides) -> "_lib.lj_krylov_options":
    k = _lib.lj_krylov_options()
    lib().lj_default_krylov_options(C.byref(k))
    for name, val in overrides.items():
        setattr(k, name, val)
    return k


def _bvec(bs, n):
    arr = (C.c_void_p * len(bs))()
    for j, b in enumerate(bs):
        arr[j] = None if b is None else _tensor_ptr(b, n, f"b[{j}]").value
    return arr


def lj_phi_combination(ctx: Context, J: Operator, bs: Sequence, h: float, tol: float, w, kopt=None, stream=None):
    """w = sum_j phi_j(h J) b_j h^j (bs = [b_0, ..., b_p], None = zero) by Krylov.
    Returns (rc, stats dict)."""
    op = J.c_struct()
    st = lj_stats()
    rc = ctx._lib.lj_phi_combination(ctx.handle, C.byref(op), len(bs) - 1, _bvec(bs, J.n), float(h), float(tol),
                                     _tensor_ptr(w, J.n, "w"), C.byref(kopt) if kopt is not None else None,
                                     C.byref(st), _stream_ptr(stream))
    ctx._check(rc)
    return rc, st.as_dict(1)


def lj_user_phi_combination(ctx: Context, U: "UserOperator", bs: Sequence, h: float, tol: float, w, kopt=None,
                            stream=None):
    op = U.c_struct()
    st = lj_stats()
    rc = ctx._lib.lj_user_phi_combination(ctx.handle, C.byref(op), len(bs) - 1, _bvec(bs, U.n), float(h),
                                          float(tol), _tensor_ptr(w, U.n, "w"),
                                          C.byref(kopt) if kopt is not None else None, C.byref(st),
                                          _stream_ptr(stream))
    _user_call(ctx, U, rc)
    return rc, st.as_dict(1)


def lj_user_integrate(ctx: Context, scheme: str, U: UserOperator, T: float, dt0: float, tol: float,
                      leja_tol: float, u_out, opt: lj_options | None = None, log_cap: int = 1000,
                      max_attempts: int = 100000, stream=None):
    """u(T) from u(0) = U.state with variable steps (Sec. 2.3) for a user
    operator.  Returns (rc, stats dict, list of attempted steps)."""
    op = U.c_struct()
    st = lj_integrate_stats()
    recs = (lj_step_record * max(log_cap, 1))()
    rc = ctx._lib.lj_user_integrate(ctx.handle, SCHEMES[scheme], C.byref(op), float(T), float(dt0), float(tol),
                                    float(leja_tol), _tensor_ptr(u_out, U.n, "u_out"),
                                    C.byref(opt) if opt is not None else None, C.byref(st), recs, int(log_cap),
                                    int(max_attempts), _stream_ptr(stream))
    _user_call(ctx, U, rc)
    n = min(st.accepted + st.rejected, log_cap)
    return rc, st.as_dict(), [recs[i].as_dict() for i in range(n)]


def family_user_operator(ctx: Context, J: Operator, finite_difference: bool = False) -> UserOperator:
    """A built-in family seen as a user operator (its lj_rhs and lj_jv as the
    callbacks), e.g. to check the callback path against the fused one."""
    def rhs(x, out):
        lj_rhs(ctx, J, x, out)

    def jv(u, x, out):
        lj_jv(ctx, J, x, out)

    return UserOperator(J.n, J.state, rhs=rhs, jv=None if finite_difference else jv)


def lj_phi_action(ctx: Context, J: Operator, v, w, l: int, h: float, tol: float, opt: lj_options | None = None,
                  stream=None):
    """w = phi_l(h J) v.  Returns (return code, stats dict)."""
    op = J.c_struct()
    st = lj_stats()
    rc = ctx._lib.lj_phi_action(ctx.handle, C.byref(op), _tensor_ptr(v, J.n, "v"), _tensor_ptr(w, J.n, "w"),
                                int(l), float(h), float(tol), C.byref(opt) if opt is not None else None,
                                C.byref(st), _stream_ptr(stream))
    ctx._check(rc)
    return rc, st.as_dict(1)


def lj_phi_action_noalloc(ctx: Context, J: Operator, v, w, l: int, h: float, tol: float,
                          opt: lj_options | None = None, stream=None):
    """lj_phi_action without device allocation: the workspace lies in the
    library's per-device scratch array.  Returns (return code, stats dict)."""
    op = J.c_struct()
    st = lj_stats()
    rc = ctx._lib.lj_phi_action_noalloc(ctx.handle, C.byref(op), _tensor_ptr(v, J.n, "v"),
                                        _tensor_ptr(w, J.n, "w"), int(l), float(h), float(tol),
                                        C.byref(opt) if opt is not None else None, C.byref(st),
                                        _stream_ptr(stream))
    ctx._check(rc)
    return rc, st.as_dict(1)


def lj_phi_vertical(ctx: Context, J: Operator, v, ls: Sequence[int], As: Sequence[float], h: float, tol: float,
                    ws: Sequence, opt: lj_options | None = None, stream=None):
    """w[k] = phi_{l[k]}(a[k] h J) v on one Newton basis.  Returns (rc, stats dict)."""
    K = len(ls)
    if len(As) != K or len(ws) != K:
        raise ValueError("ls, As and ws must have the same length")
    op = J.c_struct()
    st = lj_stats()
    larr = (C.c_int * K)(*[int(x) for x in ls])
    aarr = (C.c_double * K)(*[float(x) for x in As])
    warr = (C.c_void_p * K)(*[_tensor_ptr(w, J.n, f"w[{k}]").value for k, w in enumerate(ws)])
    rc = ctx._lib.lj_phi_vertical(ctx.handle, C.byref(op), _tensor_ptr(v, J.n, "v"), K, larr, aarr, float(h),
                                  float(tol), warr, C.byref(opt) if opt is not None else None, C.byref(st),
                                  _stream_ptr(stream))
    ctx._check(rc)
    return rc, st.as_dict(K)


def lj_step(ctx: Context, scheme: str, J: Operator, h: float, tol: float, u_out, err=None,
            opt: lj_options | None = None, stream=None):
    """One exponential-integrator step from J.state.  Returns (rc, list of stats dicts)."""
    op = J.c_struct()
    stats = (lj_stats * 4)()
    ncalls = C.c_int()
    rc = ctx._lib.lj_step(ctx.handle, SCHEMES[scheme], C.byref(op), float(h), float(tol),
                          _tensor_ptr(u_out, J.n, "u_out"),
                          _tensor_ptr(err, J.n, "err") if err is not None else None,
                          C.byref(opt) if opt is not None else None, stats, 4, C.byref(ncalls),
                          _stream_ptr(stream))
    ctx._check(rc)
    return rc, [stats[i].as_dict() for i in range(ncalls.value)]


def lj_bound_device(ctx: Context) -> int:
    """Device address of the bound the last lj_step left for its actions."""
    return ctx._lib.lj_bound_device(ctx.handle) or 0


class Deferred:
    """Deferred synchronisation (lj_defer_begin / lj_defer_end): steps and
    actions issued through it are only enqueued; leaving the with-block
    synchronises once (lj_defer_end) and fills `results`, one (rc, stats) per
    call in the form lj_step / lj_phi_action return.  Inputs of the calls must
    not be overwritten by later calls of the same block."""

    def __init__(self, ctx: Context, stream=None):
        self.ctx = ctx
        self.stream = stream
        self._calls = []  # (kind, stats array, count) plus the objects the library points at
        self.results = None
        self.rc = None

    def __enter__(self):
        self.ctx._check(self.ctx._lib.lj_defer_begin(self.ctx.handle), False)
        return self

    def step(self, scheme: str, J: Operator, h: float, tol: float, u_out, err=None, opt: lj_options | None = None):
        op = J.c_struct()
        stats = (lj_stats * 4)()
        ncalls = C.c_int()
        rc = self.ctx._lib.lj_step(self.ctx.handle, SCHEMES[scheme], C.byref(op), float(h), float(tol),
                                   _tensor_ptr(u_out, J.n, "u_out"),
                                   _tensor_ptr(err, J.n, "err") if err is not None else None,
                                   C.byref(opt) if opt is not None else None, stats, 4, C.byref(ncalls),
                                   _stream_ptr(self.stream))
        self.ctx._check(rc)
        self._calls.append(("step", stats, ncalls, (op, opt, J, u_out, err)))
        return len(self._calls) - 1

    def phi_action(self, J: Operator, v, w, l: int, h: float, tol: float, opt: lj_options | None = None):
        op = J.c_struct()
        st = lj_stats()
        rc = self.ctx._lib.lj_phi_action(self.ctx.handle, C.byref(op), _tensor_ptr(v, J.n, "v"),
                                         _tensor_ptr(w, J.n, "w"), int(l), float(h), float(tol),
                                         C.byref(opt) if opt is not None else None, C.byref(st),
                                         _stream_ptr(self.stream))
        self.ctx._check(rc)
        self._calls.append(("action", st, None, (op, opt, J, v, w)))
        return len(self._calls) - 1

    def __exit__(self, et, ev, tb):
        rc = self.ctx._lib.lj_defer_end(self.ctx.handle, _stream_ptr(self.stream))
        self.rc = rc
        if et is None:
            self.ctx._check(rc)
        self.results = []
        for kind, st, count, _ in self._calls:
            if kind == "step":
                self.results.append((rc, [st[i].as_dict() for i in range(count.value)]))
            else:
                self.results.append((rc, st.as_dict(1)))
        return False


def lj_integrate(ctx: Context, scheme: str, J: Operator, T: float, dt0: float, tol: float, leja_tol: float, u_out,
                 opt: lj_options | None = None, log_cap: int = 1000, max_attempts: int = 100000, stream=None):
    """u(T) from u(0) = J.state with variable steps (Sec. 2.3).  Returns
    (rc, stats dict, list of attempted steps)."""
    st = lj_integrate_stats()
    recs = (lj_step_record * max(log_cap, 1))()
    rc = ctx._lib.lj_integrate(ctx.handle, SCHEMES[scheme], C.byref(J.c_struct()), float(T), float(dt0), float(tol),
                               float(leja_tol), _tensor_ptr(u_out, J.n, "u_out"),
                               C.byref(opt) if opt is not None else None, C.byref(st), recs, int(log_cap),
                               int(max_attempts), _stream_ptr(stream))
    ctx._check(rc)
    n = min(st.accepted + st.rejected, log_cap)
    return rc, st.as_dict(), [recs[i].as_dict() for i in range(n)]


def lj_last_trace(ctx: Context, rows: int = 100):
    """Per-iteration device totals of the last Newton recurrence: a list of
    rows [||y_m||^2, ||p_0||^2, ..., ||p_3||^2] for m = 1..iterations."""
    buf = (C.c_double * (rows * (1 + LJ_MAX_K)))()
    n = ctx._lib.lj_last_trace(ctx.handle, buf, int(rows))
    if n < 0:
        raise LejaError(n, "lj_last_trace")
    return [list(buf[i * (1 + LJ_MAX_K):(i + 1) * (1 + LJ_MAX_K)]) for i in range(n)]


PROFILE_PHASES = ("power", "divdiff", "steps", "publish", "barrier", "decide", "commit", "halo")


def lj_last_profile(ctx: Context) -> dict:
    """Microseconds block 0 of the last action launch spent per phase."""
    buf = (C.c_double * 8)()
    ctx._check(ctx._lib.lj_last_profile(ctx.handle, buf), False)
    return dict(zip(PROFILE_PHASES, list(buf)))


def lj_timing_enable(ctx: Context, enable: bool = True) -> None:
    ctx._check(ctx._lib.lj_timing_enable(ctx.handle, 1 if enable else 0), False)


def lj_timing_read(ctx: Context, reset: bool = False) -> dict:
    t = lj_timing()
    ctx._check(ctx._lib.lj_timing_read(ctx.handle, C.byref(t), 1 if reset else 0), False)
    return {f: getattr(t, f) for f, _ in t._fields_}


class Batch:
    """A batch of independent instances run in one persistent, graph-captured
    launch (lj_batch_*).  Keeps the operators, inputs and outputs alive."""

    def __init__(self, ctx: Context, ops: Sequence[Operator], vs: Sequence, hs: Sequence[float],
                 ls: Sequence[int], As: Sequence[float], tol: float, ws: Sequence[Sequence],
                 bounds: Sequence[float] | None = None, opt: lj_options | None = None):
        n, K = len(ops), len(ls)
        if len(vs) != n or len(hs) != n or len(ws) != n or len(As) != K:
            raise ValueError("ops, vs, hs and ws need n entries; ls and As K entries")
        self.ctx, self.n, self.K = ctx, n, K
        self._keep = (list(ops), list(vs), [list(w) for w in ws])
        self._ops = (lj_operator * n)(*[J.c_struct() for J in ops])
        vp = (C.c_void_p * n)(*[_tensor_ptr(v, J.n, f"v[{i}]").value for i, (J, v) in enumerate(zip(ops, vs))])
        wp = (C.c_void_p * (n * K))()
        for i, (J, wi) in enumerate(zip(ops, ws)):
            if len(wi) != K:
                raise ValueError(f"ws[{i}] needs {K} tensors")
            for k, w in enumerate(wi):
                wp[i * K + k] = _tensor_ptr(w, J.n, f"w[{i}][{k}]").value
        harr = (C.c_double * n)(*[float(x) for x in hs])
        larr = (C.c_int * K)(*[int(x) for x in ls])
        aarr = (C.c_double * K)(*[float(x) for x in As])
        barr = (C.c_double * n)(*[float(x) for x in bounds]) if bounds is not None else None
        h = C.c_void_p()
        rc = ctx._lib.lj_batch_create(ctx.handle, self._ops, n, vp, harr, K, larr, aarr, float(tol), wp, barr,
                                      C.byref(opt) if opt is not None else None, C.byref(h))
        ctx._check(rc, False)
        self.handle = h

    def run(self, stream=None) -> None:
        self.ctx._check(self.ctx._lib.lj_batch_run(self.handle, _stream_ptr(stream)), False)

    def stats(self, stream=None):
        """Synchronises, returns (rc, per-instance stats dicts); accumulators
        the shared basis rejected were substepped inside the launch."""
        st = (lj_stats * self.n)()
        rc = self.ctx._lib.lj_batch_stats(self.handle, st, _stream_ptr(stream))
        self.ctx._check(rc)
        return rc, [st[i].as_dict(self.K) for i in range(self.n)]

    def info(self) -> dict:
        i = _lib.lj_batch_info_t()
        self.ctx._check(self.ctx._lib.lj_batch_info(self.handle, C.byref(i)), False)
        d = {f: getattr(i, f) for f, _ in i._fields_ if f != "tune_ms"}
        d["tune_ms"] = list(i.tune_ms)[:i.nschedules]
        return d

    def timeline(self):
        """(block, start_us, end_us) per instance of the run last read by stats()."""
        blk = (C.c_int * self.n)()
        t0 = (C.c_double * self.n)()
        t1 = (C.c_double * self.n)()
        self.ctx._check(self.ctx._lib.lj_batch_timeline(self.handle, blk, t0, t1), False)
        return list(blk), list(t0), list(t1)

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.ctx._lib.lj_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lj_batch_create(ctx: Context, ops, vs, hs, ls, As, tol, ws, bounds=None, opt=None) -> Batch:
    return Batch(ctx, ops, vs, hs, ls, As, tol, ws, bounds, opt)


# ---- learned proposal -------------------------------------------------------
def _ftensor_ptr(t, n: int, what: str) -> C.c_void_p:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous float32 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} entries, expected {n}")
    return C.c_void_p(t.data_ptr())


def lj_features(ctx: Context, J: Operator, h: float, l: int, feats, stream=None) -> None:
    """feats (float32 CUDA tensor of 16) = features of phi_l(h J) v."""
    op = J.c_struct()
    ctx._check(ctx._lib.lj_features(ctx.handle, C.byref(op), float(h), int(l),
                                    _ftensor_ptr(feats, _lib.LJ_NFEATURES, "feats"), _stream_ptr(stream)), False)


def lj_gershgorin_bound(ctx: Context, J: Operator, stream=None) -> float:
    """The Gershgorin bound of J at its state (largest absolute row sum)."""
    op = J.c_struct()
    out = C.c_double(0.0)
    ctx._check(ctx._lib.lj_gershgorin_bound(ctx.handle, C.byref(op), C.byref(out), _stream_ptr(stream)), False)
    return out.value


def lj_proposal_record(ctx: Context, J: Operator, h: float, l: int, bound: float, substeps: int, feats, targets,
                       stream=None) -> None:
    """feats (float32 CUDA tensor of 16) and targets (of 2) of one training
    record: the features of phi_l(h J) v, ln(bound / G), log2(substeps)."""
    op = J.c_struct()
    ctx._check(ctx._lib.lj_proposal_record(ctx.handle, C.byref(op), float(h), int(l), float(bound), int(substeps),
                                           _ftensor_ptr(feats, _lib.LJ_NFEATURES, "feats"),
                                           _ftensor_ptr(targets, 2, "targets"), _stream_ptr(stream)), False)


def lj_mlp_init(ctx: Context, seed: int = 6) -> None:
    ctx._check(ctx._lib.lj_mlp_init(ctx.handle, C.c_uint64(seed)), False)


def lj_mlp_train(ctx: Context, feats, targets, epochs: int, batch: int = 256, lr: float = 1e-3,
                 fit_normalization: bool = True, stream=None):
    """Trains on (feats n x 16, targets n x 2) float32 CUDA tensors; returns the per-epoch losses."""
    n = feats.shape[0]
    losses = (C.c_float * epochs)()
    ctx._check(ctx._lib.lj_mlp_train(ctx.handle, _ftensor_ptr(feats, n * 16, "feats"),
                                     _ftensor_ptr(targets, n * 2, "targets"), int(n), int(epochs), int(batch),
                                     float(lr), 1 if fit_normalization else 0, losses, _stream_ptr(stream)), False)
    return list(losses)


def lj_mlp_predict(ctx: Context, feats, out, stream=None) -> None:
    n = feats.shape[0]
    ctx._check(ctx._lib.lj_mlp_predict(ctx.handle, _ftensor_ptr(feats, n * 16, "feats"), int(n),
                                       _ftensor_ptr(out, n * 2, "out"), _stream_ptr(stream)), False)


def lj_mlp_grad(ctx: Context, feats, targets, grad, stream=None) -> float:
    n = feats.shape[0]
    loss = C.c_float()
    ctx._check(ctx._lib.lj_mlp_grad(ctx.handle, _ftensor_ptr(feats, n * 16, "feats"),
                                    _ftensor_ptr(targets, n * 2, "targets"), int(n),
                                    _ftensor_ptr(grad, _lib.LJ_MLP_NPARAM, "grad"), C.byref(loss),
                                    _stream_ptr(stream)), False)
    return loss.value


def lj_mlp_get(ctx: Context):
    buf = (C.c_float * _lib.LJ_MLP_MODEL_FLOATS)()
    ctx._check(ctx._lib.lj_mlp_get(ctx.handle, buf), False)
    return list(buf)


def lj_mlp_set(ctx: Context, model) -> None:
    buf = (C.c_float * _lib.LJ_MLP_MODEL_FLOATS)(*[float(x) for x in model])
    ctx._check(ctx._lib.lj_mlp_set(ctx.handle, buf), False)


def lj_mlp_save(ctx: Context, path: str) -> None:
    ctx._check(ctx._lib.lj_mlp_save(ctx.handle, str(path).encode()), False)


def lj_mlp_load(ctx: Context, path: str) -> None:
    ctx._check(ctx._lib.lj_mlp_load(ctx.handle, str(path).encode()), False)


def operator_from(prob, device: str = "cuda") -> Operator:
    """Operator for any object with kind, nx, ny, ncomp, dx, dy, coef and a
    numpy `state` (or None); the state is copied to a float64 device tensor."""
    import torch
    st = None
    if prob.state is not None:
        st = torch.as_tensor(prob.state, dtype=torch.float64).to(device).contiguous()
    return Operator(prob.kind, int(prob.nx), int(prob.ny), int(prob.ncomp), float(prob.dx), float(prob.dy),
                    tuple(float(c) for c in prob.coef), st)

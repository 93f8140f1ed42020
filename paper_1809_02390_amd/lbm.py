"""Thin Python binding of the C ABI in ``include/lbm.h`` (ctypes).

Every function here has the name of the C entry point it calls and only
marshals arguments: torch tensors become device pointers, the stream comes
from torch, status codes become ``LbmError``.  All arithmetic happens in the
HIP library.  ``Lattice`` bundles the buffers and the context for callers
that want torch to own the memory.
"""
from __future__ import annotations

import ctypes
import functools
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOCOEX, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_FP32, LBM_FP16, LBM_BF16 = 0, 1, 2
STORAGE = {"fp32": LBM_FP32, "fp16": LBM_FP16, "bf16": LBM_BF16}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lbm status {status}: {message}")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("s_p", ctypes.c_double), ("s_eps", ctypes.c_double),
                ("varpi", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("r_gas", ctypes.c_double), ("tr", ctypes.c_double), ("sigma", ctypes.c_double),
                ("width", ctypes.c_double)]


class lbm_derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "rho_g", "rho_l", "p0", "c_sigma", "c_w", "sigma", "width", "k_int", "k_eos", "g2", "kp", "rt",
        "alpha2", "beta2", "k", "h", "bs", "s_p", "s_q", "s_e", "s_eps", "tc")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"HIP library {_LIB_PATH} is missing: build it with "
                          "`python paper_1809_02390_amd/build.py` (there is no CPU fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    P, V, I, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_derive": (I, [P(lbm_params), P(lbm_derived)]),
        "lbm_sigma_paper": (I, [D, D, D, D, D, P(D)]),
        "lbm_state_bytes": (ctypes.c_size_t, [P(lbm_params)]),
        "lbm_ref_bytes": (ctypes.c_size_t, [P(lbm_params)]),
        "lbm_create": (I, [P(V), P(lbm_params), V, V, V, V]),
        "lbm_set_stream": (I, [V, V]),
        "lbm_init": (I, [V, V, V, V]),
        "lbm_set_state": (I, [V, V]),
        "lbm_get_state": (I, [V, V]),
        "lbm_step": (I, [V, ctypes.c_int32]),
        "lbm_moments": (I, [V, V, V, V, P(D)]),
        "lbm_moments_noalloc": (I, [V, V, V, V, V]),
        "lbm_checkpoint_bytes": (ctypes.c_size_t, [P(lbm_params)]),
        "lbm_save_state": (I, [V, V]),
        "lbm_load_state": (I, [V, V, ctypes.c_int64]),
        "lbm_step_saved": (I, [V, V, V]),
        "lbm_step_saved_chain": (I, [V, P(V), ctypes.c_int32]),
        "lbm_adjoint_run": (I, [V, P(V), ctypes.c_int32, V, V, P(ctypes.c_int32)]),
        "lbm_adjoint_bytes": (ctypes.c_size_t, [P(lbm_params)]),
        "lbm_adjoint_seed": (I, [V, V, V]),
        "lbm_adjoint_step": (I, [V, V, V, V]),
        "lbm_adjoint_get": (I, [V, V, V]),
        "lbm_adjoint_init": (I, [V, V, V, V, V, V]),
        "lbm_adjoint_theta": (I, [V, P(D), ctypes.c_int32]),
        "lbm_adjoint_params": (I, [V, P(D), P(D), ctypes.c_int32]),
        "lbm_param_jacobian": (I, [P(lbm_params), P(D)]),
        "lbm_time": (ctypes.c_int64, [V]),
        "lbm_get_derived": (I, [V, P(lbm_derived)]),
        "lbm_destroy": (None, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("lbm_last_error", "lbm_derive", "lbm_sigma_paper", "lbm_state_bytes", "lbm_ref_bytes",
            "lbm_create", "lbm_set_stream", "lbm_init", "lbm_set_state", "lbm_get_state", "lbm_step",
            "lbm_moments", "lbm_moments_noalloc", "lbm_checkpoint_bytes", "lbm_save_state", "lbm_load_state", "lbm_step_saved", "lbm_step_saved_chain", "lbm_adjoint_run",
            "lbm_adjoint_bytes", "lbm_adjoint_seed", "lbm_adjoint_step", "lbm_adjoint_get", "lbm_adjoint_init",
            "lbm_adjoint_theta", "lbm_adjoint_params", "lbm_param_jacobian", "lbm_time", "lbm_get_derived", "lbm_destroy")


def _check(status: int):
    if status != LBM_OK:
        raise LbmError(status, _lib.lbm_last_error().decode())


def make_params(nx, ny, *, storage="fp32", s_p=1.0, s_eps=0.0, varpi=1.0 / 6.0, a=1.0, b=4.0,
                r_gas=1.0, tr=0.8, sigma=0.0, width=10.0) -> lbm_params:
    """lbm_params from keyword arguments (sigma <= 0: the paper's sound-speed rule;
    s_eps <= 0: s_e)."""
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    return lbm_params(int(nx), int(ny), st, 0, float(s_p), float(s_eps), float(varpi), float(a), float(b),
                      float(r_gas), float(tr), float(sigma), float(width))


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# Functions named after the C entry points
# ---------------------------------------------------------------------------
def lbm_last_error() -> str:
    return _lib.lbm_last_error().decode()


def lbm_derive(params: lbm_params) -> lbm_derived:
    out = lbm_derived()
    _check(_lib.lbm_derive(ctypes.byref(params), ctypes.byref(out)))
    return out


def lbm_sigma_paper(width, tr, a=1.0, b=4.0, r_gas=1.0) -> float:
    s = ctypes.c_double()
    _check(_lib.lbm_sigma_paper(width, tr, a, b, r_gas, ctypes.byref(s)))
    return s.value


def lbm_state_bytes(params: lbm_params) -> int:
    return _lib.lbm_state_bytes(ctypes.byref(params))


def lbm_ref_bytes(params: lbm_params) -> int:
    return _lib.lbm_ref_bytes(ctypes.byref(params))


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def lbm_create(params: lbm_params, f_a, f_b, rho_ref=None, stream=None):
    nbytes = lbm_state_bytes(params)
    for t, nm in ((f_a, "f_a"), (f_b, "f_b")):
        if t is None or t.numel() * t.element_size() < nbytes:
            raise ValueError(f"{nm} must hold at least {nbytes} bytes")
    ctx = ctypes.c_void_p()
    _check(_lib.lbm_create(ctypes.byref(ctx), ctypes.byref(params), _ptr(f_a, name="f_a"),
                           _ptr(f_b, name="f_b"), _ptr(rho_ref, name="rho_ref"), _stream_handle(stream)))
    return ctx


def lbm_set_stream(ctx, stream=None):
    _check(_lib.lbm_set_stream(ctx, _stream_handle(stream)))


def lbm_init(ctx, rho0, ux0=None, uy0=None, n=None):
    _check(_lib.lbm_init(ctx, _ptr(rho0, torch.float32, n, "rho0"), _ptr(ux0, torch.float32, n, "ux0"),
                         _ptr(uy0, torch.float32, n, "uy0")))


def lbm_set_state(ctx, f, n=None):
    _check(_lib.lbm_set_state(ctx, _ptr(f, torch.float32, None if n is None else 9 * n, "f")))


def lbm_get_state(ctx, f, n=None):
    _check(_lib.lbm_get_state(ctx, _ptr(f, torch.float32, None if n is None else 9 * n, "f")))


def lbm_step(ctx, n: int):
    _check(_lib.lbm_step(ctx, int(n)))


def lbm_moments(ctx, rho=None, ux=None, uy=None, totals=True, n=None):
    tot = (ctypes.c_double * 3)()
    _check(_lib.lbm_moments(ctx, _ptr(rho, torch.float32, n, "rho"), _ptr(ux, torch.float32, n, "ux"),
                            _ptr(uy, torch.float32, n, "uy"), tot if totals else None))
    return tuple(tot) if totals else None


def lbm_moments_noalloc(ctx, rho=None, ux=None, uy=None, totals_dev=None, n=None):
    """lbm_moments without allocation or synchronisation: totals_dev, if given,
    is a device float64 tensor of 3 elements written on the stream."""
    _check(_lib.lbm_moments_noalloc(ctx, _ptr(rho, torch.float32, n, "rho"), _ptr(ux, torch.float32, n, "ux"),
                                    _ptr(uy, torch.float32, n, "uy"), _ptr(totals_dev, torch.float64, 3, "totals_dev")))


def lbm_checkpoint_bytes(params: lbm_params) -> int:
    return _lib.lbm_checkpoint_bytes(ctypes.byref(params))


def _bytes_ptr(t, nbytes, name):
    p = _ptr(t, name=name)
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} must hold at least {nbytes} bytes")
    return p


def lbm_save_state(ctx, dst, nbytes):
    _check(_lib.lbm_save_state(ctx, _bytes_ptr(dst, nbytes, "dst")))


def lbm_load_state(ctx, src, t, nbytes):
    _check(_lib.lbm_load_state(ctx, _bytes_ptr(src, nbytes, "src"), int(t)))


def lbm_step_saved(ctx, src, dst, nbytes):
    _check(_lib.lbm_step_saved(ctx, _bytes_ptr(src, nbytes, "src"), _bytes_ptr(dst, nbytes, "dst")))


def _ptr_array(ts, nbytes, name):
    arr = (ctypes.c_void_p * len(ts))()
    for j, t in enumerate(ts):
        arr[j] = _bytes_ptr(t, nbytes, f"{name}[{j}]")
    return arr


def lbm_step_saved_chain(ctx, bufs, nbytes):
    """bufs[j+1] := step(bufs[j]) for j < len(bufs) - 1."""
    if len(bufs) < 2:
        return
    _check(_lib.lbm_step_saved_chain(ctx, _ptr_array(bufs, nbytes, "bufs"), len(bufs) - 1))


def lbm_adjoint_run(ctx, f_states, adj_a, adj_b, state_bytes, adj_bytes):
    """Adjoint steps back through f_states; returns 0 or 1: which of adj_a,
    adj_b holds the result."""
    which = ctypes.c_int32(-1)
    arr = _ptr_array(f_states, state_bytes, "f_states")
    _check(_lib.lbm_adjoint_run(ctx, arr, len(f_states), _bytes_ptr(adj_a, adj_bytes, "adj_a"),
                                _bytes_ptr(adj_b, adj_bytes, "adj_b"), ctypes.byref(which)))
    return which.value


def lbm_adjoint_bytes(params: lbm_params) -> int:
    return _lib.lbm_adjoint_bytes(ctypes.byref(params))


def lbm_adjoint_seed(ctx, lam, adj, n, adj_bytes):
    _check(_lib.lbm_adjoint_seed(ctx, _ptr(lam, torch.float32, 9 * n, "lam"), _bytes_ptr(adj, adj_bytes, "adj")))


def lbm_adjoint_step(ctx, f_t, adj_next, adj_out, state_bytes, adj_bytes):
    _check(_lib.lbm_adjoint_step(ctx, _bytes_ptr(f_t, state_bytes, "f_t"), _bytes_ptr(adj_next, adj_bytes, "adj_next"),
                                 _bytes_ptr(adj_out, adj_bytes, "adj_out")))


def lbm_adjoint_get(ctx, adj, lam, n, adj_bytes):
    _check(_lib.lbm_adjoint_get(ctx, _bytes_ptr(adj, adj_bytes, "adj"), _ptr(lam, torch.float32, 9 * n, "lam")))


def lbm_adjoint_init(ctx, rho0, ux0, uy0, adj0, drho0, n, adj_bytes):
    _check(_lib.lbm_adjoint_init(ctx, _ptr(rho0, torch.float32, n, "rho0"), _ptr(ux0, torch.float32, n, "ux0"),
                                 _ptr(uy0, torch.float32, n, "uy0"), _bytes_ptr(adj0, adj_bytes, "adj0"),
                                 _ptr(drho0, torch.float32, n, "drho0")))


def lbm_adjoint_theta(ctx, read=True, reset=True):
    out = (ctypes.c_double * 3)()
    _check(_lib.lbm_adjoint_theta(ctx, out if read else None, 1 if reset else 0))
    return tuple(out) if read else None


def lbm_adjoint_params(ctx, reset=True):
    """(dL/d(sigma, W, T_r), dL/d theta) of the accumulated adjoint, each a
    3-tuple; the chain rule is applied by the library."""
    dp, dth = (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    _check(_lib.lbm_adjoint_params(ctx, dp, dth, 1 if reset else 0))
    return tuple(dp), tuple(dth)


def lbm_param_jacobian(params: lbm_params):
    """d(G'^2, K', RT)/d(sigma, W, T_r) as a 3 x 3 nested list (rows: theta)."""
    out = (ctypes.c_double * 9)()
    _check(_lib.lbm_param_jacobian(ctypes.byref(params), out))
    return [list(out[3 * k:3 * k + 3]) for k in range(3)]


def lbm_time(ctx) -> int:
    return int(_lib.lbm_time(ctx))


def lbm_get_derived(ctx) -> lbm_derived:
    out = lbm_derived()
    _check(_lib.lbm_get_derived(ctx, ctypes.byref(out)))
    return out


def lbm_destroy(ctx):
    _lib.lbm_destroy(ctx)


# ---------------------------------------------------------------------------
# Convenience owner of buffers + context
# ---------------------------------------------------------------------------
def _ordered(method):
    """Run a Lattice method with its context stream ordered after torch's
    current stream (the caller's earlier work on the tensors it passes) and
    torch's current stream ordered after the context stream (the caller's
    later use of results, and the caching allocator's reuse of tensors the
    library still reads or writes).  Nothing to do when they are the same."""
    @functools.wraps(method)
    def run(self, *args, **kw):
        cur = torch.cuda.current_stream(self.f_a.device)
        if cur == self.stream:
            return method(self, *args, **kw)
        self.stream.wait_stream(cur)
        try:
            return method(self, *args, **kw)
        finally:
            cur.wait_stream(self.stream)
    return run


class Lattice:
    """Torch-owned A/B buffers plus a library context on the current device.

    The context launches on `stream` (torch's current stream at creation if
    None); every method orders that stream with torch's current stream at
    the call, so tensors passed in and returned follow torch's stream
    semantics."""

    def __init__(self, nx, ny, device="cuda", stream=None, **kw):
        self.params = make_params(nx, ny, **kw)
        self.nx, self.ny, self.n = nx, ny, nx * ny
        nbytes = lbm_state_bytes(self.params)
        if nbytes == 0:
            lbm_derive(self.params)  # raises with the validation message
        self.f_a = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.f_b = torch.empty(nbytes, dtype=torch.uint8, device=device)
        rb = lbm_ref_bytes(self.params)
        self.rho_ref = torch.empty(rb, dtype=torch.uint8, device=device) if rb else None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.f_a.device)
        if stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.f_a.device))  # buffers allocated above
        self.ctx = lbm_create(self.params, self.f_a, self.f_b, self.rho_ref, self.stream)
        self.derived = lbm_get_derived(self.ctx)

    @_ordered
    def init(self, rho0, ux0=None, uy0=None):
        dev = self.f_a.device
        conv = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float32).to(dev).contiguous()
        self._keep = [conv(rho0), conv(ux0), conv(uy0)]
        lbm_init(self.ctx, *self._keep, n=self.n)
        return self

    @_ordered
    def set_state(self, f):
        f = torch.as_tensor(f, dtype=torch.float32).to(self.f_a.device).contiguous()
        lbm_set_state(self.ctx, f, n=self.n)
        self._keep = [f]
        return self

    @_ordered
    def state(self):
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float32, device=self.f_a.device)
        lbm_get_state(self.ctx, f, n=self.n)
        return f

    @_ordered
    def step(self, n=1):
        lbm_step(self.ctx, n)
        return self

    @_ordered
    def moments(self, fields=True):
        dev = self.f_a.device
        if fields:
            rho, ux, uy = (torch.empty((self.ny, self.nx), dtype=torch.float32, device=dev) for _ in range(3))
            tot = lbm_moments(self.ctx, rho, ux, uy, True, n=self.n)
            return rho, ux, uy, tot
        return lbm_moments(self.ctx, None, None, None, True, n=self.n)

    # ---- checkpoints -------------------------------------------------------
    def checkpoint_buffer(self):
        return torch.empty(lbm_checkpoint_bytes(self.params), dtype=torch.uint8, device=self.f_a.device)

    @_ordered
    def save_state(self, dst=None):
        dst = self.checkpoint_buffer() if dst is None else dst
        lbm_save_state(self.ctx, dst, lbm_checkpoint_bytes(self.params))
        return dst

    @_ordered
    def load_state(self, src, t=0):
        lbm_load_state(self.ctx, src, t, lbm_checkpoint_bytes(self.params))
        self._keep = [src]
        return self

    @_ordered
    def step_saved(self, src, dst):
        lbm_step_saved(self.ctx, src, dst, lbm_checkpoint_bytes(self.params))
        return dst

    # ---- adjoint -----------------------------------------------------------
    def adjoint_buffer(self):
        nbytes = lbm_adjoint_bytes(self.params)
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "the adjoint needs LBM_FP32 storage")
        return torch.empty(nbytes, dtype=torch.uint8, device=self.f_a.device)

    @_ordered
    def adjoint_seed(self, lam, adj=None):
        adj = self.adjoint_buffer() if adj is None else adj
        lam = torch.as_tensor(lam, dtype=torch.float32).to(self.f_a.device).contiguous()
        lbm_adjoint_seed(self.ctx, lam, adj, self.n, lbm_adjoint_bytes(self.params))
        return adj

    @_ordered
    def adjoint_step(self, f_t, adj_next, adj_out):
        lbm_adjoint_step(self.ctx, f_t, adj_next, adj_out, lbm_checkpoint_bytes(self.params),
                         lbm_adjoint_bytes(self.params))
        return adj_out

    @_ordered
    def step_saved_chain(self, bufs):
        lbm_step_saved_chain(self.ctx, bufs, lbm_checkpoint_bytes(self.params))

    @_ordered
    def adjoint_run(self, f_states, adj_a, adj_b):
        """Adjoint steps back through f_states; returns the buffer holding the result."""
        w = lbm_adjoint_run(self.ctx, f_states, adj_a, adj_b, lbm_checkpoint_bytes(self.params),
                            lbm_adjoint_bytes(self.params))
        return adj_a if w == 0 else adj_b

    @_ordered
    def adjoint_get(self, adj):
        lam = torch.empty((9, self.ny, self.nx), dtype=torch.float32, device=self.f_a.device)
        lbm_adjoint_get(self.ctx, adj, lam, self.n, lbm_adjoint_bytes(self.params))
        return lam

    @_ordered
    def adjoint_init(self, rho0, adj0, ux0=None, uy0=None):
        dev = self.f_a.device
        conv = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float32).to(dev).contiguous()
        rho0, ux0, uy0 = conv(rho0), conv(ux0), conv(uy0)
        drho0 = torch.empty((self.ny, self.nx), dtype=torch.float32, device=dev)
        lbm_adjoint_init(self.ctx, rho0, ux0, uy0, adj0, drho0, self.n, lbm_adjoint_bytes(self.params))
        return drho0

    @_ordered
    def adjoint_theta(self, reset=True):
        return lbm_adjoint_theta(self.ctx, True, reset)

    @property
    def time(self):
        return lbm_time(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

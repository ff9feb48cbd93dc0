"""ctypes binding of libsbiem (argument marshalling only).

Every ``sbiem_*`` function of the C ABI is available on ``lib`` with its
argument types set.  ``Plan`` and ``Batch`` wrap the handles and convert
numpy arrays (FP64, C order) to pointers; each method calls the C function
of the same name and raises ``SbiemError`` on a negative status.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "lib", "libsbiem.so")

if not os.path.exists(lib_path):
    raise ImportError(f"{lib_path} is missing: build it with "
                      "'python -m paper_2107_03550_amd.build' (hipcc, gfx950)")
# PyTorch bundles a HIP runtime with the same SONAME (libamdhip64.so.7) but
# loads it under another file name, so whichever comes first decides whether
# the process ends up with one runtime or two.  Load torch first: the library
# then binds to torch's runtime and shares devices and streams with it.
try:
    import torch  # noqa: F401
except ImportError:
    pass
lib = ctypes.CDLL(lib_path)

SBIEM_FP64 = 0
SBIEM_FP32CONV = 1
SBIEM_THETA_PAPER = 0
SBIEM_THETA_EXP = 1
SBIEM_RULE_MIDPOINT = 0
SBIEM_RULE_INTERVAL = 1
ADAPT_OUTCOMES = ("accept", "reject", "fail", "floor", "stop")
CLOSURE_PARAMS = 6466

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I64 = ctypes.POINTER(ctypes.c_int64)
_VP = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_int = ctypes.c_int
_PLAN = ctypes.c_void_p
_PPLAN = ctypes.POINTER(ctypes.c_void_p)
_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGS = {
    "sbiem_abi_version": (_int, []),
    "sbiem_status_string": (ctypes.c_char_p, [_int]),
    "sbiem_plan_create": (_int, [_PPLAN, _i64, _dbl, _dbl, _dbl, _dbl, _dbl, _D]),
    "sbiem_plan_destroy": (_int, [_PLAN]),
    "sbiem_last_error": (ctypes.c_char_p, [_PLAN]),
    "sbiem_set_precision": (_int, [_PLAN, _int]),
    "sbiem_set_theta_mode": (_int, [_PLAN, _int]),
    "sbiem_set_newton_limit": (_int, [_PLAN, _int]),
    "sbiem_set_rule": (_int, [_PLAN, _int]),
    "sbiem_set_cutoffs": (_int, [_PLAN, _dbl, _dbl]),
    "sbiem_set_adaptive": (_int, [_PLAN, _int]),
    "sbiem_step_var": (_int, [_PLAN, _dbl]),
    "sbiem_adapt": (_int, [_PLAN, _dbl, _dbl, _dbl, _i64, _D, _D, _i64, _I64]),
    "sbiem_adapt_until": (_int, [_PLAN, _dbl, _dbl, _dbl, _i64, _dbl, _D, _D, _i64, _I64,
                                 ctypes.POINTER(ctypes.c_int)]),
    "sbiem_set_constrained": (_int, [_PLAN, ctypes.POINTER(ctypes.c_uint8)]),
    "sbiem_set_conv_tile": (_int, [_PLAN, _int]),
    "sbiem_get_conv_tile": (_int, [_PLAN, ctypes.POINTER(ctypes.c_int)]),
    "sbiem_slip_scaling": (_int, [_i64, _dbl, _dbl, _D, _dbl, _D]),
    "sbiem_kernel_primitive_eval": (_int, [_dbl, _dbl, _D, _i64, _D, _D]),
    "sbiem_set_friction": (_int, [_PLAN, _D, _D, _dbl, _dbl, _dbl, _D, _D, _dbl, _dbl]),
    "sbiem_set_state": (_int, [_PLAN, _D, _D, _D, _dbl]),
    "sbiem_get_state": (_int, [_PLAN, _D, _D, _D, _D, _D, _D]),
    "sbiem_get_curvature": (_int, [_PLAN, _D]),
    "sbiem_set_dt": (_int, [_PLAN, _dbl]),
    "sbiem_window_lengths": (_int, [_PLAN, _dbl, _I64]),
    "sbiem_stress": (_int, [_PLAN, _D, _i64, _dbl, _D, _D]),
    "sbiem_step": (_int, [_PLAN, _dbl]),
    "sbiem_run": (_int, [_PLAN, _dbl, _i64]),
    "sbiem_steps_done": (_int, [_PLAN, _I64]),
    "sbiem_failures": (_int, [_PLAN, _I64, _I64]),
    "sbiem_set_stream": (_int, [_PLAN, _VP]),
    "sbiem_set_allocator": (_int, [_ALLOC, _FREE, _VP]),
    "sbiem_kernel_eval": (_int, [_dbl, _dbl, _D, _i64, _D, _D, _D, _D]),
    "sbiem_set_profiling": (_int, [_PLAN, _int]),
    "sbiem_profile": (_int, [_PLAN, _D, _I64, _D]),
    "sbiem_batch_create": (_int, [_PPLAN, ctypes.POINTER(ctypes.c_void_p), _i64]),
    "sbiem_batch_destroy": (_int, [_VP]),
    "sbiem_batch_run": (_int, [_VP, _i64]),
    "sbiem_batch_set_profiling": (_int, [_VP, _int]),
    "sbiem_batch_profile": (_int, [_VP, _D, _I64, _D]),
    "sbiem_tune": (_int, [_PLAN, _dbl, _i64, ctypes.POINTER(ctypes.c_int32)]),
    "sbiem_batch_tune": (_int, [_VP, _i64, ctypes.POINTER(ctypes.c_int32)]),
    "sbiem_set_closure": (_int, [_PLAN, _F, _F, _dbl]),
    "sbiem_closure_sample": (_int, [_PLAN, _dbl, _F, _F, _D]),
    "sbiem_closure_eval": (_int, [_F, _F, _i64, _F]),
    "sbiem_closure_train": (_int, [_F, _F, _i64, _i64, _i64, _dbl, _F, _F, _F, _I64, _D]),
    "sbiem_closure_train_noalloc": (_int, [_VP, _VP, _i64, _i64, _i64, _dbl, _VP, _VP, _VP, _I64,
                                           _VP, _VP]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED_NAMES = tuple(_SIGS)


class SbiemError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{lib.sbiem_status_string(status).decode()} ({status}): {message}")
        self.status = status


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def _arr(x, n=None, name="array"):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"{name}: expected {n} values, got {a.size}")
    return a


def _check(status, handle=None):
    if status != 0:
        msg = lib.sbiem_last_error(handle)
        raise SbiemError(status, msg.decode() if msg else "")
    return status


def abi_version():
    return lib.sbiem_abi_version()


def kernel_eval(T, cs, cp):
    """C^T, C^N, dC^T/dT, dC^N/dT at T (host extended precision)."""
    T = _arr(T)
    outs = [np.empty(T.size) for _ in range(4)]
    _check(lib.sbiem_kernel_eval(cs, cp, _ptr(T), T.size, *[_ptr(o) for o in outs]))
    return tuple(outs)


def kernel_primitive_eval(T, cs, cp):
    """P^T, P^N (integrals of the kernels over [0, T]) at T (host extended precision)."""
    T = _arr(T)
    outs = [np.empty(T.size) for _ in range(2)]
    _check(lib.sbiem_kernel_primitive_eval(cs, cp, _ptr(T), T.size, *[_ptr(o) for o in outs]))
    return tuple(outs)


def slip_scaling(slip, L, f, slip_floor=0.0):
    """sbiem_slip_scaling: (1/(f du)) d(du)/dx per element (NaN below the floor)."""
    u = _arr(slip)
    out = np.empty(u.size)
    _check(lib.sbiem_slip_scaling(u.size, float(L), float(f), _ptr(u), float(slip_floor),
                                  _ptr(out)))
    return out


def _f32(x, n=None, name="array"):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if n is not None and a.size != n:
        raise ValueError(f"{name}: expected {n} values, got {a.size}")
    return a


def _fptr(a):
    return None if a is None else a.ctypes.data_as(_F)


def closure_eval(params, X):
    """Network outputs (n, 2) for inputs X (n, 33) by the matrix-core kernel."""
    p = _f32(params, CLOSURE_PARAMS, "params")
    X = _f32(X).reshape(-1, 33)
    Y = np.empty((X.shape[0], 2), dtype=np.float32)
    _check(lib.sbiem_closure_eval(_fptr(p), _fptr(X), X.shape[0], _fptr(Y)))
    return Y


class ClosureTrainer:
    """Adam state of one network trained by sbiem_closure_train."""

    def __init__(self, params):
        self.params = _f32(params, CLOSURE_PARAMS, "params").copy()
        self.m = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
        self.v = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
        self.t = ctypes.c_int64(0)

    def train(self, X, Y, batch, steps, lr):
        X = _f32(X).reshape(-1, 33)
        Y = _f32(Y).reshape(-1, 2)
        losses = np.empty(int(steps))
        _check(lib.sbiem_closure_train(_fptr(X), _fptr(Y), X.shape[0], int(batch), int(steps), lr,
                                       _fptr(self.params), _fptr(self.m), _fptr(self.v),
                                       ctypes.byref(self.t), losses.ctypes.data_as(_D)))
        return losses


CLOSURE_TRAIN_MAX_BATCH = 4096


def closure_train_noalloc(X, Y, n, batch, steps, lr, params, adam_m, adam_v, adam_t, losses=None,
                          stream=None):
    """sbiem_closure_train_noalloc on device pointers (ints, e.g. a torch
    tensor's data_ptr()); ``adam_t`` is a ctypes.c_int64, updated.  Returns
    the status (0 when the updates were enqueued)."""
    return lib.sbiem_closure_train_noalloc(
        ctypes.c_void_p(int(X)), ctypes.c_void_p(int(Y)), int(n), int(batch), int(steps),
        float(lr), ctypes.c_void_p(int(params)), ctypes.c_void_p(int(adam_m)),
        ctypes.c_void_p(int(adam_v)), ctypes.byref(adam_t),
        None if losses is None else ctypes.c_void_p(int(losses)),
        None if stream is None else ctypes.c_void_p(int(stream)))


_torch_alloc_refs = []


def set_torch_allocator():
    """Route plan memory through torch's caching allocator (current stream)."""
    import torch

    def _alloc(nbytes, ctx):
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = _ALLOC(_alloc), _FREE(_free)
    _torch_alloc_refs[:] = [a, f]
    _check(lib.sbiem_set_allocator(a, f, None))


def set_default_allocator():
    """Back to hipMalloc/hipFree for memory allocated from now on (memory
    already allocated through torch must have been released first)."""
    _check(lib.sbiem_set_allocator(_ALLOC(), _FREE(), None))
    _torch_alloc_refs[:] = []


class Plan:
    """One fault (wraps sbiem_plan)."""

    def __init__(self, N, L, mu, nu, cs, cp, h=None):
        self.N = int(N)
        hh = None if h is None else _arr(h, self.N, "h")
        handle = ctypes.c_void_p()
        _check(lib.sbiem_plan_create(ctypes.byref(handle), self.N, L, mu, nu, cs, cp, _ptr(hh)))
        self.handle = handle
        self.L, self.mu, self.nu, self.cs, self.cp = L, mu, nu, cs, cp

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib.sbiem_plan_destroy(h)
            self.handle = None

    def _c(self, st):
        return _check(st, self.handle)

    def set_precision(self, mode):
        self._c(lib.sbiem_set_precision(self.handle, mode))

    def set_theta_mode(self, mode):
        self._c(lib.sbiem_set_theta_mode(self.handle, mode))

    def set_newton_limit(self, max_iterations):
        self._c(lib.sbiem_set_newton_limit(self.handle, int(max_iterations)))

    def set_rule(self, rule):
        self._c(lib.sbiem_set_rule(self.handle, int(rule)))

    def set_cutoffs(self, kcL_shear, kcL_normal):
        self._c(lib.sbiem_set_cutoffs(self.handle, float(kcL_shear), float(kcL_normal)))

    def set_adaptive(self, on=True):
        self._c(lib.sbiem_set_adaptive(self.handle, 1 if on else 0))

    def step_var(self, dt):
        self._c(lib.sbiem_step_var(self.handle, float(dt)))

    def step_var_status(self, dt):
        return lib.sbiem_step_var(self.handle, float(dt))

    def adapt(self, eps0, dt_max, dt, max_accepted, t_end=np.inf, log_cap=100000):
        """Controlled steps (sbiem_adapt).  Returns (status, next dt, log) with
        log an array of (t, dt, eps, outcome) rows, one per attempt."""
        d = ctypes.c_double(float(dt))
        log = np.zeros((int(log_cap), 4))
        n = ctypes.c_int64()
        st = lib.sbiem_adapt(self.handle, float(eps0), float(dt_max), float(t_end),
                             int(max_accepted), ctypes.byref(d), _ptr(log), int(log_cap),
                             ctypes.byref(n))
        if st not in (0, -4, -5, -6):
            _check(st, self.handle)
        return st, d.value, log[:min(n.value, int(log_cap))]

    def adapt_until(self, eps0, dt_max, dt, max_accepted, v_cross, t_end=float("inf"),
                    log_cap=None):
        """sbiem_adapt_until: (status, next dt, log [attempts x 5], crossed)."""
        if log_cap is None:
            log_cap = 64 * int(max_accepted) + 64
        d = ctypes.c_double(float(dt))
        log = np.zeros((int(log_cap), 5))
        n = ctypes.c_int64()
        crossed = ctypes.c_int()
        st = lib.sbiem_adapt_until(self.handle, float(eps0), float(dt_max), float(t_end),
                                   int(max_accepted), float(v_cross), ctypes.byref(d), _ptr(log),
                                   int(log_cap), ctypes.byref(n), ctypes.byref(crossed))
        if st not in (0, -4, -5, -6):
            _check(st, self.handle)
        return st, d.value, log[:min(n.value, int(log_cap))], bool(crossed.value)

    def set_constrained(self, mask):
        """Elements held at V_pl (None frees all); set_state must follow."""
        if mask is None:
            self._c(lib.sbiem_set_constrained(self.handle, None))
            return
        m = np.ascontiguousarray(np.asarray(mask).astype(np.uint8).reshape(-1))
        if m.size != self.N:
            raise ValueError(f"mask: expected {self.N} values, got {m.size}")
        self._c(lib.sbiem_set_constrained(self.handle,
                                          m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))

    def set_friction(self, a, b, Dc, V_ref, f0, sigma_load, tau_load, tau_load_rate=0.0, V_pl=0.0):
        n = self.N
        a, b, s, t = (_arr(v, n, k) for v, k in ((a, "a"), (b, "b"), (sigma_load, "sigma_load"),
                                                 (tau_load, "tau_load")))
        self._c(lib.sbiem_set_friction(self.handle, _ptr(a), _ptr(b), Dc, V_ref, f0, _ptr(s),
                                       _ptr(t), tau_load_rate, V_pl))

    def set_state(self, slip, V, theta, t=0.0):
        n = self.N
        s, v, th = _arr(slip, n, "slip"), _arr(V, n, "V"), _arr(theta, n, "theta")
        self._c(lib.sbiem_set_state(self.handle, _ptr(s), _ptr(v), _ptr(th), t))

    def get_state(self):
        n = self.N
        out = {k: np.empty(n) for k in ("slip", "V", "theta", "tau_el", "sigma_el")}
        t = ctypes.c_double()
        self._c(lib.sbiem_get_state(self.handle, _ptr(out["slip"]), _ptr(out["V"]),
                                    _ptr(out["theta"]), _ptr(out["tau_el"]),
                                    _ptr(out["sigma_el"]), ctypes.byref(t)))
        out["t"] = t.value
        return out

    def get_curvature(self):
        k = np.empty(self.N)
        self._c(lib.sbiem_get_curvature(self.handle, _ptr(k)))
        return k

    def set_dt(self, dt):
        self._c(lib.sbiem_set_dt(self.handle, dt))

    def window_lengths(self, dt):
        M = np.empty(self.N // 2, dtype=np.int64)
        self._c(lib.sbiem_window_lengths(self.handle, dt, M.ctypes.data_as(_I64)))
        return M

    def stress(self, slip_hist, dt):
        h = _arr(slip_hist).reshape(-1, self.N)
        tau, sig = np.empty(self.N), np.empty(self.N)
        self._c(lib.sbiem_stress(self.handle, _ptr(h), h.shape[0] - 1, dt, _ptr(tau), _ptr(sig)))
        return tau, sig

    def step(self, dt):
        self._c(lib.sbiem_step(self.handle, dt))

    def run(self, dt, nsteps):
        self._c(lib.sbiem_run(self.handle, dt, int(nsteps)))

    def run_status(self, dt, nsteps):
        """Like run() but returns the status instead of raising."""
        return lib.sbiem_run(self.handle, dt, int(nsteps))

    def steps_done(self):
        n = ctypes.c_int64()
        self._c(lib.sbiem_steps_done(self.handle, ctypes.byref(n)))
        return n.value

    def failures(self):
        c, i = ctypes.c_int64(), ctypes.c_int64()
        self._c(lib.sbiem_failures(self.handle, ctypes.byref(c), ctypes.byref(i)))
        return c.value, i.value

    def set_stream(self, stream_ptr):
        self._c(lib.sbiem_set_stream(self.handle, ctypes.c_void_p(int(stream_ptr))))

    def set_profiling(self, on=True):
        self._c(lib.sbiem_set_profiling(self.handle, 1 if on else 0))

    def profile(self):
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._c(lib.sbiem_profile(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def set_conv_tile(self, records):
        """FP32 conv tile (64: packed rows, 256, 320, 512, 1024 records; 0 = default by window)."""
        self._c(lib.sbiem_set_conv_tile(self.handle, int(records)))

    def conv_tile(self):
        r = ctypes.c_int()
        self._c(lib.sbiem_get_conv_tile(self.handle, ctypes.byref(r)))
        return r.value

    def tune(self, dt, steps_per_trial=64):
        """Autotune the convolution grid on ordinary steps; returns the
        chosen number of conv workgroups (the state advances)."""
        g = ctypes.c_int32()
        self._c(lib.sbiem_tune(self.handle, dt, int(steps_per_trial), ctypes.byref(g)))
        return g.value

    def last_error(self):
        m = lib.sbiem_last_error(self.handle)
        return m.decode() if m else ""

    def set_closure(self, params_shear, params_normal, cut=0.25):
        """Learned tail closure on (None, None: off)."""
        if params_shear is None:
            self._c(lib.sbiem_set_closure(self.handle, None, None, cut))
            return
        a = _f32(params_shear, CLOSURE_PARAMS, "params_shear")
        b = _f32(params_normal, CLOSURE_PARAMS, "params_normal")
        self._c(lib.sbiem_set_closure(self.handle, _fptr(a), _fptr(b), cut))

    def closure_sample(self, cut=0.25):
        """(X[2][N/2+1][33], Y[2][N/2+1][2], R[2][N/2+1]) from the current history."""
        h = self.N // 2 + 1
        X = np.empty((2, h, 33), dtype=np.float32)
        Y = np.empty((2, h, 2), dtype=np.float32)
        R = np.empty((2, h))
        self._c(lib.sbiem_closure_sample(self.handle, cut, _fptr(X), _fptr(Y), _ptr(R)))
        return X, Y, R


class Batch:
    """Ensemble of plans stepped together (wraps sbiem_batch)."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        handle = ctypes.c_void_p()
        _check(lib.sbiem_batch_create(ctypes.byref(handle), arr, len(self.plans)))
        self.handle = handle

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib.sbiem_batch_destroy(h)
            self.handle = None

    def run(self, nsteps):
        st = lib.sbiem_batch_run(self.handle, int(nsteps))
        if st != 0:
            raise SbiemError(st, lib.sbiem_last_error(None).decode())

    def run_status(self, nsteps):
        return lib.sbiem_batch_run(self.handle, int(nsteps))

    def tune(self, steps_per_trial=64):
        """Autotune the convolution grid on ordinary steps; returns the
        chosen number of conv workgroups (the faults advance)."""
        g = ctypes.c_int32()
        st = lib.sbiem_batch_tune(self.handle, int(steps_per_trial), ctypes.byref(g))
        if st != 0:
            raise SbiemError(st, lib.sbiem_last_error(None).decode())
        return g.value

    def set_profiling(self, on=True):
        _check(lib.sbiem_batch_set_profiling(self.handle, 1 if on else 0))

    def profile(self):
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(lib.sbiem_batch_profile(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

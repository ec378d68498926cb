"""Thin Python binding of the qhfpe C-ABI (include/qhfpe.h).

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch provides device memory (the workspace and the state /
response buffers) and the stream.  There is no fallback: if libqhfpe.so is
missing, importing the library raises.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqhfpe.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "qhfpe.h")

OK, EINVAL, EUNSUPPORTED, EHIP, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5
CLOSURE_KERNEL_FLOATS = 13 * 13 * 8 * 4
CLOSURE_STATS_DOUBLES = 25 * 25 * 8 * 8 + 13 * 13 * 8 * 4 + 1
CLOSURE_TRAIN_FLOATS = 203906
FP64, FP32_FP64RED = 0, 1
COMMUTATOR = 0
MAX_STATES = 3

_c_int = ctypes.c_int
_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_dbl = ctypes.c_double
_vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [
        ("n_states", _c_i32), ("nq", _c_i32), ("np", _c_i32), ("depth", _c_i32),
        ("batch", _c_i32), ("precision", _c_i32), ("low_temp_correction", _c_i32),
        ("reserved", _c_i32),
        ("q_min", _c_dbl), ("q_max", _c_dbl), ("p_min", _c_dbl), ("p_max", _c_dbl),
        ("mass", _c_dbl), ("hbar", _c_dbl),
        ("zeta", _c_dbl), ("gamma", _c_dbl), ("beta", _c_dbl),
        ("dt", _c_dbl),
        ("poly", _c_dbl * 5 * MAX_STATES * MAX_STATES),
        ("mu", _c_dbl * MAX_STATES * MAX_STATES),
    ]


POTENTIAL_FN = ctypes.CFUNCTYPE(_c_dbl, _c_i32, _c_i32, _c_dbl, _vp)


class MorseGauss(ctypes.Structure):
    """qhfpe_morse_gauss: displaced Morse diagonals and a Gaussian coupling."""
    _fields_ = [(n, _c_dbl) for n in ("D0", "D1", "a0", "a1", "q0", "q1", "dE", "dV", "qs", "sigma")]


class QHFPEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qhfpe error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libqhfpe.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    sig = {
        "qhfpe_workspace_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], _c_int),
        "qhfpe_create": ([P, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)], _c_int),
        "qhfpe_destroy": ([_vp], _c_int),
        "qhfpe_set_state": ([_vp, _vp, _c_i32, _c_i32], _c_int),
        "qhfpe_get_state": ([_vp, _vp, _c_i32], _c_int),
        "qhfpe_get_phase": ([_vp, ctypes.POINTER(_c_i32)], _c_int),
        "qhfpe_set_member_bath": ([_vp, _c_i32, _c_dbl, _c_dbl, _c_dbl], _c_int),
        "qhfpe_set_member_depth": ([_vp, _c_i32, _c_i32], _c_int),
        "qhfpe_set_tile": ([_vp, _c_i32], _c_int),
        "qhfpe_autotune": ([_vp, _c_i32, ctypes.POINTER(_c_i32)], _c_int),
        "qhfpe_set_streams": ([_vp, _c_i32], _c_int),
        "qhfpe_set_potential": ([_vp, _vp, _vp], _c_int),
        "qhfpe_set_potential_tables": ([_vp, _vp, _vp], _c_int),
        "qhfpe_morse_gauss_potential": ([_c_i32, _c_i32, _c_dbl, _vp], _c_dbl),
        "qhfpe_get_streams": ([_vp, ctypes.POINTER(_c_i32)], _c_int),
        "qhfpe_init_thermal": ([_vp, _c_dbl, _vp], _c_int),
        "qhfpe_apply_dipole": ([_vp, _c_i32], _c_int),
        "qhfpe_step": ([_vp, _c_i64, _c_i32, _vp], _c_int),
        "qhfpe_step_async": ([_vp, _c_i64, _c_i32, _vp], _c_int),
        "qhfpe_status": ([_vp], _c_int),
        "qhfpe_stream_copy": ([_vp, _vp, ctypes.c_size_t, _vp], _c_int),
        "qhfpe_graph_begin": ([_vp], _c_int),
        "qhfpe_graph_end": ([_vp, ctypes.POINTER(_vp)], _c_int),
        "qhfpe_graph_nodes": ([_vp, ctypes.POINTER(ctypes.c_size_t)], _c_int),
        "qhfpe_graph_launch": ([_vp, _vp], _c_int),
        "qhfpe_graph_destroy": ([_vp], _c_int),
        "qhfpe_response": ([_vp, _vp], _c_int),
        "qhfpe_apply_rhs": ([_vp], _c_int),
        "qhfpe_residual": ([_vp, ctypes.POINTER(_c_dbl)], _c_int),
        "qhfpe_relax": ([_vp, _c_dbl, _c_i64, _c_i32, ctypes.POINTER(_c_i64), ctypes.POINTER(_c_dbl)], _c_int),
        "qhfpe_copy_members": ([_vp, _c_i32, _vp, _c_i32, _c_i32], _c_int),
        "qhfpe_spectrum_abs": ([_vp, _c_i64, _c_dbl, _vp, _c_i32, _vp, _vp], _c_int),
        "qhfpe_spectrum_corr": ([_vp, _c_i32, _c_i32, _c_dbl, _c_dbl, _vp, _c_i32, _vp, _c_i32, _vp, _vp, _vp],
                                _c_int),
        "qhfpe_spectrum_corr_noalloc": ([_vp, _c_i32, _c_i32, _c_dbl, _c_dbl, _vp, _c_i32, _vp, _c_i32, _vp, _vp],
                                        _c_int),
        "qhfpe_closure_stats": ([_vp, _c_i32, _vp], _c_int),
        "qhfpe_closure_train": ([_vp, _vp, _c_dbl, _vp, ctypes.c_uint64, _c_i32, _c_dbl, _c_dbl, _vp,
                                 ctypes.POINTER(_c_dbl), _vp], _c_int),
        "qhfpe_closure_gmfp_kernel": ([_vp, _vp], _c_int),
        "qhfpe_closure_loss": ([_vp, _vp, _vp, ctypes.POINTER(_c_dbl), _vp], _c_int),
        "qhfpe_closure_buffer_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], _c_int),
        "qhfpe_set_closure": ([_vp, _vp, _vp, ctypes.c_size_t], _c_int),
        "qhfpe_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def declared_symbols() -> list[str]:
    """Names of the entry points declared in include/qhfpe.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(qhfpe_[a-z_0-9]+)\s*\(", text)))


def _check(rc: int):
    if rc != OK:
        raise QHFPEError(rc, lib().qhfpe_last_error().decode())


def make_params(model: dict, batch: int = 1, precision: str = "fp64") -> Params:
    p = Params()
    p.n_states = int(model["n_states"])
    p.nq = int(model["nq"])
    p.np = int(model["np"])
    p.depth = int(model["depth"])
    p.batch = int(batch)
    p.precision = {"fp64": FP64, "fp32": FP32_FP64RED}[precision]
    p.low_temp_correction = int(bool(model.get("low_temp_correction", True)))
    p.reserved = 0
    for k in ("q_min", "q_max", "p_min", "p_max", "zeta", "gamma", "beta", "dt"):
        setattr(p, k, float(model[k]))
    p.mass = float(model.get("mass", 1.0))
    p.hbar = float(model.get("hbar", 1.0))
    ns = p.n_states
    poly = np.zeros((MAX_STATES, MAX_STATES, 5))
    poly[:ns, :ns, :] = np.asarray(model["poly"], dtype=np.float64)[:ns, :ns, :5]
    mu = np.zeros((MAX_STATES, MAX_STATES))
    mu[:ns, :ns] = np.asarray(model["mu"], dtype=np.float64)
    for j in range(MAX_STATES):
        for l in range(MAX_STATES):
            p.mu[j][l] = mu[j, l]
            for k in range(5):
                p.poly[j][l][k] = poly[j, l, k]
    return p


def workspace_bytes(model: dict, batch: int = 1, precision: str = "fp64") -> int:
    p = make_params(model, batch, precision)
    n = ctypes.c_size_t(0)
    _check(lib().qhfpe_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return int(n.value)


def _ptr(t) -> int:
    return ctypes.c_void_p(t.data_ptr())


class Propagator:
    """One qhfpe handle: a batch of propagations of one model on one GPU."""

    def __init__(self, model: dict, batch: int = 1, precision: str = "fp64", device=None, stream=None):
        import torch
        self.torch = torch
        self.model = dict(model)
        self.batch = int(batch)
        self.precision = precision
        self.device = torch.device(device if device is not None else "cuda")
        self.params = make_params(model, batch, precision)
        nbytes = workspace_bytes(model, batch, precision)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = ctypes.c_void_p()
        _check(lib().qhfpe_create(ctypes.byref(self.params), _ptr(self.workspace), nbytes,
                                  ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.shape = (self.model["depth"] + 1, self.model["n_states"], self.model["n_states"],
                      self.model["nq"], self.model["np"])

    # The library works on the handle's stream, torch on the caller's current
    # stream: tensors handed to the library are ordered before its work, and
    # tensors it fills are ordered before later torch work.
    def _after_torch(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _before_torch(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().qhfpe_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ---------------------------------------------------------------
    def set_state(self, W, phase: int = 0, member: int = -1):
        t = self.torch
        W = t.as_tensor(W, dtype=t.complex128, device=self.device).contiguous()
        self._keep = W
        self._after_torch()
        _check(lib().qhfpe_set_state(self.handle, _ptr(W), int(phase), int(member)))

    def get_state(self, member: int = -1):
        t = self.torch
        n = self.batch if member < 0 else 1
        out = t.empty((n,) + self.shape, dtype=t.complex128, device=self.device)
        self._after_torch()
        _check(lib().qhfpe_get_state(self.handle, _ptr(out), int(member)))
        self._before_torch()
        return out

    @property
    def phase(self) -> int:
        v = _c_i32(0)
        _check(lib().qhfpe_get_phase(self.handle, ctypes.byref(v)))
        return int(v.value)

    def set_member_bath(self, member: int, zeta: float, gamma: float, beta: float):
        _check(lib().qhfpe_set_member_bath(self.handle, int(member), float(zeta), float(gamma), float(beta)))

    def set_member_depth(self, member: int, depth: int):
        """Hierarchy depth of one member (<= the model's depth;
        qhfpe_set_member_depth)."""
        _check(lib().qhfpe_set_member_depth(self.handle, int(member), int(depth)))

    def set_tile(self, cells_per_thread: int):
        _check(lib().qhfpe_set_tile(self.handle, int(cells_per_thread)))

    def set_potential(self, fn):
        """Surfaces from a Python function fn(j, l, x) -> U_jl(x) (j <= l),
        evaluated by the library on the host while it rebuilds the r-space
        multipliers (qhfpe_set_potential)."""
        cb = POTENTIAL_FN(lambda j, l, x, ctx: float(fn(j, l, x)))
        _check(lib().qhfpe_set_potential(self.handle, ctypes.cast(cb, _vp), None))

    def set_potential_tables(self, u_plus, u_minus):
        """Surfaces as the r-space tables U_jl(q_i +- r_m/2), host arrays of
        shape (n_states, n_states, nq, np) in DFT order along m, used as
        given (qhfpe_set_potential_tables)."""
        import numpy as np
        shape = (self.model["n_states"],) * 2 + (self.model["nq"], self.model["np"])
        up = np.ascontiguousarray(u_plus, dtype=np.float64)
        um = np.ascontiguousarray(u_minus, dtype=np.float64)
        if up.shape != shape or um.shape != shape:
            raise ValueError(f"u_plus and u_minus must have shape {shape}")
        _check(lib().qhfpe_set_potential_tables(self.handle, up.ctypes.data_as(_vp), um.ctypes.data_as(_vp)))

    def set_potential_morse_gauss(self, **params):
        """The Morse/Gaussian surfaces of Sec. III, evaluated by the library's
        own qhfpe_morse_gauss_potential (params: MorseGauss fields)."""
        c = MorseGauss(**{k: float(v) for k, v in params.items()})
        fn = ctypes.cast(lib().qhfpe_morse_gauss_potential, _vp)
        _check(lib().qhfpe_set_potential(self.handle, fn, ctypes.byref(c)))

    def set_streams(self, groups: int):
        """Member groups of step(): 1 = one launch per stage, 2..4 = that many
        member ranges on streams of their own, 0 = default."""
        _check(lib().qhfpe_set_streams(self.handle, int(groups)))

    def streams(self) -> int:
        g = ctypes.c_int32(0)
        _check(lib().qhfpe_get_streams(self.handle, ctypes.byref(g)))
        return int(g.value)

    def autotune(self, reps: int = 20) -> int:
        v = _c_i32(0)
        _check(lib().qhfpe_autotune(self.handle, int(reps), ctypes.byref(v)))
        return int(v.value)

    def init_thermal(self, omega: float, noise=None):
        t = self.torch
        ptr = None
        if noise is not None:
            noise = t.as_tensor(noise, dtype=t.float64, device=self.device).contiguous()
            if noise.numel() != self.model["nq"] * self.model["np"]:
                raise ValueError(f"noise must have nq * np = {self.model['nq'] * self.model['np']} entries")
            self._noise = noise
            ptr = _ptr(noise)
            self._after_torch()
        _check(lib().qhfpe_init_thermal(self.handle, float(omega), ptr))

    # -- dynamics ------------------------------------------------------------
    def apply_dipole(self):
        _check(lib().qhfpe_apply_dipole(self.handle, COMMUTATOR))

    def step(self, nsteps: int, stride: int = 1, record: bool = True, out=None, asynchronous: bool = False):
        """nsteps RK4 steps; with record, the trace every stride steps into
        out (complex128 [B][nsteps/stride + 1], allocated if None).
        asynchronous: qhfpe_step_async (no status read back; see status())."""
        t = self.torch
        fn = lib().qhfpe_step_async if asynchronous else lib().qhfpe_step
        if not record:
            _check(fn(self.handle, int(nsteps), int(stride), None))
            return None
        n = nsteps // stride + 1
        if out is None:
            out = t.empty((self.batch, n), dtype=t.complex128, device=self.device)
        elif (out.dtype != t.complex128 or tuple(out.shape) != (self.batch, n) or not out.is_contiguous()
              or out.device != self.workspace.device):
            raise ValueError(f"out must be a contiguous complex128 tensor of shape ({self.batch}, {n}) "
                             f"on {self.workspace.device}")
        self._after_torch()
        _check(fn(self.handle, int(nsteps), int(stride), _ptr(out)))
        return out

    def status(self):
        """Raise QHFPEError(ENONFINITE) if an asynchronous step saw a
        non-finite trace since the last check (synchronises the stream)."""
        _check(lib().qhfpe_status(self.handle))

    def response(self):
        t = self.torch
        out = t.empty((self.batch,), dtype=t.complex128, device=self.device)
        self._after_torch()
        _check(lib().qhfpe_response(self.handle, _ptr(out)))
        self._before_torch()
        return out

    def apply_rhs(self):
        _check(lib().qhfpe_apply_rhs(self.handle))

    def residual(self) -> np.ndarray:
        out = (_c_dbl * (2 * self.batch))()
        _check(lib().qhfpe_residual(self.handle, out))
        return np.array(out[:]).reshape(self.batch, 2)

    def relax(self, tol: float, max_steps: int, check_every: int = 100):
        steps = _c_i64(0)
        res = _c_dbl(0.0)
        _check(lib().qhfpe_relax(self.handle, float(tol), int(max_steps), int(check_every),
                                 ctypes.byref(steps), ctypes.byref(res)))
        return int(steps.value), float(res.value)

    def copy_members_from(self, src: "Propagator", src_member: int, dst_member: int, count: int):
        _check(lib().qhfpe_copy_members(src.handle, int(src_member), self.handle, int(dst_member), int(count)))

    def synchronize(self):
        self.stream.synchronize()

    # -- learned terminator ---------------------------------------------------
    def closure_stats(self, level: int, stats):
        """Accumulate the closure statistics of (level, level + 1) into stats
        (float64 device tensor of CLOSURE_STATS_DOUBLES, zeroed by the caller)."""
        if stats.dtype != self.torch.float64 or stats.numel() != CLOSURE_STATS_DOUBLES or not stats.is_contiguous():
            raise ValueError(f"stats must be a contiguous float64 tensor of {CLOSURE_STATS_DOUBLES}")
        self._after_torch()
        _check(lib().qhfpe_closure_stats(self.handle, int(level), _ptr(stats)))
        self._before_torch()

    def closure_gmfp_kernel(self):
        """The kernel of Eq. (GMFP) for this handle's bath and grid (numpy float32 [13][13][8][4])."""
        k = (ctypes.c_float * CLOSURE_KERNEL_FLOATS)()
        _check(lib().qhfpe_closure_gmfp_kernel(self.handle, k))
        return np.array(k[:], dtype=np.float32).reshape(13, 13, 8, 4)

    def set_closure(self, kernel=None):
        """Use the closure kernel (float32 [13][13][8][4] device tensor) at the
        deepest level; None switches back to Eq. (GMFP)."""
        t = self.torch
        if kernel is None:
            _check(lib().qhfpe_set_closure(self.handle, None, None, 0))
            self._closure_buf = None
            return
        kernel = t.as_tensor(kernel, dtype=t.float32, device=self.device).contiguous()
        if kernel.numel() != CLOSURE_KERNEL_FLOATS:
            raise ValueError(f"the closure kernel has {CLOSURE_KERNEL_FLOATS} entries")
        n = ctypes.c_size_t(0)
        _check(lib().qhfpe_closure_buffer_bytes(ctypes.byref(self.params), ctypes.byref(n)))
        self._closure_buf = t.empty(int(n.value), dtype=t.uint8, device=self.device)
        self._after_torch()
        _check(lib().qhfpe_set_closure(self.handle, _ptr(kernel), _ptr(self._closure_buf), int(n.value)))
        self.synchronize()  # the kernel tensor is read during the call


def closure_train(stats, iters: int = 3000, lr: float = 3e-3, lr_final: float = 1e-5, seed: int = 1706,
                  prior=None, ridge: float = 0.0, stream=None):
    """Train the closure's three layers on the statistics (float64 device
    tensor), with a ridge pull of weight `ridge` towards the kernel `prior`;
    returns (composite kernel float32 [13][13][8][4], normalised data loss)."""
    import torch
    state = torch.empty(CLOSURE_TRAIN_FLOATS, dtype=torch.float32, device=stats.device)
    kernel = torch.empty((13, 13, 8, 4), dtype=torch.float32, device=stats.device)
    if prior is not None:
        prior = torch.as_tensor(prior, dtype=torch.float32, device=stats.device).contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(stats.device)
    loss = _c_dbl(0.0)
    _check(lib().qhfpe_closure_train(_ptr(stats), _ptr(prior) if prior is not None else None, float(ridge),
                                     _ptr(state), int(seed), int(iters), float(lr), float(lr_final), _ptr(kernel),
                                     ctypes.byref(loss), ctypes.c_void_p(s.cuda_stream)))
    return kernel, float(loss.value)


def closure_loss(stats, kernel, stream=None) -> float:
    """The normalised data loss of a closure kernel on the statistics."""
    import torch
    kernel = torch.as_tensor(kernel, dtype=torch.float32, device=stats.device).contiguous()
    state = torch.empty(CLOSURE_TRAIN_FLOATS, dtype=torch.float32, device=stats.device)
    s = stream if stream is not None else torch.cuda.current_stream(stats.device)
    loss = _c_dbl(0.0)
    _check(lib().qhfpe_closure_loss(_ptr(stats), _ptr(kernel), _ptr(state), ctypes.byref(loss),
                                    ctypes.c_void_p(s.cuda_stream)))
    return float(loss.value)


def stream_copy(dst, src, stream=None):
    """dst <- src (same byte count, 16-byte aligned device tensors) with the
    library's streaming copy kernel."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    s = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(lib().qhfpe_stream_copy(_ptr(dst), _ptr(src), nbytes, ctypes.c_void_p(s.cuda_stream)))


class Graph:
    """A recorded sequence of asynchronous library calls on one stream
    (qhfpe_graph_begin ... qhfpe_graph_end), replayed by launch()."""

    def __init__(self, stream):
        self.stream = stream
        self.handle = None

    def __enter__(self):
        _check(lib().qhfpe_graph_begin(ctypes.c_void_p(self.stream.cuda_stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        h = ctypes.c_void_p()
        rc = lib().qhfpe_graph_end(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if exc_type is None:
            _check(rc)
            self.handle = h
        elif rc == OK:
            lib().qhfpe_graph_destroy(h)
        return False

    @property
    def nodes(self) -> int:
        n = ctypes.c_size_t(0)
        _check(lib().qhfpe_graph_nodes(self.handle, ctypes.byref(n)))
        return int(n.value)

    def launch(self, stream=None):
        s = stream if stream is not None else self.stream
        _check(lib().qhfpe_graph_launch(self.handle, ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().qhfpe_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spectrum_abs(series, dt: float, omegas, stream=None):
    import torch
    series = torch.as_tensor(series, dtype=torch.complex128, device="cuda").contiguous()
    om = torch.as_tensor(omegas, dtype=torch.float64, device=series.device).contiguous()
    out = torch.empty_like(om)
    s = stream if stream is not None else torch.cuda.current_stream(series.device)
    _check(lib().qhfpe_spectrum_abs(_ptr(series), series.numel(), float(dt), _ptr(om), om.numel(), _ptr(out),
                                    ctypes.c_void_p(s.cuda_stream)))
    return out


def spectrum_corr(r3, dt1: float, dt3: float, omega1, omega3, stream=None):
    """r3: complex [n1][n3] for one waiting time; returns [len(omega3), len(omega1)]."""
    import torch
    r3 = torch.as_tensor(r3, dtype=torch.complex128, device="cuda").contiguous()
    w1 = torch.as_tensor(omega1, dtype=torch.float64, device=r3.device).contiguous()
    w3 = torch.as_tensor(omega3, dtype=torch.float64, device=r3.device).contiguous()
    n1, n3 = r3.shape
    work = torch.empty((n1, w3.numel(), 2), dtype=torch.float64, device=r3.device)
    out = torch.empty((w3.numel(), w1.numel()), dtype=torch.float64, device=r3.device)
    s = stream if stream is not None else torch.cuda.current_stream(r3.device)
    _check(lib().qhfpe_spectrum_corr(_ptr(r3), n1, n3, float(dt1), float(dt3), _ptr(w1), w1.numel(), _ptr(w3),
                                     w3.numel(), _ptr(work), _ptr(out), ctypes.c_void_p(s.cuda_stream)))
    return out

"""Thin Python binding of the C ABI in ``include/ebit.h`` (argument
marshalling only: every step of the hot path runs in the HIP library).

PyTorch provides device memory and streams.  The binding fails loudly if the
built library is missing; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebit.so")

EBIT_OK, EBIT_EINVAL, EBIT_ECFL, EBIT_ESTATE, EBIT_EHIP, EBIT_ENOSURR, EBIT_ESCRATCH = 0, -1, -2, -3, -4, -5, -6
EBIT_ETOOBIG = -7
EBIT_MLP_STATIC_MAX_ROWS = 8192
EBIT_FP64, EBIT_FP32 = 0, 1
EBIT_OPT_FULL_GRID, EBIT_OPT_TIMING, EBIT_OPT_FUSE, EBIT_OPT_SUBLIST_CAP, EBIT_OPT_ORDER = 1, 2, 3, 4, 5

_lib = None


class EbitError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("s", (ctypes.c_void_p * 3) * 2),
        ("flags", ctypes.c_void_p * 2),
        ("scratch", ctypes.c_void_p),
        ("scratch_bytes", ctypes.c_size_t),
    ]


class Timing(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("sweep_ms", ctypes.c_double),
                ("f2v", ctypes.c_int64), ("f2v_ms", ctypes.c_double),
                ("fused", ctypes.c_int64), ("fused_ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("volume", ctypes.c_double),
        ("volume_comp", ctypes.c_double),
        ("n_interfacial", ctypes.c_int64),
        ("n_ambiguous", ctypes.c_int64),
        ("n_markers", ctypes.c_int64 * 3),
        ("n_fallback", ctypes.c_int64),
        ("n_multi", ctypes.c_int64),
        ("n_cfl", ctypes.c_int64),
        ("n_merged", ctypes.c_int64),
        ("n_active_cells", ctypes.c_int64),
        ("step_sweeps", ctypes.c_int64),
        ("n_interfacial_sum", ctypes.c_int64),
        ("max_courant", ctypes.c_double),
        ("n_annihilated", ctypes.c_int64),
        ("n_ambig_faces", ctypes.c_int64),
        ("n_surrogate", ctypes.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["n_markers"] = list(self.n_markers)
        return d


class Errors(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_double), ("volume_ref", ctypes.c_double), ("l1_diff", ctypes.c_double),
                ("e_shape", ctypes.c_double), ("e_mass", ctypes.c_double), ("samples", ctypes.c_int64)]


def lib():
    """Load ``libebit.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or python -m paper_2509_26361_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.ebit_scratch_bytes.argtypes = [ctypes.c_int32]
        L.ebit_scratch_bytes.restype = ctypes.c_size_t
        L.ebit_init.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Desc), P, P, P, P]
        L.ebit_init.restype = ctypes.c_int
        L.ebit_advect_sweep.argtypes = [P, ctypes.c_int, P, ctypes.c_double, ctypes.c_double, P]
        L.ebit_advect_sweep.restype = ctypes.c_int
        L.ebit_front2vof.argtypes = [P, P, P]
        L.ebit_front2vof.restype = ctypes.c_int
        L.ebit_stats.argtypes = [P, P, ctypes.POINTER(Stats), P]
        L.ebit_stats.restype = ctypes.c_int
        L.ebit_errors.argtypes = [P, P, P, ctypes.c_int, ctypes.POINTER(Errors), P]
        L.ebit_errors.restype = ctypes.c_int
        L.ebit_curvature_work_bytes.argtypes = [ctypes.c_int32]
        L.ebit_curvature_work_bytes.restype = ctypes.c_size_t
        L.ebit_curvature.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_size_t, P]
        L.ebit_curvature.restype = ctypes.c_int
        L.ebit_csf.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_double, P, P]
        L.ebit_csf.restype = ctypes.c_int
        L.ebit_refine_work_bytes.argtypes = [ctypes.c_int32]
        L.ebit_refine_work_bytes.restype = ctypes.c_size_t
        L.ebit_refine_band.argtypes = [ctypes.c_int32, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.ebit_refine_band.restype = ctypes.c_int
        L.ebit_current.argtypes = [P]
        L.ebit_current.restype = ctypes.c_int
        L.ebit_set_option.argtypes = [P, ctypes.c_int, ctypes.c_int]
        L.ebit_set_option.restype = ctypes.c_int
        L.ebit_destroy.argtypes = [P]
        L.ebit_destroy.restype = None
        L.ebit_strerror.argtypes = [ctypes.c_int]
        L.ebit_strerror.restype = ctypes.c_char_p
        L.ebit_mlp_param_count.argtypes = []
        L.ebit_mlp_param_count.restype = ctypes.c_int
        L.ebit_mlp_scratch_bytes.argtypes = []
        L.ebit_mlp_scratch_bytes.restype = ctypes.c_size_t
        L.ebit_mlp_forward.argtypes = [P, P, ctypes.c_int64, P, P]
        L.ebit_mlp_forward.restype = ctypes.c_int
        L.ebit_mlp_gradient.argtypes = [P, P, P, ctypes.c_int64, P, P, P, ctypes.c_size_t, P]
        L.ebit_mlp_gradient.restype = ctypes.c_int
        L.ebit_mlp_gradient_static.argtypes = [P, P, P, ctypes.c_int64, P, P, P]
        L.ebit_mlp_gradient_static.restype = ctypes.c_int
        L.ebit_mlp_adam.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_float, P]
        L.ebit_mlp_adam.restype = ctypes.c_int
        L.ebit_mlp_train.argtypes = [P, P, P, P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64, P,
                                     ctypes.c_int64, P, P, ctypes.c_size_t, P]
        L.ebit_mlp_train.restype = ctypes.c_int
        L.ebit_set_surrogate.argtypes = [P, P]
        L.ebit_set_surrogate.restype = ctypes.c_int
        L.ebit_surrogate_dataset.argtypes = [P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P]
        L.ebit_surrogate_dataset.restype = ctypes.c_int
        L.ebit_advance.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_double, P, P]
        L.ebit_advance.restype = ctypes.c_int
        L.ebit_timing.argtypes = [P, ctypes.POINTER(Timing)]
        L.ebit_timing.restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().ebit_strerror(int(code)).decode()
    except Exception:  # library missing: still format the error
        return "error"


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _ptr_array(ts):
    if ts is None:
        return None
    arr = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])
    return ctypes.cast(arr, ctypes.c_void_p), arr


class Ebit:
    """An EBIT state on one GPU: two state buffers, scratch and a context."""

    def __init__(self, n: int, precision: str = "fp64", device="cuda"):
        if n < 8 or n % 4:
            raise ValueError("n must be a multiple of 4 and >= 8")
        self.n = n
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device(device)
        shape = (n, n, n)
        self.flags = [torch.zeros(shape, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.s = [[torch.zeros(shape, dtype=self.dtype, device=self.device) for _ in range(3)] for _ in range(2)]
        nbytes = lib().ebit_scratch_bytes(n)
        self.scratch = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p(None)
        d = Desc()
        d.n = n
        d.precision = EBIT_FP64 if precision == "fp64" else EBIT_FP32
        for b in range(2):
            for e in range(3):
                d.s[b][e] = self.s[b][e].data_ptr()
            d.flags[b] = self.flags[b].data_ptr()
        d.scratch = self.scratch.data_ptr()
        d.scratch_bytes = nbytes
        self._desc = d

    # -- state ---------------------------------------------------------------
    def init(self, phi_nodes, phi_faces, s_exact=None, stream=None):
        """Markers and colours from sampled phi (device float64 tensors)."""
        self._destroy()
        pf, keep_pf = _ptr_array(phi_faces)
        se = _ptr_array(s_exact)
        rc = lib().ebit_init(ctypes.byref(self.ctx), ctypes.byref(self._desc), _ptr(phi_nodes), pf,
                             se[0] if se else None, _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_init")
        return self

    def load_state(self, flags, s, stream=None):
        """Start from a given state (e.g. a checkpoint): copies into buffer 0."""
        self._destroy()
        self.flags[0].copy_(flags)
        for e in range(3):
            self.s[0][e].copy_(s[e])
        rc = lib().ebit_init(ctypes.byref(self.ctx), ctypes.byref(self._desc), None, None, None, _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_init")
        return self

    def current(self):
        return lib().ebit_current(self.ctx)

    def state(self):
        """(flags, [s_x, s_y, s_z]) of the current buffer (views)."""
        c = self.current()
        return self.flags[c], self.s[c]

    def set_option(self, option, value):
        rc = lib().ebit_set_option(self.ctx, option, int(value))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_set_option")

    # -- hot path ------------------------------------------------------------
    def sweep(self, d: int, U, g: float, dt: float, stream=None):
        rc = lib().ebit_advect_sweep(self.ctx, int(d), _ptr(U), float(g), float(dt), _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_advect_sweep")

    def step(self, Uxyz, g: float, dt: float, order=(0, 1, 2), stream=None):
        for d in order:
            self.sweep(d, Uxyz[d], g, dt, stream)

    def advance(self, Uxyz, g, dt: float, C=None, stream=None):
        """len(g) steps (sweeps x, y, z with time factor g[k], then Front2VOF
        into C unless None), launched by the library (a Front2VOF and the next
        x sweep in one launch unless EBIT_OPT_FUSE is off)."""
        gs = (ctypes.c_double * max(1, len(g)))(*[float(v) for v in g])
        U = (ctypes.c_void_p * 3)(*[_ptr(u) for u in Uxyz])
        rc = lib().ebit_advance(self.ctx, len(g), U, gs, float(dt), _ptr(C) if C is not None else None,
                                _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_advance")

    def timing(self):
        """Launch times recorded since the last call (EBIT_OPT_TIMING on)."""
        t = Timing()
        rc = lib().ebit_timing(self.ctx, ctypes.byref(t))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_timing")
        return {k: getattr(t, k) for k, _ in Timing._fields_}

    def front2vof(self, C, stream=None):
        rc = lib().ebit_front2vof(self.ctx, _ptr(C), _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_front2vof")
        return C

    def stats(self, C, stream=None, check_cfl=True):
        st = Stats()
        rc = lib().ebit_stats(self.ctx, _ptr(C), ctypes.byref(st), _stream(stream))
        if rc not in (EBIT_OK, EBIT_ECFL) or (check_cfl and rc == EBIT_ECFL):
            raise EbitError(rc, "ebit_stats")
        return st.as_dict()

    def errors(self, C, C0, reset=False, stream=None):
        """E_mass (mean over the calls since a reset) and E_shape of C
        against C0 (paper eqs. Eq_error_surface, Eq_error_shape)."""
        e = Errors()
        rc = lib().ebit_errors(self.ctx, _ptr(C), _ptr(C0), int(bool(reset)), ctypes.byref(e), _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_errors")
        return {k: getattr(e, k) for k, _ in Errors._fields_}

    def set_surrogate(self, theta):
        """Front2VOF uses the surrogate for unambiguous cells (None: off)."""
        self._surr = theta
        rc = lib().ebit_set_surrogate(self.ctx, _ptr(theta) if theta is not None else None)
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_set_surrogate")

    def dataset(self, stream=None):
        """(x_bf16 (m, 32), c (m,)) training rows of the last Front2VOF."""
        cnt = ctypes.c_int64(0)
        rc = lib().ebit_surrogate_dataset(self.ctx, None, None, 0, ctypes.byref(cnt), _stream(stream))
        if rc != EBIT_OK:
            raise EbitError(rc, "ebit_surrogate_dataset")
        m = cnt.value
        x = torch.zeros((m, 32), dtype=torch.bfloat16, device=self.device)
        c = torch.zeros(m, dtype=torch.float32, device=self.device)
        if m:
            rc = lib().ebit_surrogate_dataset(self.ctx, _ptr(x), _ptr(c), m, ctypes.byref(cnt), _stream(stream))
            if rc != EBIT_OK:
                raise EbitError(rc, "ebit_surrogate_dataset")
        return x, c

    def _destroy(self):
        if self.ctx:
            lib().ebit_destroy(self.ctx)
            self.ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self._destroy()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# coupling of C to a flow solver: height-function curvature, CSF force
# ----------------------------------------------------------------------------

def _precision_of(t):
    if t.dtype == torch.float64:
        return EBIT_FP64
    if t.dtype == torch.float32:
        return EBIT_FP32
    raise ValueError("C must be float64 or float32")


def curvature(C, kappa=None, status=None, work=None, stream=None):
    """Height-function curvature of a cubic (n, n, n) C field: (kappa,
    status) device tensors (ebit_curvature)."""
    n = C.shape[0]
    if kappa is None:
        kappa = torch.empty_like(C)
    if status is None:
        status = torch.empty(C.shape, dtype=torch.uint8, device=C.device)
    if work is None:
        work = torch.empty(lib().ebit_curvature_work_bytes(n), dtype=torch.uint8, device=C.device)
    rc = lib().ebit_curvature(n, _precision_of(C), _ptr(C), _ptr(kappa), _ptr(status), _ptr(work), work.numel(),
                              _stream(stream))
    if rc != EBIT_OK:
        raise EbitError(rc, "ebit_curvature")
    return kappa, status


def csf(C, kappa, status, sigma, F=None, stream=None):
    """CSF face forces [F_x, F_y, F_z] (ebit_csf)."""
    if F is None:
        F = [torch.empty_like(C) for _ in range(3)]
    arr = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in F])
    rc = lib().ebit_csf(C.shape[0], _precision_of(C), _ptr(C), _ptr(kappa), _ptr(status), float(sigma),
                        ctypes.cast(arr, ctypes.c_void_p), _stream(stream))
    if rc != EBIT_OK:
        raise EbitError(rc, "ebit_csf")
    return F


def refine_band(flags, mask_prev=None, out=None, stream=None):
    """(mask, bricks, counts[interfacial, masked, bricks, escaped]) of a
    state's flags (ebit_refine_band); counts is a device int64 tensor.
    `out`: the (mask, bricks, counts, work) tensors of an earlier call to
    reuse."""
    n = flags.shape[0]
    if out is None:
        out = (torch.empty_like(flags), torch.empty((n // 4,) * 3, dtype=torch.uint8, device=flags.device),
               torch.empty(4, dtype=torch.int64, device=flags.device),
               torch.empty(lib().ebit_refine_work_bytes(n), dtype=torch.uint8, device=flags.device))
    mask, bricks, counts, work = out
    rc = lib().ebit_refine_band(n, _ptr(flags), _ptr(mask_prev), _ptr(mask), _ptr(bricks), _ptr(counts),
                                _ptr(work), work.numel(), _stream(stream))
    if rc != EBIT_OK:
        raise EbitError(rc, "ebit_refine_band")
    return mask, bricks, counts


# ----------------------------------------------------------------------------
# learned Front2VOF surrogate
# ----------------------------------------------------------------------------

def _check(rc, what):
    if rc != EBIT_OK:
        raise EbitError(rc, what)


def mlp_param_count() -> int:
    return lib().ebit_mlp_param_count()


def mlp_forward(theta, x_bf16, y=None, stream=None):
    """theta: float32 device vector; x_bf16: (m, 32) bfloat16 device rows."""
    m = x_bf16.shape[0]
    if y is None:
        y = torch.empty(m, dtype=torch.float32, device=x_bf16.device)
    _check(lib().ebit_mlp_forward(_ptr(theta), _ptr(x_bf16), m, _ptr(y), _stream(stream)), "ebit_mlp_forward")
    return y


def mlp_gradient_static(theta, x_bf16, c, grad, loss=None, stream=None):
    """ebit_mlp_gradient_static: the gradient into `grad` (and the loss into
    `loss`) with the library's static work space (at most
    EBIT_MLP_STATIC_MAX_ROWS rows, no allocation by the library)."""
    _check(lib().ebit_mlp_gradient_static(_ptr(theta), _ptr(x_bf16), _ptr(c), x_bf16.shape[0], _ptr(grad),
                                          _ptr(loss), _stream(stream)), "ebit_mlp_gradient_static")
    return grad, loss


class MlpTrainer:
    """Device buffers for gradient / Adam steps of the surrogate."""

    def __init__(self, theta, device="cuda"):
        self.theta = theta
        n = mlp_param_count()
        self.m1 = torch.zeros(n, dtype=torch.float32, device=device)
        self.m2 = torch.zeros(n, dtype=torch.float32, device=device)
        self.grad = torch.zeros(n, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.scratch = torch.empty(lib().ebit_mlp_scratch_bytes(), dtype=torch.uint8, device=device)
        self.t = 0

    def gradient(self, x_bf16, c, stream=None):
        L = lib()
        _check(L.ebit_mlp_gradient(_ptr(self.theta), _ptr(x_bf16), _ptr(c), x_bf16.shape[0], _ptr(self.grad),
                                   _ptr(self.loss), _ptr(self.scratch), self.scratch.numel(), _stream(stream)),
               "ebit_mlp_gradient")
        return self.grad, self.loss

    def step(self, x_bf16, c, lr, stream=None):
        self.gradient(x_bf16, c, stream)
        self.t += 1
        _check(lib().ebit_mlp_adam(_ptr(self.theta), _ptr(self.m1), _ptr(self.m2), _ptr(self.grad), self.t,
                                   float(lr), _stream(stream)), "ebit_mlp_adam")
        return self.loss

    def train(self, x_bf16, c, idx, lrs, stream=None):
        """len(lrs) steps in one native call; step s uses rows
        idx[s * batch:(s + 1) * batch] (idx: int64 device tensor of
        len(lrs) x batch entries in [0, rows)).  Returns the per-step losses
        (device tensor)."""
        steps = len(lrs)
        nrows = x_bf16.shape[0]
        if idx.dtype != torch.int64 or not idx.is_contiguous() or steps == 0 or idx.numel() % steps:
            raise ValueError("idx must be a contiguous int64 tensor of steps x batch entries")
        if int(idx.min()) < 0 or int(idx.max()) >= nrows:
            raise ValueError("row index out of range")
        batch = idx.numel() // steps
        lr = (ctypes.c_float * steps)(*[float(v) for v in lrs])
        lrp = ctypes.cast(lr, ctypes.c_void_p)
        losses = torch.empty(steps, dtype=torch.float32, device=self.theta.device)
        _check(lib().ebit_mlp_train(_ptr(self.theta), _ptr(self.m1), _ptr(self.m2), _ptr(x_bf16), _ptr(c), nrows,
                                    _ptr(idx), batch, steps, lrp, self.t, _ptr(losses), _ptr(self.scratch),
                                    self.scratch.numel(), _stream(stream)), "ebit_mlp_train")
        self.t += steps
        return losses

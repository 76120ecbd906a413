"""ctypes wrapper of the CPU FP64 oracle (``ebit_oracle.c``).

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use this module.  It never touches the HIP
library and the HIP library never touches it.

State arrays follow the shared layout (numpy ``(n, n, n)`` arrays indexed
``[k, j, i]``): ``flags`` uint8 and three float64 fraction arrays ``s[0..2]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ebit_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

# -O2 without contraction or fast-math: every operation rounds as written
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def build_variant(source: str, workdir: str):
    """Compile oracle source text (e.g. a copy with a deliberately planted
    mistake, for tests that show a pin detects it) into ``workdir`` and return
    the loaded library; the oracle itself is not touched."""
    src = os.path.join(workdir, "variant.c")
    so = os.path.join(workdir, "libvariant.so")
    with open(src, "w") as f:
        f.write(source)
    subprocess.check_call(["gcc", *CFLAGS, "-o", so, src, "-lm"])
    return _declare(ctypes.CDLL(so))


def source() -> str:
    with open(_SRC) as f:
        return f.read()


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _declare(ctypes.CDLL(_SO))
    return _lib


def _declare(L):
    """Argument and result types of the exported functions."""
    P = ctypes.c_void_p
    L.orc_init.argtypes = [ctypes.c_int] + [P] * 11
    L.orc_init.restype = ctypes.c_int
    L.orc_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            P, P, P, P, P, P, P, P, P, P]
    L.orc_sweep.restype = ctypes.c_int
    L.orc_f2v.argtypes = [ctypes.c_int, P, P, P, P, P, P]
    L.orc_f2v.restype = None
    L.orc_volume.argtypes = [ctypes.c_long, P, P]
    L.orc_volume.restype = ctypes.c_double
    L.orc_count_interfacial.argtypes = [ctypes.c_int, P]
    L.orc_count_interfacial.restype = ctypes.c_long
    L.orc_fit_height.argtypes = [P, P]
    L.orc_fit_height.restype = ctypes.c_double
    L.orc_cell_loops.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, P, P, P]
    L.orc_cell_loops.restype = ctypes.c_int
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class State:
    n: int
    flags: np.ndarray
    s: list

    def copy(self):
        return State(self.n, self.flags.copy(), [x.copy() for x in self.s])


def init(shape, exact: bool = False) -> State:
    """Markers and colours from a sampled shape (paper sec. 3.1).  With
    ``exact`` the markers sit at ``shape.s_exact`` instead of the linear zero."""
    n = shape.n
    flags = np.zeros((n, n, n), np.uint8)
    s = [np.zeros((n, n, n)) for _ in range(3)]
    phi = _f64(shape.phi_nodes)
    pf = [_f64(f) for f in shape.phi_faces]
    se = [_f64(x) for x in shape.s_exact] if exact else [None, None, None]
    rc = lib().orc_init(n, _p(phi), _p(pf[0]), _p(pf[1]), _p(pf[2]),
                        _p(se[0]), _p(se[1]), _p(se[2]),
                        _p(flags), _p(s[0]), _p(s[1]), _p(s[2]))
    if rc != 0:
        raise ValueError(f"orc_init failed ({rc}); n must be >= 8")
    return State(n, flags, s)


def sweep(st: State, d: int, g: float, dt: float, U, L=None) -> tuple:
    """One advection sweep along axis ``d`` (0, 1, 2); returns (new state,
    counters[fallback, multi-crossing, cfl, aligned-merges, of which
    annihilations]).  ``L``: a
    library from build_variant instead of the oracle."""
    n = st.n
    U = _f64(U)
    out = State(n, np.zeros_like(st.flags), [np.zeros_like(x) for x in st.s])
    cnt = np.zeros(5, np.int64)
    (L or lib()).orc_sweep(n, int(d), float(g), float(dt), _p(U), _p(st.flags),
                    _p(st.s[0]), _p(st.s[1]), _p(st.s[2]), _p(out.flags),
                    _p(out.s[0]), _p(out.s[1]), _p(out.s[2]), _p(cnt))
    return out, cnt


def step(st: State, Uxyz, g: float, dt: float, order=(0, 1, 2)) -> tuple:
    """Three sweeps x, y, z at the same time level (one time step)."""
    tot = np.zeros(5, np.int64)
    for d in order:
        st, c = sweep(st, d, g, dt, Uxyz[d])
        tot += c
    return st, tot


def f2v(st: State):
    """Volume fraction of every cell and the ambiguity mask (paper sec. 2.5)."""
    n = st.n
    C = np.zeros((n, n, n))
    amb = np.zeros((n, n, n), np.uint8)
    lib().orc_f2v(n, _p(st.flags), _p(st.s[0]), _p(st.s[1]), _p(st.s[2]), _p(C), _p(amb))
    return C, amb


def volume(C) -> tuple:
    """Compensated sum of C: (sum, compensation)."""
    C = _f64(C)
    comp = ctypes.c_double(0.0)
    s = lib().orc_volume(C.size, _p(C), ctypes.cast(ctypes.pointer(comp), ctypes.c_void_p))
    return s, comp.value


def count_interfacial(st: State) -> int:
    return int(lib().orc_count_interfacial(st.n, _p(st.flags)))


def fit_height(P1, P2, P3, P4) -> tuple:
    """Unaligned-marker rule for four points (test hook): returns (height of
    the new marker on the line X = 0, straight-line crossing of P2-P3)."""
    p = np.array([*P1, *P2, *P3, *P4], dtype=np.float64)
    key = ctypes.c_double(0.0)
    y = lib().orc_fit_height(_p(p), ctypes.cast(ctypes.pointer(key), ctypes.c_void_p))
    return y, key.value


def cell_loops(st: State, x: int, y: int, z: int) -> tuple:
    """Loops of one cell in traversal order (test hook): (list of (m,3)
    arrays in the cell frame, volume fraction)."""
    pts = np.zeros((12, 3))
    lens = np.zeros(6, np.int32)
    C = ctypes.c_double(0.0)
    k = lib().orc_cell_loops(st.n, _p(st.flags), _p(st.s[0]), _p(st.s[1]), _p(st.s[2]),
                             int(x), int(y), int(z), _p(pts), _p(lens),
                             ctypes.cast(ctypes.pointer(C), ctypes.c_void_p))
    out, o = [], 0
    for t in range(k):
        out.append(pts[o:o + lens[t]].copy())
        o += lens[t]
    return out, C.value

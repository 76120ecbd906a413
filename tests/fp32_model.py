"""A CPU model of the FP32 precision form: the oracle's own source with one
change -- the marker velocity is interpolated along its edge in FP32 and the
displacement formed in FP32 from the FP32 time factor; every later step
(advected positions, crossings, circle fits) stays in FP64.  Built on the CPU
into a temporary directory, like the planted-mistake variants: the oracle
itself is untouched."""
import os
import tempfile

from oracle import oracle as O

_OLD = '''                        double U0 = U[q], U1 = U[nidx3(n, r)];
                        double u = U0 + s[e][q] * (U1 - U0);
                        double delta = c * u;'''
_NEW = '''                        float U0f = (float)U[q], U1f = (float)U[nidx3(n, r)], sf = (float)s[e][q];
                        float uf = U0f + sf * (U1f - U0f);
                        double delta = (double)((float)c * uf);'''

_lib = None


def library():
    global _lib
    if _lib is None:
        src = O.source()
        assert src.count(_OLD) == 1, "the oracle's Euler step changed; update the FP32 model"
        d = tempfile.mkdtemp(prefix="ebit_fp32_model_")
        _lib = O.build_variant(src.replace(_OLD, _NEW), d)
        _lib._dir = d
    return _lib


def sweep(st, d, g, dt, U):
    return O.sweep(st, d, g, dt, U, L=library())

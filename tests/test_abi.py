"""Host-only checks of the C ABI: the library loads, exports every entry
point declared in include/ebit.h, and rejects bad arguments before any GPU
work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebit.h")
LIB = os.path.join(ROOT, "paper_2509_26361_amd", "libebit.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ebit_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libebit.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "ebit_init" in names and "ebit_advect_sweep" in names
    assert "ebit_front2vof" in names and "ebit_stats" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_scratch_size_rules(lib):
    lib.ebit_scratch_bytes.restype = ctypes.c_size_t
    assert lib.ebit_scratch_bytes(7) == 0
    assert lib.ebit_scratch_bytes(30) == 0
    assert lib.ebit_scratch_bytes(32) > 0
    assert lib.ebit_scratch_bytes(512) > lib.ebit_scratch_bytes(256)


def test_bad_arguments_rejected_on_host(lib):
    from paper_2509_26361_amd import ebit as E
    L = E.lib()
    ctx = ctypes.c_void_p(None)
    assert L.ebit_init(ctypes.byref(ctx), None, None, None, None, None) == E.EBIT_EINVAL
    d = E.Desc()
    d.n = 30
    assert L.ebit_init(ctypes.byref(ctx), ctypes.byref(d), None, None, None, None) == E.EBIT_EINVAL
    d.n = 32
    for b in range(2):
        d.flags[b] = 4096
        for e in range(3):
            d.s[b][e] = 4096
    d.scratch = 4096
    d.scratch_bytes = 16
    assert L.ebit_init(ctypes.byref(ctx), ctypes.byref(d), None, None, None, None) == E.EBIT_ESCRATCH
    d.precision = 7
    assert L.ebit_init(ctypes.byref(ctx), ctypes.byref(d), None, None, None, None) == E.EBIT_EINVAL
    assert not ctx
    assert L.ebit_advect_sweep(None, 0, None, 1.0, 0.1, None) == E.EBIT_EINVAL
    assert L.ebit_front2vof(None, None, None) == E.EBIT_EINVAL
    assert L.ebit_strerror(E.EBIT_ECFL).decode().startswith("Courant")


def test_mlp_entry_points_reject_bad_arguments_on_host(lib):
    """ebit_mlp_gradient / ebit_mlp_train argument checks (the pointers are
    never dereferenced: every call returns before any GPU work)."""
    from paper_2509_26361_amd import ebit as E
    L = E.lib()
    P = ctypes.c_void_p
    need = L.ebit_mlp_scratch_bytes()
    assert need > 256 * L.ebit_mlp_param_count() * 4        # partial sums of 256 workgroups and more
    ok, odd = P(4096), P(4100)                                # aligned / not 16-byte aligned
    lr = (ctypes.c_float * 4)(1e-3, 1e-3, 1e-3, 1e-3)
    lrp = ctypes.cast(lr, P)

    def train(theta=ok, x=ok, c=ok, nrows=100, idx=ok, batch=10, steps=4, lrs=lrp, step0=0, scratch=ok,
              nbytes=need):
        return L.ebit_mlp_train(theta, ok, ok, x, c, nrows, idx, batch, steps, lrs, step0, None, scratch, nbytes,
                                None)

    assert train(steps=0) == E.EBIT_OK                        # nothing to do
    assert train(theta=None) == E.EBIT_EINVAL
    assert train(x=None) == E.EBIT_EINVAL
    assert train(nrows=0) == E.EBIT_EINVAL
    assert train(batch=0) == E.EBIT_EINVAL
    assert train(steps=-1) == E.EBIT_EINVAL
    assert train(step0=-1) == E.EBIT_EINVAL
    assert train(lrs=None) == E.EBIT_EINVAL
    assert train(idx=None, batch=101) == E.EBIT_EINVAL         # rows 0..batch-1 must exist
    assert train(scratch=None) == E.EBIT_EINVAL
    assert train(scratch=odd) == E.EBIT_EINVAL
    assert train(nbytes=need - 1) == E.EBIT_ESCRATCH
    assert L.ebit_mlp_gradient(ok, ok, ok, 10, ok, None, odd, need, None) == E.EBIT_EINVAL
    assert L.ebit_mlp_gradient(ok, ok, ok, 10, ok, None, ok, need - 16, None) == E.EBIT_ESCRATCH
    assert L.ebit_mlp_gradient(ok, ok, ok, 0, ok, None, ok, need, None) == E.EBIT_EINVAL
    assert L.ebit_mlp_adam(ok, ok, ok, ok, 0, 1e-3, None) == E.EBIT_EINVAL


def test_static_gradient_rejects_bad_arguments_on_host(lib):
    """ebit_mlp_gradient_static checks its arguments before it looks up its
    static work space or enqueues anything."""
    from paper_2509_26361_amd import ebit as E
    L = E.lib()
    ok = ctypes.c_void_p(4096)
    assert L.ebit_mlp_gradient_static(ok, ok, ok, 0, ok, None, None) == E.EBIT_EINVAL
    assert L.ebit_mlp_gradient_static(None, ok, ok, 10, ok, None, None) == E.EBIT_EINVAL
    assert L.ebit_mlp_gradient_static(ok, ok, ok, E.EBIT_MLP_STATIC_MAX_ROWS + 1, ok, None, None) == E.EBIT_ETOOBIG
    assert L.ebit_strerror(E.EBIT_ETOOBIG).decode().startswith("input larger")

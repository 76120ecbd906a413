"""Height-function curvature and the CSF force (ebit_curvature, ebit_csf)
against the CPU oracle (oracle/curvature.py): exact ball fractions, the volume
fractions of the deformation run's Front2VOF at 128^3 and at the benchmark's
256^3 size, FP32 fields, a ragged grid and degenerate fields."""
import numpy as np
import pytest
import torch

from oracle import curvature as K
from oracle import oracle as O
from paper_2509_26361_amd import ebit as E
from paper_2509_26361_amd import inputs as I
from tests.exact_shapes import ball_fractions

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def compare(C, sigma=0.7, dtype=torch.float64, tol=0.0):
    """GPU and oracle on the same field C (numpy float64, already rounded to
    the precision's type); returns the oracle status array."""
    Cg = torch.from_numpy(np.ascontiguousarray(C)).to(dev()).to(dtype)
    kap, st = E.curvature(Cg)
    F = E.csf(Cg, kap, st, sigma)
    torch.cuda.synchronize()
    ko, so = K.curvature(C)
    Fo = K.csf(C, ko, so, sigma)
    sg = st.cpu().numpy()
    bad = np.argwhere(sg != so)
    assert len(bad) == 0, f"{len(bad)} status mismatches, first {bad[:3].tolist()}"
    kg = kap.cpu().numpy().astype(np.float64)
    scale = max(1.0, float(np.abs(ko).max()))
    assert np.max(np.abs(kg - ko)) <= tol * scale, np.max(np.abs(kg - ko))
    for d in range(3):
        fd = F[d].cpu().numpy().astype(np.float64)
        fs = max(1.0, float(np.abs(Fo[d]).max()))
        assert np.max(np.abs(fd - Fo[d])) <= tol * fs, (d, np.max(np.abs(fd - Fo[d])))
    return so


def test_ball_fp64_bit_exact():
    C = ball_fractions(32, (0.5123, 0.4871, 0.5032), 0.3)
    so = compare(C)
    assert np.count_nonzero(so == K.STATUS_HF) > 1000


def test_ball_fp32():
    C = ball_fractions(24, (0.5123, 0.4871, 0.5032), 0.3).astype(np.float32).astype(np.float64)
    compare(C, dtype=torch.float32, tol=1e-6)


def _deformation_C(n, steps):
    sh = I.sphere_shape(n)
    U = [torch.from_numpy(u).to(dev()) for u in I.deformation_velocity(n)]
    dt = 0.5 / n
    e = E.Ebit(n, "fp64", dev())
    e.init(torch.from_numpy(sh.phi_nodes).to(dev()), [torch.from_numpy(f).to(dev()) for f in sh.phi_faces])
    C = torch.zeros((n, n, n), dtype=torch.float64, device=dev())
    e.front2vof(C)
    e.advance(U, [I.deformation_time_factor(k * dt, 3.0) for k in range(steps)], dt, C)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def test_deformation_field_128():
    """Front2VOF's C of the stretched interface (height functions and the
    neighbour-mean fallback both occur)."""
    so = compare(_deformation_C(128, 250))
    for s in (K.STATUS_HF, K.STATUS_MEAN):
        assert np.count_nonzero(so == s) > 0, s


def test_full_size_256():
    """The benchmark's grid and state (256^3, after 200 steps), every cell."""
    so = compare(_deformation_C(256, 200), sigma=0.0728)
    assert np.count_nonzero(so) > 20000


def test_ragged_grid_and_degenerate_fields():
    # n = 10: 1000 cells, a partial last block
    C = ball_fractions(10, (0.47, 0.52, 0.5), 0.31)
    compare(C)
    n = 12
    # no interface: empty list, all zeros
    Cg = torch.ones((n, n, n), dtype=torch.float64, device=dev())
    kap, st = E.curvature(Cg)
    assert int(st.max()) == 0 and float(kap.abs().max()) == 0.0
    # every cell mixed: no valid column anywhere, status 4, curvature 0
    compare(np.full((n, n, n), 0.5))
    Cg = torch.full((n, n, n), 0.5, dtype=torch.float64, device=dev())
    kap, st = E.curvature(Cg)
    assert int(st.min()) == K.STATUS_MISSING and float(kap.abs().max()) == 0.0


def test_bad_arguments():
    n = 16
    C = torch.zeros((n, n, n), dtype=torch.float64, device=dev())
    L = E.lib()
    w = torch.empty(L.ebit_curvature_work_bytes(n), dtype=torch.uint8, device=dev())
    k = torch.empty_like(C)
    s = torch.empty(C.shape, dtype=torch.uint8, device=dev())
    assert L.ebit_curvature(n, 0, E._ptr(C), E._ptr(k), E._ptr(s), E._ptr(w), w.numel() - 1, None) == E.EBIT_ESCRATCH
    assert L.ebit_curvature(7, 0, E._ptr(C), E._ptr(k), E._ptr(s), E._ptr(w), w.numel(), None) == E.EBIT_EINVAL
    assert L.ebit_curvature(n, 5, E._ptr(C), E._ptr(k), E._ptr(s), E._ptr(w), w.numel(), None) == E.EBIT_EINVAL

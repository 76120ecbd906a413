"""Pins of the curvature / surface-force oracle (height functions and the
CSF term that couple Front2VOF's C to the flow solver, paper sec. 2.5)
against closed forms: exact volume fractions of planes and balls
(tests/exact_shapes.py) have known curvature 0, 2/R and -2/R, the height
function estimate converges to 2/R at second order, and the CSF force on a
half-space of the ball telescopes to the Laplace pressure jump 2 sigma / R on
its cross-section, -2 pi sigma R."""
import functools
import math

import numpy as np
import pytest

from oracle import curvature as K
from tests.exact_shapes import ball_fractions, plane_fractions

R = 0.3
CENTRE = (0.5123, 0.4871, 0.5032)


@functools.lru_cache(maxsize=None)
def ball(n, inside=True):
    return ball_fractions(n, CENTRE, R, inside)


def test_plane_has_zero_curvature():
    n = 24
    C = plane_fractions(n, (0.3, -0.5, 0.8), (0.5, 0.5, 0.5))
    kap, st = K.curvature(C)
    core = np.zeros(C.shape, bool)
    core[5:-5, 5:-5, 5:-5] = True                 # away from the wrap of the periodic grid
    hf = core & (st == K.STATUS_HF)
    assert hf.sum() > 300
    assert np.abs(kap[hf]).max() < 1e-12
    assert np.all(st[(C == 0.0) | (C == 1.0)] == K.STATUS_NONE)


def _sphere_error(n):
    kap, st = K.curvature(ball(n))
    m = (st >= K.STATUS_HF) & (st <= K.STATUS_MEAN)
    return float(np.mean(np.abs(kap[m] - 2.0 / R)) / (2.0 / R)), st


def test_sphere_curvature_converges_at_second_order():
    """Mean relative error over the cells with a curvature: about 1.9e-2,
    6.7e-3, 3.6e-3 at R/h = 4.8, 7.2, 9.6 (second order: x4 per halving)."""
    e16, st16 = _sphere_error(16)
    e24, _ = _sphere_error(24)
    e32, st32 = _sphere_error(32)
    assert e32 < 5e-3
    assert e16 / e32 > 3.5
    assert e16 > e24 > e32
    # most interfacial cells get a height-function curvature at R/h = 9.6
    inter = st32 > 0
    assert np.count_nonzero(st32 == K.STATUS_HF) > 0.65 * np.count_nonzero(inter)


def test_bubble_curvature_is_negative():
    """Phase 1 outside the ball: the interface is concave seen from phase 1."""
    kap, st = K.curvature(ball(24, inside=False))
    m = st == K.STATUS_HF
    assert abs(kap[m].mean() / (-2.0 / R) - 1.0) < 0.02


@pytest.mark.parametrize("sigma", [1.0, 0.07])
def test_csf_force_on_a_half_ball_is_the_laplace_jump(sigma):
    """Sum over the faces beyond the centre plane x = x_c of F_x h^3:
    sigma kappa_f times the telescoped jump of C along each x-line, which for
    kappa_f = 2/R is -sigma (2/R) (pi R^2)."""
    want = -2.0 * math.pi * sigma * R
    errs = []
    for n in (16, 32):
        C = ball(n)
        kap, st = K.curvature(C)
        F = K.csf(C, kap, st, sigma)
        h = 1.0 / n
        faces = np.arange(n) * h > CENTRE[0]      # F_x at cell i sits on the face x = i h
        tot = F[0][:, :, faces].sum() * h ** 3
        errs.append(abs(tot / want - 1.0))
        # no force across faces whose cells have equal C
        for d in range(3):
            same = C == np.roll(C, 1, axis=2 - d)
            assert np.all(F[d][same] == 0.0)
    assert errs[1] < 3e-3
    assert errs[1] < errs[0]


def test_csf_face_curvature_rule():
    """Face curvature: mean of the two cells' curvatures when both have one,
    the one that has it otherwise, 0 when neither."""
    n = 8
    C = np.zeros((n, n, n))
    C[2, 2, 3] = 0.25
    C[2, 2, 4] = 0.5
    C[2, 2, 6] = 0.75
    kap = np.zeros_like(C)
    st = np.zeros(C.shape, np.int8)
    kap[2, 2, 3], st[2, 2, 3] = 2.0, K.STATUS_HF
    kap[2, 2, 4], st[2, 2, 4] = 4.0, K.STATUS_MEAN
    kap[2, 2, 6], st[2, 2, 6] = 8.0, K.STATUS_MISSING
    F = K.csf(C, kap, st, 1.0)
    h = 1.0 / n
    assert F[0][2, 2, 4] == 3.0 * (0.5 - 0.25) / h          # both valid
    assert F[0][2, 2, 3] == 2.0 * 0.25 / h                  # only the cell at x = 3
    assert F[0][2, 2, 5] == 4.0 * (0.0 - 0.5) / h           # only the cell at x = 4
    assert F[0][2, 2, 6] == 0.0                             # status 4 has no curvature

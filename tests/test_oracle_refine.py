"""Pins of the refinement-band oracle (paper sec. 2.3): a brute-force loop
over cells on a small grid, the 3x3x3 block of one marked edge, and the
paper's argument -- with a Courant number of at most one per sweep the
interface stays inside the previous step's refined region -- checked on the
method itself, including the case that shows the check can fail (a move of
two cells)."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from oracle import refine as Rf
from paper_2509_26361_amd import inputs as I
from tests.ebit_states import make_state


def test_against_brute_force_loops():
    n = 8
    rng = np.random.default_rng(3)
    col = (rng.uniform(size=(n, n, n)) < 0.04).astype(np.uint8)
    st = make_state(col)
    f = st.flags
    want_int = np.zeros((n, n, n), bool)
    for k, j, i in itertools.product(range(n), repeat=3):
        for e in range(3):
            for oa in (0, 1):
                for ob in (0, 1):
                    off = [0, 0, 0]
                    others = [x for x in range(3) if x != e]
                    off[others[0]], off[others[1]] = oa, ob
                    q = ((k + off[2]) % n, (j + off[1]) % n, (i + off[0]) % n)
                    want_int[k, j, i] |= bool((f[q] >> (4 + e)) & 1)
    assert np.array_equal(Rf.interfacial(f), want_int)
    want_mask = np.zeros_like(want_int)
    for k, j, i in itertools.product(range(n), repeat=3):
        want_mask[k, j, i] = any(want_int[(k + dz) % n, (j + dy) % n, (i + dx) % n]
                                 for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    assert np.array_equal(Rf.refine_mask(f), want_mask)
    b = Rf.refine_bricks(want_mask)
    for bz, by, bx in itertools.product(range(2), repeat=3):
        assert b[bz, by, bx] == want_mask[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4].any()


def test_one_marked_edge():
    """A single phase-1 node: its 6 edges carry markers, the 8 cells around
    it are interfacial and the refined region is the 4^3 block of cells
    -2..1 around the node."""
    n = 12
    col = np.zeros((n, n, n), np.uint8)
    col[5, 6, 7] = 1
    f = make_state(col).flags
    it = Rf.interfacial(f)
    assert it.sum() == 8 and it[4:6, 5:7, 6:8].all()
    m = Rf.refine_mask(f)
    assert m.sum() == 64 and m[3:7, 4:8, 5:9].all()


@pytest.mark.parametrize("case", ["deformation", "random"])
def test_interface_stays_in_previous_refined_region(case):
    """Courant number up to one (sec. 2.3): after every step the interfacial
    cells lie inside the region refined around the previous step's."""
    if case == "deformation":
        n = 32
        st = O.init(I.sphere_shape(n))
        U = I.deformation_velocity(n)
        dt, gs = 0.5 / n, [1.0] * 12          # |lambda u| reaches 1 where |u| = 2
    else:
        n = 24
        st = O.init(I.random_shape(n, 9), exact=True)
        U = I.fourier_velocity(n, seed=10, modes=4)
        dt, gs = 1.0 / n, [1.0, -0.9, 0.8, 1.0, -1.0, 0.95]
    for g in gs:
        mask = Rf.refine_mask(st.flags)
        st, c = O.step(st, U, g, dt)
        assert c[2] == 0                       # no marker moved more than one cell
        assert Rf.escaped(st.flags, mask) == 0


def test_a_move_of_two_cells_escapes():
    """Two steps at Courant number one move a sphere by two cells per axis:
    against the region refined two steps earlier its interface escapes."""
    n = 24
    st = O.init(I.sphere_shape(n, centre=(0.5, 0.5, 0.5), R=0.2), exact=True)
    U = I.uniform_velocity(n)
    mask0 = Rf.refine_mask(st.flags)
    st, _ = O.step(st, U, 1.0, 1.0 / n)
    assert Rf.escaped(st.flags, mask0) == 0
    st, _ = O.step(st, U, 1.0, 1.0 / n)
    assert Rf.escaped(st.flags, mask0) > 0

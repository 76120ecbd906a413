"""Pins of the oracle's marker initialisation (paper sec. 3.1)."""
import numpy as np

from oracle import oracle as O
from paper_2509_26361_amd import inputs as I


def _edge_pairs(n, e):
    ax = 2 - e
    return lambda a: np.roll(a, -1, axis=ax)


def test_linear_markers_are_zeros_of_the_linear_interpolant():
    n = 32
    sh = I.sphere_shape(n)
    st = O.init(sh)
    phi = sh.phi_nodes
    col = st.flags & 1
    assert np.array_equal(col, (phi > 0).astype(np.uint8))
    for e in range(3):
        nxt = _edge_pairs(n, e)
        ex = ((st.flags >> (4 + e)) & 1).astype(bool)
        assert np.array_equal(ex, col != nxt(col))
        s = st.s[e][ex]
        pa, pb = phi[ex], nxt(phi)[ex]
        # phi_a + s (phi_b - phi_a) vanishes at the marker
        assert np.max(np.abs(pa + s * (pb - pa)) / np.abs(pb - pa)) < 1e-15
        assert np.all(st.s[e][~ex] == 0.0)


def test_exact_markers_lie_on_the_sphere():
    n = 32
    c, R = np.array([0.35, 0.35, 0.35]), 0.15
    st = O.init(I.sphere_shape(n, centre=tuple(c), R=R), exact=True)
    for e in range(3):
        ex = np.argwhere((st.flags >> (4 + e)) & 1)
        for k, j, i in ex:
            p = np.array([i, j, k], float)
            p[e] += st.s[e][k, j, i]
            assert abs(np.sum((p / n - c) ** 2) - R * R) < 1e-15


def test_face_colours_canonical_without_markers():
    n = 16
    st = O.init(I.random_shape(n, 3), exact=True)
    f = st.flags
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        eb = (f >> (4 + b)) & 1
        ec = (f >> (4 + c)) & 1
        anym = eb | np.roll(eb, -1, axis=2 - c) | ec | np.roll(ec, -1, axis=2 - b)
        face = (f >> (1 + a)) & 1
        assert np.array_equal(face[anym == 0], (f & 1)[anym == 0])

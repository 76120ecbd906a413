"""Pins of the oracle's face-centre colour update (paper sec. 2.2-2.4; the
rule itself is left to the 2D predecessor of the method, and the oracle reads
it as the phase at the face centre relative to the advected interface).

The brute force below is written from that statement alone, in numpy, with no
code shared with the oracle: it builds the old interface segments of every
face of a sweep plane, advects their end points, and finds the phase at each
face centre by counting crossings of straight paths from each of the face's
four new corners to its centre (the even-odd rule: the four answers must
agree).  The oracle's face bit must equal that phase on every face whose new
corners differ, equal the corner colour on the other faces of the plane, and
stay unchanged on the faces normal to the sweep axis.

Planting a mistake in a copy of the oracle (on the CPU) shows the pin has
teeth: dropping the flips from markers on the bottom line of the walk, or
inverting its side test, makes the comparison fail."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_26361_amd import inputs as I
from tests.ebit_states import roll_state

CORNERS = ((0, 0), (1, 0), (0, 1), (1, 1))


def _plane(arr, d, a):
    """View of a (z,y,x) array as [i_d, i_a, i_b] (numpy axis of spatial
    axis e is 2 - e)."""
    b = 3 - d - a
    return np.moveaxis(arr, (2 - d, 2 - a, 2 - b), (0, 1, 2))


def _bit(f, k):
    return ((f >> k) & 1).astype(np.int64)


def _face_segments(fl, s, U, d, a, lam_g):
    """Advected old segments of every face of the (d, a) planes, in the
    face's own frame (X along d from its lowest node, Y along a).  Returns
    (segs (n,n,n,2,4) = P.x, P.y, Q.x, Q.y; valid (n,n,n,2))."""
    b = 3 - d - a
    F = _plane(fl, d, a)
    Sd, Sa, Up = _plane(s[d], d, a), _plane(s[a], d, a), _plane(U, d, a)
    up_d = lambda x: np.roll(x, -1, axis=0)      # value at the next node along d
    up_a = lambda x: np.roll(x, -1, axis=1)
    # displacement of a marker on an edge: velocity linear along its own edge
    dd = lam_g * (Up + Sd * (up_d(Up) - Up))     # markers on d-edges
    da = lam_g * (Up + Sa * (up_a(Up) - Up))     # markers on a-edges
    has = np.stack([_bit(F, 4 + d), _bit(up_a(F), 4 + d), _bit(F, 4 + a), _bit(up_d(F), 4 + a)], -1)
    # points: bottom, top, left, right
    px = np.stack([Sd + dd, up_a(Sd) + up_a(dd), da, 1.0 + up_d(da)], -1)
    py = np.stack([np.zeros_like(Sd), np.ones_like(Sd), Sa, up_d(Sa)], -1)
    cnt = has.sum(-1)
    assert np.all((cnt == 0) | (cnt == 2) | (cnt == 4)), "odd marker count on a face"
    c00 = _bit(F, 0)
    face = _bit(F, 1 + b)
    segs = np.zeros(F.shape + (2, 4))
    valid = np.zeros(F.shape + (2,), bool)
    # two markers: the segment joining them
    two = cnt == 2
    order = np.argsort(-has, axis=-1, kind="stable")[..., :2]       # the two marked sides
    for t, k in enumerate((0, 1)):
        idx = order[..., k]
        X = np.take_along_axis(px, idx[..., None], -1)[..., 0]
        Y = np.take_along_axis(py, idx[..., None], -1)[..., 0]
        segs[..., 0, 2 * t] = np.where(two, X, 0.0)
        segs[..., 0, 2 * t + 1] = np.where(two, Y, 0.0)
    valid[..., 0] = two
    # four markers: the face colour names the phase at the centre; the two
    # corners of the other colour are cut off, each by the segment joining
    # the markers of the two sides that meet there
    four = cnt == 4
    keep_00 = face == c00                      # centre joined to corners 00 and 11
    B, T, L, R = 0, 1, 2, 3
    pairs_a = ((B, R), (T, L))                 # cut corners 10 and 01
    pairs_b = ((B, L), (T, R))                 # cut corners 00 and 11
    for t in range(2):
        for k in range(2):
            sa, sb = pairs_a[t][k], pairs_b[t][k]
            X = np.where(keep_00, px[..., sa], px[..., sb])
            Y = np.where(keep_00, py[..., sa], py[..., sb])
            segs[..., t, 2 * k] = np.where(four, X, segs[..., t, 2 * k])
            segs[..., t, 2 * k + 1] = np.where(four, Y, segs[..., t, 2 * k + 1])
    valid[..., 0] |= four
    valid[..., 1] = four
    return segs, valid


def _orient(ax, ay, bx, by, px, py):
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax)


def polyline_phase(old, new, U, d, a, lam_g, reach=3):
    """Phase at the centre of every face of the (d, a) planes, relative to the
    advected old segments of the faces of the same row, from each of the four
    new corners: returns (phase from corner 00, all four agree)."""
    segs, valid = _face_segments(old.flags, old.s, U, d, a, lam_g)
    Fn = _plane(new.flags, d, a)
    col = _bit(Fn, 0)
    corner_col = [np.roll(np.roll(col, -cx, axis=0), -cy, axis=1) for cx, cy in CORNERS]
    parity = [np.zeros(col.shape, np.int64) for _ in CORNERS]
    for o in range(-reach, reach + 1):
        S = np.roll(segs, -o, axis=0)
        V = np.roll(valid, -o, axis=0)
        for t in range(2):
            Px, Py = S[..., t, 0] + o, S[..., t, 1]
            Qx, Qy = S[..., t, 2] + o, S[..., t, 3]
            for k, (cx, cy) in enumerate(CORNERS):
                o1 = _orient(cx, cy, 0.5, 0.5, Px, Py)
                o2 = _orient(cx, cy, 0.5, 0.5, Qx, Qy)
                o3 = _orient(Px, Py, Qx, Qy, cx, cy)
                o4 = _orient(Px, Py, Qx, Qy, 0.5, 0.5)
                cross = V[..., t] & (o1 * o2 < 0) & (o3 * o4 < 0)
                parity[k] += cross
    phases = [(corner_col[k] + parity[k]) & 1 for k in range(4)]
    agree = (phases[0] == phases[1]) & (phases[0] == phases[2]) & (phases[0] == phases[3])
    uniform = (corner_col[0] == corner_col[1]) & (corner_col[0] == corner_col[2]) & (corner_col[0] == corner_col[3])
    return phases[0], agree, uniform, corner_col[0]


def check_face_colours(old, new, U, d, lam_g):
    """Compare the new face bits of a sweep along d with the brute force;
    returns (#faces compared, #mismatches, #corner-path disagreements,
    #uniform faces whose centre phase differs from their corners)."""
    compared = bad = disagree = pockets = 0
    for a in range(3):
        if a == d:
            continue
        b = 3 - d - a
        ph, agree, uniform, c00 = polyline_phase(old, new, U, d, a, lam_g)
        got = _bit(_plane(new.flags, d, a), 1 + b)
        mixed = ~uniform
        disagree += int(np.sum(mixed & ~agree))
        use = mixed & agree
        compared += int(use.sum())
        bad += int(np.sum(use & (got != ph)))
        # faces with one colour at all four corners take that colour
        bad += int(np.sum(uniform & (got != c00)))
        pockets += int(np.sum(uniform & agree & (ph != c00)))
    # faces normal to the sweep axis are not touched
    bad += int(np.sum(_bit(new.flags, 1 + d) != _bit(old.flags, 1 + d)))
    return compared, bad, disagree, pockets


def _random_case(seed, n=16):
    st = O.init(I.random_shape(n, seed), exact=True)
    U = I.fourier_velocity(n, seed=seed + 11, modes=4)
    return st, U


@pytest.mark.parametrize("seed", range(4))
def test_face_colours_are_the_phase_at_the_face_centre(seed):
    n = 16
    st, U = _random_case(seed, n)
    dt = 0.9 / n
    total = 0
    for d in (0, 1, 2):
        new, c = O.sweep(st, d, 1.0, dt, U[d])
        assert c[0] == 0 and c[2] == 0
        compared, bad, disagree, _ = check_face_colours(st, new, U[d], d, dt * n)
        assert disagree == 0, disagree
        assert bad == 0, (d, bad, compared)
        total += compared
        st = new
    assert total > 500


def _four_marker_faces(fl, a):
    """Faces with normal a carrying a marker on each of their four edges."""
    b, c = (a + 1) % 3, (a + 2) % 3
    m = _bit(fl, 4 + b) + _bit(np.roll(fl, -1, axis=2 - c), 4 + b) + _bit(fl, 4 + c) + \
        _bit(np.roll(fl, -1, axis=2 - b), 4 + c)
    return m == 4


def _saddle_state(seed, n=16):
    st = O.init(I.random_shape(n, seed, modes=4), exact=True)
    assert sum(int(_four_marker_faces(st.flags, a).sum()) for a in range(3)) > 20
    return st


@pytest.mark.parametrize("seed", [1, 2])
def test_zero_velocity_keeps_face_colours_of_four_marker_faces(seed):
    """With no motion the advected interface is the old one: on a 4-marker
    face the centre lies between the two cut-off corners, so its colour is
    kept; on every face the new bit is the brute-force phase."""
    n = 16
    st = _saddle_state(seed, n)
    zero = np.zeros((n, n, n))
    for d in range(3):
        new, c = O.sweep(st, d, 1.0, 0.5 / n, zero)
        assert c.sum() == 0
        for a in range(3):
            four = _four_marker_faces(st.flags, a)
            assert np.array_equal(_bit(new.flags, 1 + a)[four], _bit(st.flags, 1 + a)[four])
        compared, bad, disagree, pockets = check_face_colours(st, new, zero, d, 0.0)
        assert bad == 0 and disagree == 0 and pockets == 0 and compared > 100


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_unit_courant_shifts_face_colours(axis):
    """|lambda u| = 1 along the sweep axis: on the two face families that
    contain it, 4-marker faces carry the colours of the faces one cell behind;
    the family normal to it keeps its bits."""
    n = 16
    st = _saddle_state(3, n)
    U = np.ones((n, n, n))
    new, c = O.sweep(st, axis, 1.0, 1.0 / n, U)
    assert c[0] == 0 and c[2] == 0
    want = roll_state(st, 1, axis)
    for a in range(3):
        got = _bit(new.flags, 1 + a)
        if a == axis:
            assert np.array_equal(got, _bit(st.flags, 1 + a))
        else:
            four = _four_marker_faces(want.flags, a)
            assert four.sum() > 0
            assert np.array_equal(got[four], _bit(want.flags, 1 + a)[four])
    compared, bad, disagree, _ = check_face_colours(st, new, U, axis, 1.0)
    assert bad == 0 and disagree == 0


MUTATIONS = {
    # the walk along the bottom line ignores the markers it passes
    "no bottom-line flips": ("if (0.0 <= X && X < 0.5) par ^= 1;", "if (0) par ^= 1;"),
    # the walk up to the centre counts crossings above it instead of below
    "inverted side test": ("if (y < 0.5) par ^= 1;", "if (y >= 0.5) par ^= 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes_in_the_face_rule_are_caught(name, tmp_path):
    """A copy of the oracle with one mistake planted in its face-colour walk
    (CPU only) fails the brute-force comparison."""
    src = O.source()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1
    L = O.build_variant(src.replace(old, new), str(tmp_path))
    n = 16
    st, U = _random_case(0, n)
    dt = 0.9 / n
    bad_total = 0
    for d in (0, 1, 2):
        out, _ = O.sweep(st, d, 1.0, dt, U[d], L=L)
        _, bad, _, _ = check_face_colours(st, out, U[d], d, dt * n)
        bad_total += bad
        st = out
    assert bad_total > 0, name

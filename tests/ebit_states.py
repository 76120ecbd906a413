"""Test-side construction of hand-made EBIT states (no method arithmetic:
colours, markers and face colours are set directly, existence bits follow the
one-marker-per-edge invariant of the paper, sec. 2.2)."""
from __future__ import annotations

import numpy as np

from oracle.oracle import State


def make_state(colours, s=None, faces=None):
    """State from node colours (n,n,n) {0,1}, fractions s[3] and face
    colours faces[3]; an edge carries a marker iff its end colours differ."""
    c = np.asarray(colours, np.uint8) & 1
    n = c.shape[0]
    flags = c.copy()
    ss = []
    for e in range(3):
        ax = 2 - e                         # numpy axis of spatial axis e
        other = np.roll(c, -1, axis=ax)
        ex = (c != other)
        flags |= (ex.astype(np.uint8) << (4 + e))
        se = np.zeros((n, n, n)) if s is None else np.where(ex, s[e], 0.0)
        ss.append(np.ascontiguousarray(se, dtype=np.float64))
    if faces is not None:
        for a in range(3):
            flags |= (np.asarray(faces[a], np.uint8) & 1) << (1 + a)
    else:
        for a in range(3):
            flags |= c << (1 + a)
    return State(n, np.ascontiguousarray(flags), ss)


def roll_state(st, shift, axis_xyz):
    """Periodic shift of a whole state by `shift` nodes along spatial axis."""
    ax = 2 - axis_xyz
    return State(st.n, np.roll(st.flags, shift, axis=ax), [np.roll(x, shift, axis=ax) for x in st.s])


def permute_state(st, perm):
    """Relabel spatial axes: new axis perm[e] <- old axis e (a rotation or
    reflection of the cube that only permutes axes)."""
    n = st.n
    # numpy axes are (z, y, x) = spatial (2, 1, 0)
    inv = [0, 0, 0]
    for e in range(3):
        inv[perm[e]] = e
    # new array axis for spatial axis E is 2-E; it takes old spatial axis inv[E]
    np_axes = tuple(2 - inv[2 - t] for t in range(3))
    fl = np.transpose(st.flags, np_axes)
    newfl = fl & 1
    for e in range(3):
        newfl |= ((fl >> (4 + e)) & 1) << (4 + perm[e])
        newfl |= ((fl >> (1 + e)) & 1) << (1 + perm[e])
    s = [None] * 3
    for e in range(3):
        s[perm[e]] = np.ascontiguousarray(np.transpose(st.s[e], np_axes))
    return State(n, np.ascontiguousarray(newfl.astype(np.uint8)), s)


def reflect_state(st, axis_xyz):
    """Mirror x_a -> -x_a (periodic).  Node i -> -i; an edge along a from
    node i (fraction s) becomes the edge from node -i-1 with fraction 1-s;
    a face normal to a at x_a = i moves to node -i; faces along a move to -i-1."""
    n = st.n
    ax = 2 - axis_xyz
    idx = (-np.arange(n)) % n              # node i -> -i
    idx1 = (-np.arange(n) - 1) % n         # edge/cell i -> -i-1
    take_node = np.argsort(idx)
    take_edge = np.argsort(idx1)
    fl = st.flags
    col = np.take(fl & 1, take_node, axis=ax)
    out = col.copy()
    s = [None] * 3
    for e in range(3):
        eb = (fl >> (4 + e)) & 1
        if e == axis_xyz:
            eb2 = np.take(eb, take_edge, axis=ax)
            se = np.take(st.s[e], take_edge, axis=ax)
            se = np.where(eb2 == 1, np.minimum(1.0 - se, 0.9999999999999998), 0.0)
        else:
            eb2 = np.take(eb, take_node, axis=ax)
            se = np.take(st.s[e], take_node, axis=ax)
        out |= eb2 << (4 + e)
        s[e] = np.ascontiguousarray(se)
    for a in range(3):
        fb = (fl >> (1 + a)) & 1
        fb2 = np.take(fb, take_node if a == axis_xyz else take_edge, axis=ax)
        out |= fb2 << (1 + a)
    return State(n, np.ascontiguousarray(out.astype(np.uint8)), s)


def reflect_cells(C, axis_xyz):
    n = C.shape[0]
    ax = 2 - axis_xyz
    idx1 = (-np.arange(n) - 1) % n
    return np.take(C, np.argsort(idx1), axis=ax)

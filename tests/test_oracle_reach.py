"""How far one sweep's changes reach from the markers present at its start,
measured on the oracle (no GPU).  The GPU band narrows its neighbour claims
by this reach when it knows the next sweep's axis D'; this test pins the
reach on the method itself, independently of the GPU code.

Positions are those of the node storing a marker (the lower end of its
edge) and of the node whose flags or fractions changed, periodic:
- from a marker on an edge along D': -1..+1 along D', -1..0 across it;
- from a marker on an edge across D': -2..+1 along D', 0 across it;
- besides, nodes of bricks (4^3) the previous sweep changed (faces normal
  to the previous axis keep a colour that the next sweep may correct)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_26361_amd import inputs as I


def _shifted_or(mask, axis_offsets):
    """OR of the mask rolled by every offset tuple (offsets along x, y, z;
    numpy axis 2 - e is spatial axis e)."""
    out = np.zeros_like(mask)
    for off in axis_offsets:
        out |= np.roll(mask, shift=(off[2], off[1], off[0]), axis=(0, 1, 2))
    return out


def _reach(flags, dn):
    """Nodes a sweep along dn can change, from the markers in `flags`."""
    an, bn = (dn + 1) % 3, (dn + 2) % 3
    along = ((flags >> (4 + dn)) & 1).astype(bool)
    across = (((flags >> (4 + an)) & 1) | ((flags >> (4 + bn)) & 1)).astype(bool)
    offs_along, offs_across = [], []
    for dd in range(-2, 2):
        for da in (-1, 0):
            for db in (-1, 0):
                o = [0, 0, 0]
                o[dn], o[an], o[bn] = dd, da, db
                if dd >= -1:
                    offs_along.append(tuple(o))
                if da == 0 and db == 0:
                    offs_across.append(tuple(o))
    return _shifted_or(along, offs_along) | _shifted_or(across, offs_across)


def _bricks(mask):
    """Every node of a 4^3 brick holding a node of the mask."""
    n = mask.shape[0]
    b = mask.reshape(n // 4, 4, n // 4, 4, n // 4, 4).any(axis=(1, 3, 5))
    return np.repeat(np.repeat(np.repeat(b, 4, 0), 4, 1), 4, 2)


def _changed(a, b):
    ch = a.flags != b.flags
    for k in range(3):
        ch |= a.s[k] != b.s[k]
    return ch


@pytest.mark.parametrize("case", [("random", 1, 0.5), ("random", 2, 1.0), ("random", 3, 0.9),
                                  ("sphere", 4, 1.0)])
def test_sweep_changes_stay_within_marker_reach(case):
    kind, seed, courant = case
    n = 20
    sh = I.random_shape(n, seed) if kind == "random" else I.sphere_shape(n, centre=(0.4, 0.45, 0.55), R=0.22)
    U = I.fourier_velocity(n, seed=seed + 10)           # max |u| = 1
    dt = courant / n
    st = O.init(sh)
    prev_changed = np.zeros((n, n, n), bool)
    checked = 0
    for step in range(4):
        for d in range(3):
            out, cnt = O.sweep(st, d, 1.0, dt, U[d])
            assert cnt[2] == 0                            # within the Courant limit
            ch = _changed(st, out)
            allowed = _reach(st.flags, d) | _bricks(prev_changed)
            bad = np.argwhere(ch & ~allowed)
            assert len(bad) == 0, f"step {step} axis {d}: {len(bad)} changes out of reach, e.g. {bad[:3].tolist()}"
            checked += int(ch.sum())
            prev_changed = ch
            st = out
    assert checked > 1000

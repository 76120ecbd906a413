"""CPU oracle of the AMR-compatible refinement band (paper sec. 2.3, the
paragraph on tree-based adaptive refinement): every cell of the 3x3x3 block
around an interfacial cell is refined to the finest level; with a Courant
number of at most one, the next step's interfacial cells stay inside that
region, so the interface never reaches a cell of another level.

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the HIP library never does, and the two share no code.

Layout: flags (n, n, n) uint8 indexed [k, j, i] (x fastest), periodic; bit
4 + e marks a marker on the edge along axis e from node (i, j, k).  A cell
(i, j, k) is interfacial when any of its 12 edges carries a marker (sec. 2.2:
the cell holds interface segments).  READING (block-structured refinement):
the refined region is kept as 4^3-cell bricks, a brick refined when any of its
cells is.
"""
from __future__ import annotations

import numpy as np


def interfacial(flags):
    """Cells with a marker on any of their 12 edges, (n, n, n) bool."""
    f = np.asarray(flags)
    out = np.zeros(f.shape, bool)
    for e in range(3):
        m = ((f >> (4 + e)) & 1).astype(bool)
        a, b = [2 - x for x in range(3) if x != e]       # numpy axes of the two other spatial axes
        out |= m | np.roll(m, -1, axis=a) | np.roll(m, -1, axis=b) | np.roll(np.roll(m, -1, axis=a), -1, axis=b)
    return out


def refine_mask(flags):
    """Cells within the 3x3x3 block around an interfacial cell."""
    it = interfacial(flags)
    mask = np.zeros_like(it)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                mask |= np.roll(it, (dz, dy, dx), axis=(0, 1, 2))
    return mask


def refine_bricks(mask):
    """4^3-cell bricks holding a refined cell, (n/4, n/4, n/4) bool."""
    n = mask.shape[0]
    b = n // 4
    return mask.reshape(b, 4, b, 4, b, 4).any(axis=(1, 3, 5))


def escaped(flags, mask_prev):
    """Interfacial cells of a state outside an earlier refined region."""
    return int(np.count_nonzero(interfacial(flags) & ~np.asarray(mask_prev, bool)))

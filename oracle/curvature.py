"""CPU FP64 oracle of interface curvature by height functions and of the
continuum-surface-force term built from it.

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the HIP library never does, and the two share no code.

The paper couples the volume fraction C of Front2VOF (sec. 2.5) to the flow
solver through a well-balanced continuum-surface-force (CSF) term whose
curvature comes from the generalised height-function method (sec. 2.5, the
coupling paragraph).  The paper gives no formulas for either; what follows is
the standard construction, with each choice that the paper leaves open
marked READING.

Layout: C is an (n, n, n) array indexed [k, j, i] (x fastest), periodic,
cell size h = 1/n.  The numpy axis of spatial axis d is 2 - d.

Curvature of a cell with 0 < C < 1:
  1. Normal estimate (READING: Youngs' 3x3x3 gradient): g_d = sum over the
     3x3 cells across d, weights (1,2,1) x (1,2,1), of C(+1) - C(-1) along d.
     Candidate directions d in order of decreasing |g_d| (ties: lower axis).
  2. For direction d: 9 columns (offsets a, b in {-1,0,1} on the two other
     axes, in increasing axis order), each the 7 cells k = -3..3 along d from
     the cell's own layer.  A column is valid when its end cells hold 1 and 0
     exactly (READING: full and empty ends); its orientation o = +1 when the
     phase-1 end is at k = -3, -1 when at k = +3, and all 9 must agree.
     Height of the interface above the centre of layer 0, in cells:
        z = (sum_k C_k) - 7/2   (o = +1),      z = 7/2 - sum_k C_k   (o = -1),
     the 7 values added in order k = -3..3.
  3. With z_ab the height of column (a, b):
        za = (z_{1,0} - z_{-1,0}) / 2,   zb = (z_{0,1} - z_{0,-1}) / 2,
        zaa = z_{1,0} - 2 z_{0,0} + z_{-1,0},   zbb likewise,
        zab = (z_{1,1} - z_{1,-1} - z_{-1,1} + z_{-1,-1}) / 4,
        kappa = -o (zaa (1 + zb^2) + zbb (1 + za^2) - 2 zab za zb)
                / ((1 + za^2 + zb^2)^(3/2) h),
     the mean-curvature sum of the surface z(a, b), positive where phase 1 is
     convex (2/R for a sphere of phase 1).  The first candidate direction
     whose 9 columns are valid gives the cell's curvature (status 1 for the
     first candidate, 2 for a later one).
  4. READING (the paper's generalised method falls back to other estimates):
     a cell with no valid direction takes the mean of the curvatures of its 26
     neighbours that got one in step 3 (status 3), summed in [k, j, i] order;
     with none it gets 0 (status 4).
Cells with C = 0 or 1 get curvature 0 and status 0.

CSF term on the faces (READING: the face curvature is the mean of the valid
cell curvatures beside the face; Basilisk's well-balanced form): the force on
the face between cell p - e_d and cell p, stored at p, is
    F_d(p) = sigma kappa_f (C(p) - C(p - e_d)) / h,
kappa_f = mean of the curvatures of those two cells that have status 1-3
(one or both), else 0.
"""
from __future__ import annotations

import math

import numpy as np

STATUS_NONE, STATUS_HF, STATUS_HF_OTHER, STATUS_MEAN, STATUS_MISSING = 0, 1, 2, 3, 4


def _at(C, x, y, z):
    n = C.shape[0]
    return C[z % n, y % n, x % n]


def _youngs(C, p):
    """Youngs' gradient of C at cell p = (x, y, z)."""
    g = [0.0, 0.0, 0.0]
    for d in range(3):
        t1, t2 = [a for a in range(3) if a != d]
        acc = 0.0
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                w = (2 - abs(a)) * (2 - abs(b))
                q = list(p)
                q[t1] += a
                q[t2] += b
                up, dn = list(q), list(q)
                up[d] += 1
                dn[d] -= 1
                acc += w * (_at(C, *up) - _at(C, *dn))
        g[d] = acc
    return g


def _heights(C, p, d):
    """Heights z[a+1][b+1] and orientation of the 9 columns along d at p,
    or None when a column is invalid or orientations differ."""
    t1, t2 = [a for a in range(3) if a != d]
    z = [[0.0] * 3 for _ in range(3)]
    orient = 0
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            col = []
            for k in range(-3, 4):
                q = list(p)
                q[t1] += a
                q[t2] += b
                q[d] += k
                col.append(float(_at(C, *q)))
            if col[0] == 1.0 and col[6] == 0.0:
                o = 1
            elif col[0] == 0.0 and col[6] == 1.0:
                o = -1
            else:
                return None
            if orient and o != orient:
                return None
            orient = o
            s = 0.0
            for v in col:
                s += v
            z[a + 1][b + 1] = s - 3.5 if o == 1 else 3.5 - s
    return z, orient


def _kappa_from_heights(z, o, h):
    za = (z[2][1] - z[0][1]) / 2.0
    zb = (z[1][2] - z[1][0]) / 2.0
    zaa = z[2][1] - 2.0 * z[1][1] + z[0][1]
    zbb = z[1][2] - 2.0 * z[1][1] + z[1][0]
    zab = (z[2][2] - z[2][0] - z[0][2] + z[0][0]) / 4.0
    num = zaa * (1.0 + zb * zb) + zbb * (1.0 + za * za) - 2.0 * zab * za * zb
    t = 1.0 + za * za + zb * zb
    den = t * math.sqrt(t)                     # t^(3/2)
    return -o * num / (den * h)


def curvature(C):
    """Curvature (1/length, unit-cube units) and status of every cell."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    h = 1.0 / n
    kap = np.zeros_like(C)
    status = np.zeros(C.shape, np.int8)
    cells = np.argwhere((C > 0.0) & (C < 1.0))          # rows (k, j, i), in index order
    for k, j, i in cells:
        p = (int(i), int(j), int(k))
        g = _youngs(C, p)
        order = sorted(range(3), key=lambda d: (-abs(g[d]), d))
        for rank, d in enumerate(order):
            hz = _heights(C, p, d)
            if hz is None:
                continue
            kap[k, j, i] = _kappa_from_heights(hz[0], hz[1], h)
            status[k, j, i] = STATUS_HF if rank == 0 else STATUS_HF_OTHER
            break
        else:
            status[k, j, i] = STATUS_MISSING
    # fallback: mean of the neighbours with a height-function curvature
    for k, j, i in cells:
        if status[k, j, i] != STATUS_MISSING:
            continue
        s, m = 0.0, 0
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    q = ((k + dz) % n, (j + dy) % n, (i + dx) % n)
                    if status[q] in (STATUS_HF, STATUS_HF_OTHER):
                        s += kap[q]
                        m += 1
        if m:
            kap[k, j, i] = s / m
            status[k, j, i] = STATUS_MEAN
    return kap, status


def csf(C, kap, status, sigma):
    """Face forces F[d] (arrays like C): sigma kappa_f (C(p) - C(p - e_d)) / h
    on the face between p - e_d and p."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    h = 1.0 / n
    valid = (status >= STATUS_HF) & (status <= STATUS_MEAN)
    F = []
    for d in range(3):
        ax = 2 - d
        Cm = np.roll(C, 1, axis=ax)
        km = np.roll(kap, 1, axis=ax)
        vm = np.roll(valid, 1, axis=ax)
        both = valid & vm
        kf = np.where(both, (kap + km) / 2.0, np.where(valid, kap, np.where(vm, km, 0.0)))
        F.append(sigma * kf * (C - Cm) / h)
    return F

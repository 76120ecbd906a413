"""Exact cell volume fractions of simple shapes, for pinning the curvature
oracle (test-side only; no method arithmetic).

* Half-spaces n . x < alpha: the closed form of the volume of a unit cube cut
  by a plane (inclusion-exclusion of the corner tetrahedra, n_i > 0).
* Balls: per cell, the area of the disk section x = const intersected with
  the cell's (y, z) rectangle, in closed form, integrated along x by adaptive
  quadrature split at every radius where that area is not smooth.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate


def _cube_cut(m, alpha):
    """Volume of {x in [0,1]^3 : m . x <= alpha} for m_i > 0."""
    m1, m2, m3 = m
    if alpha <= 0.0:
        return 0.0
    if alpha >= m1 + m2 + m3:
        return 1.0
    tot = 0.0
    for sgn, shift in ((1, 0.0), (-1, m1), (-1, m2), (-1, m3), (1, m1 + m2), (1, m1 + m3), (1, m2 + m3),
                       (-1, m1 + m2 + m3)):
        t = alpha - shift
        if t > 0:
            tot += sgn * t ** 3
    return min(1.0, max(0.0, tot / (6.0 * m1 * m2 * m3)))


def plane_fractions(n, normal, point):
    """C of the half-space {(x - point) . normal < 0} (phase 1 there) on an
    n^3 unit-cube grid, [k, j, i] layout, no periodic wrap (the plane must
    keep its cells away from the boundary in the region used)."""
    nv = np.asarray(normal, dtype=np.float64)
    h = 1.0 / n
    C = np.zeros((n, n, n))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                lo = np.array([i, j, k], dtype=np.float64) * h
                # map the cell to [0,1]^3 with every normal component positive
                m = np.abs(nv) * h
                corner = lo + h * (nv < 0)
                alpha = float(np.dot(nv, np.asarray(point) - corner))
                C[k, j, i] = _cube_cut(m, alpha)
    return C


def _G(X, Y, r):
    """Area of the disk |(s, t)| <= r intersected with {s <= X, t <= Y}."""
    if X <= -r or Y <= -r or r <= 0.0:
        return 0.0
    X, Y = min(X, r), min(Y, r)
    w = lambda s: math.sqrt(max(r * r - s * s, 0.0))
    I = lambda s: 0.5 * (s * w(s) + r * r * math.asin(max(-1.0, min(1.0, s / r))))
    sY = w(Y)                      # |s| beyond which the chord top is below Y (Y >= 0)
    if Y >= 0.0:
        tot = 0.0
        a = min(X, -sY)            # s in [-r, -sY]: full chord 2 w(s)
        if a > -r:
            tot += 2.0 * (I(a) - I(-r))
        lo, hi = -sY, min(X, sY)   # s in [-sY, sY]: chord cut at Y
        if hi > lo:
            tot += Y * (hi - lo) + (I(hi) - I(lo))
        if X > sY:                 # s in [sY, X]: full chord again
            tot += 2.0 * (I(X) - I(sY))
        return tot
    lo, hi = -sY, min(X, sY)       # only |s| <= sY reaches above -|Y|
    if hi <= lo:
        return 0.0
    return Y * (hi - lo) + (I(hi) - I(lo))


def disk_rect_area(r, a0, a1, b0, b1):
    """Area of the disk of radius r at the origin inside [a0,a1] x [b0,b1]."""
    return _G(a1, b1, r) - _G(a0, b1, r) - _G(a1, b0, r) + _G(a0, b0, r)


def ball_fractions(n, centre, R, inside=True):
    """C of a ball (phase 1 inside, or outside with inside=False) on an n^3
    unit-cube grid, [k, j, i] layout; the ball must not cross the boundary."""
    h = 1.0 / n
    C = np.zeros((n, n, n)) if inside else np.ones((n, n, n))
    c = np.asarray(centre, dtype=np.float64)
    lo_i = [int(math.floor((c[a] - R) * n)) - 1 for a in range(3)]
    hi_i = [int(math.floor((c[a] + R) * n)) + 1 for a in range(3)]
    for k in range(lo_i[2], hi_i[2] + 1):
        for j in range(lo_i[1], hi_i[1] + 1):
            for i in range(lo_i[0], hi_i[0] + 1):
                x0, x1 = i * h - c[0], (i + 1) * h - c[0]
                y0, y1 = j * h - c[1], (j + 1) * h - c[1]
                z0, z1 = k * h - c[2], (k + 1) * h - c[2]
                near = math.sqrt(sum(max(0.0, lo_, -hi_) ** 2 for lo_, hi_ in ((x0, x1), (y0, y1), (z0, z1))))
                far = math.sqrt(sum(max(lo_ * lo_, hi_ * hi_) for lo_, hi_ in ((x0, x1), (y0, y1), (z0, z1))))
                a, b = max(x0, -R), min(x1, R)
                if far <= R:
                    vol = h ** 3
                elif near >= R or a >= b:
                    vol = 0.0
                else:
                    # radii at which the section's area is not smooth
                    rads = {abs(y0), abs(y1), abs(z0), abs(z1)}
                    rads |= {math.hypot(yy, zz) for yy in (y0, y1) for zz in (z0, z1)}
                    pts = sorted(s * math.sqrt(R * R - q * q) for q in rads if q < R for s in (-1, 1)
                                 if a < s * math.sqrt(R * R - q * q) < b)
                    f = lambda x: disk_rect_area(math.sqrt(max(R * R - x * x, 0.0)), y0, y1, z0, z1)
                    edges = [a] + pts + [b]
                    vol = 0.0
                    for u, v in zip(edges[:-1], edges[1:]):
                        with warnings.catch_warnings():
                            warnings.simplefilter("ignore", integrate.IntegrationWarning)
                            val, _ = integrate.quad(f, u, v, epsabs=1e-13 * h ** 3, epsrel=1e-11, limit=50)
                        vol += val
                frac = min(1.0, max(0.0, vol / h ** 3))
                C[k % n, j % n, i % n] = frac if inside else 1.0 - frac
    return C

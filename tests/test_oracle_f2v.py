"""Pins of the oracle's Front2VOF (paper sec. 2.5) against closed forms,
invariants and brute force, independent of the oracle's own formula."""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_26361_amd import inputs as I
from tests.ebit_states import make_state, permute_state, reflect_state, reflect_cells


def plane_cube_volume(nrm, alpha):
    """Volume of {x in [0,1]^3 : nrm.x < alpha} by inclusion-exclusion over
    the cube corners (the standard closed form for a plane cut of a cube)."""
    nrm = np.array(nrm, dtype=float)
    a = float(alpha)
    for e in range(3):
        if nrm[e] < 0:
            a -= nrm[e]
            nrm[e] = -nrm[e]
    tot = 0.0
    for v in itertools.product((0, 1), repeat=3):
        t = a - float(np.dot(nrm, v))
        if t > 0:
            tot += (-1) ** sum(v) * t ** 3
    return tot / (6.0 * nrm[0] * nrm[1] * nrm[2])


def test_single_corner_tetrahedra():
    """One phase-1 node: each of its 8 cells holds a tetrahedron whose legs
    are the marker distances from that node; volume = product / 6."""
    n = 8
    col = np.zeros((n, n, n), np.uint8)
    col[4, 4, 4] = 1
    rng = np.random.default_rng(3)
    s = [rng.uniform(0.05, 0.95, size=(n, n, n)) for _ in range(3)]
    st = make_state(col, s)
    C, amb = O.f2v(st)
    for dz, dy, dx in itertools.product((0, 1), repeat=3):
        # cell (4-dx, 4-dy, 4-dz) has the node as its corner (dx, dy, dz)
        cx, cy, cz = 4 - dx, 4 - dy, 4 - dz
        legs = []
        for e, dd in zip(range(3), (dx, dy, dz)):
            # edge along e touching the node inside this cell starts at node-e_e if dd else at node
            p = [4, 4, 4]
            if dd:
                p[e] -= 1
            f = s[e][p[2], p[1], p[0]]
            legs.append(1.0 - f if dd else f)
        want = legs[0] * legs[1] * legs[2] / 6.0
        assert abs(C[cz, cy, cx] - want) < 1e-15, (dx, dy, dz)
    assert amb.sum() == 0
    # every other cell is empty
    mask = np.ones_like(C, bool)
    mask[3:5, 3:5, 3:5] = False
    assert np.all(C[mask] == 0.0)


@pytest.mark.parametrize("seed", range(6))
def test_plane_cuts_match_closed_form(seed):
    """A plane cut with exact markers: the fan of a planar polygon is exact,
    so every cell equals the analytic plane-cube volume."""
    rng = np.random.default_rng(seed)
    n = 10
    nrm = rng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    nrm = np.where(np.abs(nrm) < 0.15, 0.15 * np.sign(nrm + 1e-300), nrm)
    alpha = float(nrm @ np.array([4.3, 4.6, 4.1]))
    ii = np.arange(n, dtype=float)
    X = ii[None, None, :]
    Y = ii[None, :, None]
    Z = ii[:, None, None]
    val = nrm[0] * X + nrm[1] * Y + nrm[2] * Z
    col = (val < alpha).astype(np.uint8)
    s = [np.clip((alpha - val) / nrm[e], 0.0, 1.0) for e in range(3)]
    st = make_state(col, s)
    C, amb = O.f2v(st)
    checked = 0
    for k in range(n - 1):
        for j in range(n - 1):
            for i in range(n - 1):
                want = plane_cube_volume(nrm, alpha - (nrm[0] * i + nrm[1] * j + nrm[2] * k))
                assert abs(C[k, j, i] - want) < 1e-12, (i, j, k, C[k, j, i], want)
                checked += 1
    assert checked == (n - 1) ** 3
    assert amb[: n - 1, : n - 1, : n - 1].sum() == 0


@pytest.mark.parametrize("kappa", [0.11, -0.11, 0.2, -0.03])
def test_face_centre_colour_selects_pairing(kappa):
    """Saddle phi = -(x-4.5)(y-4.5) + kappa, extruded along z: the face of
    cell (4,4) carries four markers and its centre phase is [kappa > 0]
    (sec. 2.2, 2.4).  kappa > 0 joins the phase-1 corners (1,0),(0,1) through
    the centre and cuts off the other two: C = 1 - (1/2 - 2 kappa)^2; kappa < 0
    cuts off the phase-1 corners: C = (1/2 + 2 kappa)^2 (triangle areas)."""
    n = 10
    ii = np.arange(n, dtype=float)

    def phi_at(ox, oy, oz):
        x = (ii + ox)[None, None, :]
        y = (ii + oy)[None, :, None]
        return np.broadcast_to(-(x - 4.5) * (y - 4.5) + kappa, (n, n, n)).copy()

    sh = I.Shape(n, phi_at(0, 0, 0), [phi_at(0, .5, .5), phi_at(.5, 0, .5), phi_at(.5, .5, 0)],
                 [np.zeros((n, n, n))] * 3)
    st = O.init(sh)                      # phi is linear along each edge: exact markers
    C, amb = O.f2v(st)
    want = 1.0 - (0.5 - 2 * kappa) ** 2 if kappa > 0 else (0.5 + 2 * kappa) ** 2
    for k in range(n):
        assert abs(C[k, 4, 4] - want) < 1e-14
        assert amb[k, 4, 4] == 1


def _random_state(n, seed):
    sh = I.random_shape(n, seed)
    return O.init(sh, exact=True)


@pytest.mark.parametrize("seed", range(4))
def test_complement(seed):
    """Swapping the phases (all corner and face colours) gives 1 - C."""
    st = _random_state(12, seed)
    C, _ = O.f2v(st)
    st2 = st.copy()
    st2.flags = st2.flags ^ np.uint8(0b1111)
    C2, _ = O.f2v(st2)
    assert np.max(np.abs(C + C2 - 1.0)) < 1e-13


@pytest.mark.parametrize("seed", range(2))
def test_cube_symmetries(seed):
    """C is invariant under the 48 symmetries of the cube (axis permutations
    times reflections) applied to the whole state."""
    st = _random_state(10, seed)
    C, _ = O.f2v(st)
    for perm in itertools.permutations(range(3)):
        sp = permute_state(st, perm)
        Cp, _ = O.f2v(sp)
        # transpose C the same way
        inv = [0, 0, 0]
        for e in range(3):
            inv[perm[e]] = e
        axes = tuple(2 - inv[2 - t] for t in range(3))
        assert np.max(np.abs(Cp - np.transpose(C, axes))) < 1e-13, perm
        for refl in range(8):
            sr = sp
            Cr = np.transpose(C, axes)
            for a in range(3):
                if refl >> a & 1:
                    sr = reflect_state(sr, a)
                    Cr = reflect_cells(Cr, a)
            Cs, _ = O.f2v(sr)
            assert np.max(np.abs(Cs - Cr)) < 1e-12, (perm, refl)


def _seg_tri_hits(P, Q, A, B, Cc):
    """Vectorised segment P->Q (arrays (m,3)) vs triangle ABC intersection
    (Moller-Trumbore restricted to the segment)."""
    e1 = B - A
    e2 = Cc - A
    d = Q - P
    h = np.cross(d, e2)
    a = h @ e1
    ok = np.abs(a) > 1e-14
    f = np.where(ok, 1.0 / np.where(ok, a, 1.0), 0.0)
    s = P - A
    u = f * np.einsum("ij,ij->i", s, h)
    q = np.cross(s, e1)
    v = f * np.einsum("ij,ij->i", q, d)
    t = f * (q @ e2)
    return ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0) & (t < 1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_point_sampling(seed):
    """Point sampling: a point's phase is the colour of cell corner (0,0,0)
    flipped once per fan triangle crossed on the way there (the interface
    inside a cell is exactly the fan).  Cells with a single loop."""
    st = _random_state(10, seed + 20)
    C, amb = O.f2v(st)
    m = 20
    g = (np.arange(m) + 0.5) / m + 1e-7
    pts = np.stack(np.meshgrid(g, g * 0.999 + 3e-4, g * 0.998 + 7e-4, indexing="ij"), -1).reshape(-1, 3)
    tested = 0
    for k in range(10):
        for j in range(10):
            for i in range(10):
                loops, c = O.cell_loops(st, i, j, k)
                if len(loops) != 1:
                    continue
                L = loops[0]
                G = L.mean(axis=0)
                q = np.zeros(3)
                par = np.zeros(len(pts), np.int64)
                for t in range(len(L)):
                    hit = _seg_tri_hits(pts, np.broadcast_to(q, pts.shape), G, L[(t + 1) % len(L)], L[t])
                    par ^= hit.astype(np.int64)
                col0 = st.flags[k, j, i] & 1
                frac = np.mean(par ^ col0)
                assert abs(frac - c) < 0.03, (i, j, k, frac, c)
                tested += 1
                if tested >= 25:
                    return
    assert tested > 5


def test_sphere_volume_second_order():
    """Exact-root markers on a sphere: sum of C converges to 4/3 pi R^3 at
    second order in h (polyhedral approximation of a smooth surface)."""
    errs = []
    for n in (16, 32, 64):
        sh = I.sphere_shape(n, centre=(0.5, 0.5, 0.5), R=0.3)
        st = O.init(sh, exact=True)
        C, _ = O.f2v(st)
        V = sum(O.volume(C)) / n ** 3
        errs.append(abs(V - 4.0 / 3.0 * math.pi * 0.3 ** 3))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def test_neumaier_sum_matches_exact():
    """Compensated sum against an exact (fsum) reference: volume-fraction-like
    data within 2 ulp; adversarial data within the Neumaier bound
    2u|S| + 2 n u^2 sum|x|."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(0, 1, 200000), np.ones(50000), np.zeros(50000)])
    rng.shuffle(x)
    s, c = O.volume(x)
    exact = math.fsum(x)
    assert abs((s + c) - exact) <= 2 * np.spacing(exact)
    y = np.concatenate([rng.uniform(0, 1, 100000), [1e16, -1e16, 3.0, 1e-9] * 10])
    rng.shuffle(y)
    s, c = O.volume(y)
    exact = math.fsum(y)
    u = 2.0 ** -53
    bound = 2 * u * abs(exact) + 2 * len(y) * u * u * np.sum(np.abs(y))
    assert abs((s + c) - exact) <= bound
    assert abs(np.sum(y) - exact) > bound      # the plain sum is visibly worse

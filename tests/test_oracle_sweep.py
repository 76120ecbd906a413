"""Pins of the oracle's advection sweep (paper sec. 2.1-2.4) and of a whole
time step, against the paper's published errors, exact translations, closed
forms and an independent 1D brute force."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_26361_amd import inputs as I
from tests.ebit_states import make_state, roll_state

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
S_MAX = 1.0 - 2.0 ** -52


def _errors(n, centre, vel, dt, steps, gfun):
    sh = I.sphere_shape(n, centre=centre)
    st = O.init(sh)
    C0, _ = O.f2v(st)
    V0 = sum(O.volume(C0))
    em = 0.0
    tot = np.zeros(5, np.int64)
    for s in range(steps):
        st, c = O.step(st, vel, gfun(s, dt), dt)
        tot += c
        C, _ = O.f2v(st)
        V = sum(O.volume(C))
        em += abs(V - V0)
    return em / steps / V0, np.abs(C - C0).sum() / C0.sum(), tot, (V - V0) / V0


@pytest.mark.parametrize("n", [32, 64])
def test_translation_errors_match_paper_table2(n):
    """Translation with reversal at T/2, CFL 0.125 (sec. 3.1): the shape error
    matches Table 2 within 1 % at N = 32 and 64 (measured: 0.1 %).  The mass
    error is 1.42x (N = 32) and 1.69x (N = 64) the printed one; the band
    asserted here records that gap, whose cause is not identified."""
    ref = json.load(open(os.path.join(GOLDEN, "translation_table2.json")))
    k = ref["N"].index(n)
    dt = 0.125 / n
    steps = int(round(1.0 / dt))
    em, es, tot, _ = _errors(n, (0.25, 0.25, 0.25), I.uniform_velocity(n), dt, steps,
                          lambda s, dt: 1.0 if s < steps // 2 else -1.0)
    assert abs(es / ref["E_shape"][k] - 1.0) < 0.01, es
    assert 1.3 < em / ref["E_mass"][k] < 1.8, em
    assert tot[0] == 0 and tot[2] == 0


def test_deformation_errors_same_order_as_paper_table3():
    """3D deformation, T = 3, CFL 0.125 on v_max, N = 32 (sec. 3.2): a mass
    loss at T, as the paper reports for N = 32 and 64; errors below the
    printed ones at this under-resolved size (measured: E_shape 0.67x,
    E_mass 0.43x Table 3; at N = 128 the GPU path, identical to this oracle,
    gives E_shape within 1 % of Table 3)."""
    ref = json.load(open(os.path.join(GOLDEN, "deformation_table3.json")))
    n = 32
    dt = 0.125 / n
    steps = int(round(3.0 / dt))
    em, es, tot, dv = _errors(n, (0.35, 0.35, 0.35), I.deformation_velocity(n), dt, steps,
                              lambda s, dt: I.deformation_time_factor(s * dt, 3.0))
    assert dv < 0.0, dv
    assert 0.6 < es / ref["E_shape"][0] < 0.75, es
    assert 0.35 < em / ref["E_mass"][0] < 0.5, em
    assert tot[0] == 0 and tot[2] == 0


def test_translation_is_exact_for_exact_sphere_markers():
    """Sphere sections are circles, so the circle fit is exact (sec. 3.1.2):
    with markers exactly on the sphere, 20 steps at CFL 0.5 move the state by
    exactly 10 cells along each axis."""
    n = 32
    sh = I.sphere_shape(n)
    st0 = O.init(sh, exact=True)
    C0, _ = O.f2v(st0)
    st = st0
    for _ in range(20):
        st, c = O.step(st, I.uniform_velocity(n), 1.0, 0.5 / n)
        assert c[0] == 0 and c[2] == 0
    want = st0
    for a in range(3):
        want = roll_state(want, 10, a)
    colours = 0b1110001
    assert np.array_equal(st.flags & colours, want.flags & colours)
    for e in range(3):
        assert np.max(np.abs(st.s[e] - want.s[e])) < 1e-12
    C, _ = O.f2v(st)
    assert np.max(np.abs(C - np.roll(C0, (10, 10, 10), axis=(0, 1, 2)))) < 1e-12


@pytest.mark.parametrize("shape", ["sphere", "ellipsoid"])
def test_zero_velocity_leaves_state(shape):
    n = 24
    if shape == "sphere":
        sh = I.sphere_shape(n, centre=(0.47, 0.52, 0.49), R=0.31)
    else:
        rot = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))[0]
        sh = I.ellipsoids_shape(n, [(0.5, 0.5, 0.5)], [(0.35, 0.2, 0.27)], [rot])
    st = O.init(sh)
    zero = [np.zeros((n, n, n))] * 3
    st2, c = O.step(st, zero, 1.0, 0.5 / n)
    assert c.sum() == 0
    keep = 0b1110001
    assert np.array_equal(st2.flags & keep, st.flags & keep)
    for e in range(3):
        # markers that do not move stay exactly where they are
        assert np.array_equal(st2.s[e], st.s[e])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_unit_courant_shifts_one_cell(axis):
    """|lambda u| = 1 moves every marker exactly one cell along the sweep
    axis: the state is the old one shifted by one node."""
    n = 24
    rot = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))[0]
    sh = I.ellipsoids_shape(n, [(0.5, 0.45, 0.55)], [(0.33, 0.22, 0.27)], [rot])
    st = O.init(sh)
    U = np.ones((n, n, n))
    st2, c = O.sweep(st, axis, 1.0, 1.0 / n, U)
    assert c[0] == 0 and c[2] == 0
    want = roll_state(st, 1, axis)
    keep = 0b1110001
    assert np.array_equal(st2.flags & keep, want.flags & keep)
    for e in range(3):
        assert np.max(np.abs(st2.s[e] - want.s[e])) < 1e-12


def _line_bruteforce(col, pos_exists, pos_s, delta, n):
    """Aligned markers of one periodic line moved by a constant delta:
    colours are pulled back (new colour at node i = old phase at i - delta)
    and markers are binned per edge, an even count annihilating and three
    leaving the middle one (sec. 2.2).  Also returns the number of edges
    reached by more than one marker and, of those, by an even number."""
    Xold = [i + pos_s[i] for i in range(n) if pos_exists[i]]
    newcol = np.zeros(n, np.uint8)
    for i in range(n):
        x = i - delta
        i0 = math.floor(x)
        ph = col[i0 % n]
        for X in Xold:
            # unwrap the marker to the period containing [i0, x)
            for sh in (-n, 0, n):
                if i0 <= X + sh < x:
                    ph ^= 1
        newcol[i] = ph
    bins = {}
    for X in Xold:
        Xn = X + delta
        k = math.floor(Xn)
        bins.setdefault(k % n, []).append(Xn - k)
    ex = np.zeros(n, bool)
    s = np.zeros(n)
    merged = sum(1 for v in bins.values() if len(v) > 1)
    annihilated = sum(1 for v in bins.values() if len(v) > 1 and len(v) % 2 == 0)
    for k, v in bins.items():
        if len(v) % 2 == 1:
            ex[k] = True
            s[k] = sorted(v)[len(v) // 2]
    return newcol, ex, s, merged, annihilated


@pytest.mark.parametrize("seed", range(3))
def test_aligned_markers_and_colours_bruteforce(seed):
    """Independent per-line recount for a velocity constant along each line
    (dyadic values so every sum is exact): colours, markers, and the counts of
    edges reached by several markers and of annihilated pairs."""
    n = 16
    rng = np.random.default_rng(seed)
    sh = I.random_shape(n, seed + 40)
    col = (sh.phi_nodes > 0).astype(np.uint8)
    s = [np.floor(rng.uniform(0, 1, (n, n, n)) * 2 ** 20) / 2 ** 20 for _ in range(3)]
    st = make_state(col, s)
    total_annihilated = 0
    for d in range(3):
        f = rng.integers(-1024, 1025, size=(n, n)) / 1024.0
        shape = [n, n, n]
        shape[2 - d] = 1
        U = np.broadcast_to(f.reshape(shape), (n, n, n)).copy()
        st2, c = O.sweep(st, d, 1.0, 1.0 / n, U)
        assert c[0] == 0
        ax = 2 - d
        F = np.moveaxis(st.flags, ax, -1)
        S = np.moveaxis(st.s[d], ax, -1)
        F2 = np.moveaxis(st2.flags, ax, -1)
        S2 = np.moveaxis(st2.s[d], ax, -1)
        Uf = np.moveaxis(U, ax, -1)
        merged = annihilated = 0
        for a in range(n):
            for b in range(n):
                newcol, ex, sn, m, an = _line_bruteforce(F[a, b] & 1, (F[a, b] >> (4 + d)) & 1,
                                                         S[a, b], Uf[a, b, 0], n)
                merged += m
                annihilated += an
                assert np.array_equal(F2[a, b] & 1, newcol)
                assert np.array_equal(((F2[a, b] >> (4 + d)) & 1).astype(bool), ex)
                assert np.array_equal(np.where(ex, S2[a, b], 0.0), np.where(ex, sn, 0.0))
        assert c[3] == merged and c[4] == annihilated
        total_annihilated += annihilated
    assert total_annihilated > 0        # the counts are not vacuous


# --------------------------------------------------------------------------
# circle fit (sec. 2.1, Fig. 2)
# --------------------------------------------------------------------------

def _on_circle(c, r, t):
    return (c[0] + r * math.cos(t), c[1] + r * math.sin(t))


def _circle_through(P, Q, R):
    A = np.array([[Q[0] - P[0], Q[1] - P[1]], [R[0] - P[0], R[1] - P[1]]]) * 2.0
    b = np.array([Q[0] ** 2 - P[0] ** 2 + Q[1] ** 2 - P[1] ** 2,
                  R[0] ** 2 - P[0] ** 2 + R[1] ** 2 - P[1] ** 2])
    cen = np.linalg.solve(A, b)
    return cen, math.hypot(P[0] - cen[0], P[1] - cen[1])


def test_circle_fit_exact_on_a_circle():
    c, r = (0.3, 1.2), 0.9
    t2, t3 = -math.pi / 2 - 0.5, -math.pi / 2 + 0.2
    P = [_on_circle(c, r, t) for t in (t2 - 0.4, t2, t3, t3 + 0.4)]
    y, key = O.fit_height(*P)
    t = -math.acos(-c[0] / r)
    want = c[1] + r * math.sin(t)
    assert abs(y - want) < 1e-13
    assert abs(key - want) > 1e-3          # the chord alone is visibly off


def test_circle_fit_collinear_is_the_straight_crossing():
    P = [(-1.5, -0.25), (-0.5, 0.25), (0.5, 0.75), (1.5, 1.25)]
    y, key = O.fit_height(*P)
    assert y == key == 0.5


def test_circle_fit_radius_ratio_above_10_takes_larger_circle():
    cB, rB = (0.1, 20.4), 20.0
    P2 = _on_circle(cB, rB, -math.pi / 2 - 0.01)
    P3 = _on_circle(cB, rB, -math.pi / 2 + 0.01)
    P4 = _on_circle(cB, rB, -math.pi / 2 + 0.03)
    # a small circle (r ~ 0.5) through P2, P3 gives P1
    mid = ((P2[0] + P3[0]) / 2, (P2[1] + P3[1]) / 2)
    half = math.hypot(P3[0] - P2[0], P3[1] - P2[1]) / 2
    cA = (mid[0], mid[1] + math.sqrt(0.25 - half * half))
    tA = math.atan2(P2[1] - cA[1], P2[0] - cA[0]) - 0.6
    P1 = _on_circle(cA, 0.5, tA)
    cenA, rA = _circle_through(P1, P2, P3)
    assert rB / rA > 10
    y, key = O.fit_height(P1, P2, P3, P4)
    want = cB[1] - math.sqrt(rB * rB - cB[0] * cB[0])
    assert abs(y - want) < 1e-11


def test_circle_fit_mean_of_two_circles():
    """Radius ratio below 10: the new marker is the mean of both circle roots."""
    P1, P2, P3, P4 = (-1.2, 0.55), (-0.4, 0.2), (0.5, 0.3), (1.3, 0.9)
    roots = []
    for T in (P1, P4):
        cen, r = _circle_through(T, P2, P3)
        ys = [cen[1] - math.sqrt(r * r - cen[0] ** 2), cen[1] + math.sqrt(r * r - cen[0] ** 2)]
        # the root on the arc P2..P3 away from T: opposite side of the chord
        side_T = (P3[0] - P2[0]) * (T[1] - P2[1]) - (P3[1] - P2[1]) * (T[0] - P2[0])
        pick = [yy for yy in ys if ((P3[0] - P2[0]) * (yy - P2[1]) - (P3[1] - P2[1]) * (0 - P2[0])) * side_T < 0]
        assert len(pick) == 1
        roots.append((pick[0], r))
    assert max(roots[0][1], roots[1][1]) / min(roots[0][1], roots[1][1]) < 10
    y, _ = O.fit_height(P1, P2, P3, P4)
    assert abs(y - 0.5 * (roots[0][0] + roots[1][0])) < 1e-13


@pytest.mark.parametrize("seed", range(3))
def test_random_states_stay_consistent(seed):
    """Arbitrary states (saddles, thin necks, random marker positions) under
    a random smooth velocity with |lambda u| <= 1: no fallback, one marker
    exactly where the edge colours differ, faces without markers canonical."""
    n = 16
    st = O.init(I.random_shape(n, seed), exact=True)
    U = I.fourier_velocity(n, seed=seed + 5, modes=4)
    for d in range(3):
        st, c = O.sweep(st, d, 1.0, 1.0 / n, U[d])
        assert c[0] == 0 and c[2] == 0
        col = st.flags & 1
        for e in range(3):
            ex = (st.flags >> (4 + e)) & 1
            assert np.array_equal(ex, col ^ np.roll(col, -1, axis=2 - e))
            assert np.all(st.s[e][ex == 0] == 0.0)
            assert np.all((st.s[e] >= 0) & (st.s[e] <= S_MAX))

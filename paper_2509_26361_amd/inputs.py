"""Seeded synthetic workloads for the 3D EBIT hot path.

This module only describes *inputs*: interface shapes sampled at grid nodes and
face centres, the parameters of edge crossings of those shapes, and node
velocity fields.  It contains none of the method's arithmetic (no marker
placement rule, no colour rule, no advection, no volume computation); both the
HIP library and the CPU oracle consume exactly these arrays.

Conventions
-----------
* Periodic unit cube meshed by ``n**3`` cubic cells of size ``h = 1/n``.  Grid
  node ``(i, j, k)`` sits at ``(i, j, k) * h``.
* Every array has ``n**3`` entries, linear index ``i + n*(j + n*k)`` (x fastest);
  as a numpy array that is shape ``(n, n, n)`` indexed ``[k, j, i]``.
* ``phi`` is positive inside the reference phase (paper section 3.1: the
  signed quantity R^2 - |x - x_c|^2 sampled at cell vertices).
* ``phi_faces[a]`` samples the same function at the centre of the face whose
  normal is axis ``a`` and whose lowest corner is node ``(i, j, k)``.
* ``s_exact[e]`` is, for the edge along axis ``e`` that starts at node
  ``(i, j, k)``, the fraction in ``[0, 1]`` at which the analytic surface
  crosses that edge (only meaningful where the surface does cross it).

Velocity fields are node arrays of the *spatial* factor; a time factor ``g``
multiplies them per sweep (the deformation case of paper section 3.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Shape",
    "sphere_shape",
    "spheres_shape",
    "ellipsoids_shape",
    "random_shape",
    "uniform_velocity",
    "deformation_velocity",
    "deformation_time_factor",
    "fourier_velocity",
    "fourier_velocity_device",
    "random_nonoverlapping_spheres",
    "WORKLOADS",
]


@dataclass
class Shape:
    """Sampled description of an interface on an ``n**3`` periodic grid."""

    n: int
    phi_nodes: np.ndarray                      # (n,n,n) float64
    phi_faces: list = field(default_factory=list)   # 3 x (n,n,n) float64
    s_exact: list = field(default_factory=list)     # 3 x (n,n,n) float64 in [0,1]


def _coords(n):
    ax = np.arange(n, dtype=np.float64)
    return ax


def _sphere_phi_at(n, centre, R, off):
    """R^2 - |x - c|^2 at points (i+off0, j+off1, k+off2)*h, minimum image."""
    h = 1.0 / n
    ax = _coords(n)
    comps = []
    for a in range(3):
        x = (ax + off[a]) * h - centre[a]
        x = x - np.round(x)            # periodic minimum image in the unit cube
        comps.append(x * x)
    # broadcast to [k, j, i]
    return R * R - (comps[2][:, None, None] + comps[1][None, :, None] + comps[0][None, None, :])


def _sphere_edge_roots(n, centre, R):
    """Crossing fraction of each edge with a sphere (cell units, minimum image).

    For the edge along axis e starting at node p the line is p + t e_e; the
    sphere |x - c| = R meets it at t = c_e' +- sqrt(R'^2 - rho^2) (primes: cell
    units relative to p).  The root lying in the edge is returned; where the
    line misses the sphere 0.5 is returned (the value is then never used).
    """
    Rc = R * n
    ax = _coords(n)
    rel = []
    for a in range(3):
        x = ax - centre[a] * n
        x = x - n * np.round(x / n)    # minimum image, cell units
        rel.append(x)                 # node coordinate minus centre
    out = []
    for e in range(3):
        o = [b for b in range(3) if b != e]
        sq = [rel[b] ** 2 for b in range(3)]
        rho2 = np.zeros((n, n, n))
        for b in o:
            shape = [1, 1, 1]
            shape[2 - b] = n
            rho2 = rho2 + sq[b].reshape(shape)
        q = Rc * Rc - rho2
        shape = [1, 1, 1]
        shape[2 - e] = n
        pe = rel[e].reshape(shape) * np.ones((n, n, n))    # node coord - centre along e
        root = np.sqrt(np.maximum(q, 0.0))
        # node inside -> the crossing is the exit root (+), else the entry root (-)
        inside = (pe * pe + rho2) < Rc * Rc
        t = np.where(inside, root - pe, -root - pe)
        t = np.where(q >= 0.0, t, 0.5)
        out.append(np.clip(t, 0.0, 1.0))
    return out


def sphere_shape(n, centre=(0.35, 0.35, 0.35), R=0.15) -> Shape:
    """Single sphere (paper sections 3.1 and 3.2)."""
    phi = _sphere_phi_at(n, centre, R, (0.0, 0.0, 0.0))
    faces = [
        _sphere_phi_at(n, centre, R, (0.0, 0.5, 0.5)),
        _sphere_phi_at(n, centre, R, (0.5, 0.0, 0.5)),
        _sphere_phi_at(n, centre, R, (0.5, 0.5, 0.0)),
    ]
    return Shape(n, phi, faces, _sphere_edge_roots(n, centre, R))


def sphere_shape_device(n, centre=(0.35, 0.35, 0.35), R=0.15, device="cuda"):
    """sphere_shape evaluated with torch in float64 on a device (the same
    formulas, for grids too large to build on the host; equal to it up to an
    ulp of the exact roots).  Returns (phi_nodes, [phi_faces x3],
    [s_exact x3]) as (n,n,n) tensors."""
    import torch
    dt = torch.float64
    h = 1.0 / n
    ax = torch.arange(n, dtype=dt, device=device)

    def phi_at(off):
        comps = []
        for a in range(3):
            x = (ax + off[a]) * h - centre[a]
            x = x - torch.round(x)
            comps.append(x * x)
        return R * R - (comps[2][:, None, None] + comps[1][None, :, None] + comps[0][None, None, :])

    phi = phi_at((0.0, 0.0, 0.0))
    faces = [phi_at((0.0, 0.5, 0.5)), phi_at((0.5, 0.0, 0.5)), phi_at((0.5, 0.5, 0.0))]
    Rc = R * n
    rel = []
    for a in range(3):
        x = ax - centre[a] * n
        rel.append(x - n * torch.round(x / n))
    roots = []
    for e in range(3):
        o = [b for b in range(3) if b != e]
        rho2 = torch.zeros((n, n, n), dtype=dt, device=device)
        for b in o:
            shape = [1, 1, 1]
            shape[2 - b] = n
            rho2 = rho2 + (rel[b] * rel[b]).reshape(shape)
        q = Rc * Rc - rho2
        shape = [1, 1, 1]
        shape[2 - e] = n
        pe = rel[e].reshape(shape).expand(n, n, n)
        root = torch.sqrt(torch.clamp(q, min=0.0))
        inside = (pe * pe + rho2) < Rc * Rc
        t = torch.where(inside, root - pe, -root - pe)
        t = torch.where(q >= 0.0, t, torch.full_like(t, 0.5))
        roots.append(torch.clamp(t, 0.0, 1.0))
        del rho2, q, root, inside, t
    return phi, faces, roots


def spheres_shape(n, centres, radii, with_s=True) -> Shape:
    """Union of disjoint spheres: at each sample point the largest
    ``R^2 - |x-c|^2`` over the spheres, positive exactly inside the union.
    Each sphere is rasterised only over its bounding box (plus a margin) so
    512^3 grids with thousands of spheres stay cheap.  ``s_exact`` is not
    provided (0.5): these workloads use the paper's linear marker placement."""
    h = 1.0 / n
    phi = np.full((n, n, n), -1.0)
    faces = [np.full((n, n, n), -1.0) for _ in range(3)]
    offs = [(0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)]
    for c, R in zip(centres, radii):
        rc = int(math.ceil(R * n)) + 2
        lo = [int(math.floor(c[a] * n)) - rc for a in range(3)]
        idx = [np.arange(lo[a], lo[a] + 2 * rc + 2) for a in range(3)]
        wrapped = [np.mod(ix, n) for ix in idx]
        sel = np.ix_(wrapped[2], wrapped[1], wrapped[0])
        for which, off in enumerate(offs):
            comps = []
            for a in range(3):
                x = (idx[a] + off[a]) * h - c[a]
                comps.append(x * x)
            val = R * R - (comps[2][:, None, None] + comps[1][None, :, None] + comps[0][None, None, :])
            tgt = phi if which == 0 else faces[which - 1]
            tgt[sel] = np.maximum(tgt[sel], val)
    s = [np.full((n, n, n), 0.5) for _ in range(3)] if with_s else None
    return Shape(n, phi, faces, s)


def ellipsoids_shape(n, centres, semi_axes, rotations) -> Shape:
    """Union of disjoint ellipsoids given by centre, semi-axes (unit-cube
    units) and a 3x3 rotation each.  phi = 1 - |A^-1 R^T (x - c)|^2 scaled by
    the smallest semi-axis squared, which is positive exactly inside."""
    h = 1.0 / n
    phi = np.full((n, n, n), -1.0)
    faces = [np.full((n, n, n), -1.0) for _ in range(3)]
    offs = [(0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)]
    for c, ax, Rm in zip(centres, semi_axes, rotations):
        rc = int(math.ceil(max(ax) * n)) + 2
        lo = [int(math.floor(c[a] * n)) - rc for a in range(3)]
        idx = [np.arange(lo[a], lo[a] + 2 * rc + 2) for a in range(3)]
        wrapped = [np.mod(ix, n) for ix in idx]
        sel = np.ix_(wrapped[2], wrapped[1], wrapped[0])
        amin = min(ax)
        for which, off in enumerate(offs):
            X = [((idx[a] + off[a]) * h - c[a]) for a in range(3)]
            Z, Y, Xx = np.meshgrid(X[2], X[1], X[0], indexing="ij")
            P = np.stack([Xx, Y, Z], axis=-1) @ np.asarray(Rm)   # R^T (x - c)
            q = (P[..., 0] / ax[0]) ** 2 + (P[..., 1] / ax[1]) ** 2 + (P[..., 2] / ax[2]) ** 2
            val = (1.0 - q) * amin * amin
            tgt = phi if which == 0 else faces[which - 1]
            cur = tgt[sel]
            tgt[sel] = np.maximum(cur, val)
    s = [np.full((n, n, n), 0.5) for _ in range(3)]
    return Shape(n, phi, faces, s)


def random_shape(n, seed, modes=3, amp_faces=1.0, exact_uniform=True) -> Shape:
    """Smooth seeded random field (a few periodic Fourier modes) for stress
    tests: many blobs, saddles (4-marker faces) and thin necks.  ``s_exact`` is
    drawn uniformly in [0, 1) so edges carry arbitrary marker positions;
    ``phi_faces`` is an independent random field so face-centre phases vary."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    ax = np.arange(n) * h

    def field_(offs, rr):
        out = np.zeros((n, n, n))
        for _ in range(modes * 4):
            k = rr.integers(-modes, modes + 1, size=3)
            a = rr.normal()
            ph = rr.uniform(0, 2 * np.pi)
            arg = 2 * np.pi * (k[0] * (ax + offs[0] * h)[None, None, :]
                               + k[1] * (ax + offs[1] * h)[None, :, None]
                               + k[2] * (ax + offs[2] * h)[:, None, None])
            out += a * np.cos(arg + ph)
        return out

    base_state = rng.bit_generator.state
    phi = field_((0, 0, 0), np.random.Generator(np.random.PCG64(seed * 7919 + 1)))
    faces = [field_(o, np.random.Generator(np.random.PCG64(seed * 7919 + 2 + a)))
             * amp_faces for a, o in enumerate([(0, .5, .5), (.5, 0, .5), (.5, .5, 0)])]
    del base_state
    s = [rng.uniform(0.0, 1.0, size=(n, n, n)) for _ in range(3)]
    return Shape(n, phi, faces, s)


# ----------------------------------------------------------------------------
# velocity fields (node arrays of the spatial factor)
# ----------------------------------------------------------------------------

def uniform_velocity(n, u=(1.0, 1.0, 1.0)):
    """Constant velocity (paper section 3.1)."""
    return [np.full((n, n, n), float(c)) for c in u]


def deformation_velocity(n):
    """Spatial factor of LeVeque's 3D deformation field (paper section 3.2),
    sampled at the grid nodes."""
    x = np.arange(n) / n
    s1 = np.sin(np.pi * x)
    s2 = np.sin(2 * np.pi * x)
    X = (slice(None), None, None)
    ux = 2.0 * (s1 ** 2)[None, None, :] * s2[None, :, None] * s2[:, None, None]
    uy = -s2[None, None, :] * (s1 ** 2)[None, :, None] * s2[:, None, None]
    uz = -s2[None, None, :] * s2[None, :, None] * (s1 ** 2)[:, None, None]
    del X
    return [np.ascontiguousarray(ux), np.ascontiguousarray(uy), np.ascontiguousarray(uz)]


def deformation_time_factor(t, T=3.0):
    """Reversal factor cos(pi t / T): the field slows, reverses at T/2 and the
    interface returns to its start at t = T (paper section 3.2)."""
    return math.cos(math.pi * t / T)


def _fourier_modes(seed, modes):
    """The random draws of fourier_velocity: per component of A, `modes`
    (wave vector, amplitude, phase) triples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for comp in range(3):
        for _ in range(modes):
            while True:
                k = rng.integers(-8, 9, size=3)
                if np.any(k != 0):
                    break
            amp = rng.normal() / np.linalg.norm(k)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            out.append((comp, k, amp, ph))
    return out


# curl: u_x = dA_z/dy - dA_y/dz, u_y = dA_x/dz - dA_z/dx, u_z = dA_y/dx - dA_x/dy;
# (comp, b) -> (velocity component, sign) for dA_comp / dx_b
_CURL = {(2, 1): (0, 1.0), (1, 2): (0, -1.0), (0, 2): (1, 1.0), (2, 0): (1, -1.0), (1, 0): (2, 1.0), (0, 1): (2, -1.0)}


def fourier_velocity(n, seed=1, modes=8):
    """Seeded divergence-free periodic field u = curl A.

    A has ``modes`` random Fourier modes per component with integer wave
    vectors in {-8..8}^3 \\ 0, amplitudes N(0,1)/|k| and uniform phases; the
    curl is taken analytically at the nodes and the field is scaled so that
    the largest nodal speed is 1."""
    x = np.arange(n) / n
    u = [np.zeros((n, n, n)) for _ in range(3)]
    for comp, k, amp, ph in _fourier_modes(seed, modes):
        # A_comp = amp * cos(2 pi k.x + ph);  dA/dx_b = -amp 2 pi k_b sin(...), the
        # sine evaluated separably from 1D phase tables
        ex = [np.exp(1j * 2 * np.pi * k[a] * x) for a in range(3)]
        arg = (ex[2][:, None, None] * ex[1][None, :, None] * ex[0][None, None, :]) * np.exp(1j * ph)
        sn = arg.imag
        for b in range(3):
            if (comp, b) in _CURL:
                c, sg = _CURL[(comp, b)]
                u[c] += sg * (-amp * 2 * np.pi * k[b] * sn)
    mag = np.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2).max()
    return [np.ascontiguousarray(c / mag) for c in u]


def fourier_velocity_device(n, seed=1, modes=8, device="cuda", dtype=None):
    """The field of fourier_velocity (same draws), evaluated with torch on a
    device in float64 -- for grids where the host version is slow."""
    import torch
    dt = torch.float64
    x = torch.arange(n, dtype=dt, device=device) / n
    u = [torch.zeros((n, n, n), dtype=dt, device=device) for _ in range(3)]
    for comp, k, amp, ph in _fourier_modes(seed, modes):
        th = [2 * math.pi * float(k[a]) * x for a in range(3)]
        ang = th[2][:, None, None] + th[1][None, :, None] + th[0][None, None, :] + ph
        sn = torch.sin(ang)
        for b in range(3):
            if (comp, b) in _CURL:
                c, sg = _CURL[(comp, b)]
                u[c] += sg * (-amp * 2 * math.pi * float(k[b])) * sn
        del ang, sn
    mag = torch.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2).max()
    return [(c / mag).to(dtype or dt).contiguous() for c in u]


def random_nonoverlapping_spheres(count, rmin_cells, rmax_cells, n, gap_cells=2.0, seed=0,
                                  max_tries=200000):
    """Seeded random sphere packing in the periodic unit cube: radii
    U(rmin, rmax) cells, uniform centres, rejection so that surfaces are at
    least ``gap_cells`` apart.  Returns (centres, radii) in unit-cube units."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    cs = np.zeros((0, 3))
    rs = np.zeros(0)
    tries = 0
    cell = (2 * rmax_cells + gap_cells) * h
    ncell = max(1, int(1.0 / cell))
    buckets = {}
    while len(rs) < count and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin_cells, rmax_cells) * h
        c = rng.uniform(0.0, 1.0, size=3)
        b = tuple((c * ncell).astype(int) % ncell)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((b[0] + dx) % ncell, (b[1] + dy) % ncell, (b[2] + dz) % ncell)
                    for m in buckets.get(key, ()):
                        d = c - cs[m]
                        d -= np.round(d)
                        if np.sqrt(d @ d) < r + rs[m] + gap_cells * h:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            buckets.setdefault(b, []).append(len(rs))
            cs = np.vstack([cs, c])
            rs = np.append(rs, r)
    return cs, rs


def mlp_init(seed, nin=20, nh=128):
    """Seeded initial parameters of the surrogate network (He-uniform weights,
    zero biases), in the parameter order W1, b1, W2, b2, w3, b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.uniform(-1, 1, size=(nin, nh)) * math.sqrt(6.0 / nin)
    W2 = rng.uniform(-1, 1, size=(nh, nh)) * math.sqrt(6.0 / nh)
    w3 = rng.uniform(-1, 1, size=nh) * math.sqrt(6.0 / nh) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(nh), W2.ravel(), np.zeros(nh), w3, [0.0]])


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    shape: str
    velocity: str
    dt: float
    steps: int
    T: float = 3.0


def _wl_translation(n=32):
    # CFL 0.5 with |u| = 1: dt = h/2; 20 steps move the sphere by 10 cells
    return Workload("translation_32", n, "sphere", "uniform", 0.5 / n, 20)


def _wl_deformation(n):
    # dt from v_max = 1 at t = 0 and CFL 0.5: dt = h/2; T = 3 -> 6n steps
    return Workload(f"deformation_{n}", n, "sphere", "deformation", 0.5 / n, 6 * n, 3.0)


WORKLOADS = {
    "translation_32": _wl_translation(32),
    "deformation_128": _wl_deformation(128),
    "deformation_256": _wl_deformation(256),
    "deformation_64": _wl_deformation(64),
    "deformation_32": _wl_deformation(32),
}

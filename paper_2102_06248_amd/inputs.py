"""Seeded synthetic inputs: tetrahedral meshes and particle sets.

This module only *generates* inputs (node coordinates, tetrahedra, Cartesian particle
positions and momenta).  It holds none of the PIC method's arithmetic: no barycentric
coordinates, no Whitney forms, no assembly, no push.  Both the HIP library and the CPU
oracle consume what it produces, each through its own code.

Meshes stand in for the paper's (its beam cylinder and plasma ball meshes are not
published, Sec. IV-B/IV-C); shapes and sizes follow the workloads in ``workloads``.

All random draws use numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# Physical constants used only to turn energies/temperatures into momenta (CODATA 2018).
ELEMENTARY_CHARGE = 1.602176634e-19      # C
ELECTRON_MASS = 9.1093837015e-31         # kg
PROTON_ELECTRON_MASS_RATIO = 1836.0      # the round mass ratio the plasma workload names
SPEED_OF_LIGHT = 299792458.0             # m/s


# --------------------------------------------------------------------------- meshes

def kuhn_cube(n: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Box [lo, hi] split into n^3 cubes, each cut into the 6 Kuhn (Freudenthal) tets.

    Every tet of cube (i,j,k) is the monotone lattice path corner -> +e_a -> +e_b -> +e_c
    for a permutation (a,b,c) of the axes, so neighbouring cubes share face diagonals.
    Returns (xyz float64 [(n+1)^3, 3], tets int32 [6 n^3, 4]).
    Node id = i + (n+1) * (j + (n+1) * k).
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    m = n + 1
    g = np.arange(m, dtype=np.float64) / n
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    xyz = np.stack([g[i.ravel()], g[j.ravel()], g[k.ravel()]], axis=1)
    xyz = lo + xyz * (hi - lo)

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ck.ravel(), cj.ravel(), ci.ravel()       # cube order: i fastest

    def nid(a, b, c):
        return a + m * (b + m * c)

    tets = []
    unit = np.eye(3, dtype=np.int64)
    for perm in itertools.permutations(range(3)):
        p = np.zeros(3, dtype=np.int64)
        verts = [nid(ci, cj, ck)]
        for ax in perm:
            p = p + unit[ax]
            verts.append(nid(ci + p[0], cj + p[1], ck + p[2]))
        tets.append(np.stack(verts, axis=1))
    # interleave so the 6 tets of one cube are contiguous
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return xyz, tets


def kuhn_interior_nodes(n: int):
    """Boolean mask of nodes of kuhn_cube(n) not on the box surface."""
    m = n + 1
    idx = np.arange(m ** 3)
    i, j, k = idx % m, (idx // m) % m, idx // (m * m)
    return (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)


def jitter_nodes(xyz, movable_mask, h, frac, seed):
    """Move the nodes in movable_mask by a uniform random offset in [-frac*h, frac*h]^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = xyz.copy()
    d = rng.uniform(-frac * h, frac * h, size=(int(movable_mask.sum()), 3))
    out[movable_mask] += d
    return out


def hex_disk(radius: float, n_rings: int):
    """Disk triangulated in n_rings hexagonal rings: ring i has 6i nodes on the circle of
    radius radius*i/n_rings; 6 n_rings^2 triangles.  Returns (xy [n,2], tris int [t,3])."""
    pts = [(0.0, 0.0)]
    starts = [0]
    for i in range(1, n_rings + 1):
        starts.append(len(pts))
        r = radius * i / n_rings
        for kk in range(6 * i):
            a = 2.0 * math.pi * kk / (6 * i)
            pts.append((r * math.cos(a), r * math.sin(a)))
    tris = []
    for i in range(1, n_rings + 1):
        no, ni = 6 * i, 6 * (i - 1)

        def outer(q):
            return starts[i] + (q % no)

        def inner(q):
            return 0 if i == 1 else starts[i - 1] + (q % ni)

        for s in range(6):
            for jj in range(i):
                o0, o1 = outer(s * i + jj), outer(s * i + jj + 1)
                a = inner(s * (i - 1) + jj)
                tris.append((a, o0, o1))
                if jj < i - 1:
                    tris.append((a, o1, inner(s * (i - 1) + jj + 1)))
    return np.asarray(pts, dtype=np.float64), np.asarray(tris, dtype=np.int64)


def prism_cylinder(radius: float, length: float, n_rings: int, n_layers: int):
    """Cylinder r <= radius, 0 <= z <= length: hex_disk extruded in n_layers prism layers,
    each prism cut into 3 tets.  The cut of each prism follows the global order of its
    bottom nodes (diagonal of each side quad from the lower-numbered bottom node to the
    higher-numbered top node), which makes neighbouring prisms conforming.
    Returns (xyz [n,3], tets int32 [3 * 6 n_rings^2 * n_layers, 4])."""
    xy, tris = hex_disk(radius, n_rings)
    n2 = xy.shape[0]
    z = np.arange(n_layers + 1, dtype=np.float64) * (length / n_layers)
    xyz = np.concatenate([np.column_stack([xy, np.full(n2, zz)]) for zz in z], axis=0)
    tri = np.sort(tris, axis=1)
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    out = []
    for layer in range(n_layers):
        o0, o1 = layer * n2, (layer + 1) * n2
        A, B, C = a + o0, b + o0, c + o0
        A2, B2, C2 = a + o1, b + o1, c + o1
        t = np.stack([np.stack([A, B, C, C2], 1), np.stack([A, B, B2, C2], 1),
                      np.stack([A, A2, B2, C2], 1)], axis=1).reshape(-1, 4)
        out.append(t)
    return xyz, np.concatenate(out, axis=0).astype(np.int32)


# --------------------------------------------------------------------------- particles

def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gamma_from_kinetic(kinetic_eV, mass):
    return 1.0 + kinetic_eV * ELEMENTARY_CHARGE / (mass * SPEED_OF_LIGHT ** 2)


def thermal_sigma_v(T_eV, mass):
    """Per-component velocity spread sqrt(kT/m) of a Maxwellian."""
    return math.sqrt(T_eV * ELEMENTARY_CHARGE / mass)


def beam_particles(n, radius, z_lo, z_hi, kinetic_eV, thermal_eV, mass, seed):
    """Electron-beam macroparticles: uniform on a disk r <= radius (r = radius*sqrt(U)),
    z uniform in [z_lo, z_hi) (z_lo == z_hi puts them all on that plane), drift along +z
    at the given kinetic energy plus a Gaussian thermal spread per component.
    Returns x [n,3], u [n,3] with u = gamma v (m/s)."""
    g = _rng(seed)
    r = radius * np.sqrt(g.random(n))
    th = 2.0 * math.pi * g.random(n)
    z = np.full(n, z_lo) if z_hi == z_lo else z_lo + (z_hi - z_lo) * g.random(n)
    x = np.column_stack([r * np.cos(th), r * np.sin(th), z])
    gam = gamma_from_kinetic(kinetic_eV, mass)
    vz = SPEED_OF_LIGHT * math.sqrt(1.0 - 1.0 / gam ** 2)
    v = g.normal(0.0, thermal_sigma_v(thermal_eV, mass), size=(n, 3))
    v[:, 2] += vz
    gv = 1.0 / np.sqrt(1.0 - np.sum(v * v, axis=1) / SPEED_OF_LIGHT ** 2)
    return x, v * gv[:, None]


def gaussian_ball_pairs(n, sigma, trunc_sigmas, Te_eV, Ti_eV, m_e, m_i, seed, center=(0.0, 0.0, 0.0)):
    """Co-located electron/ion pairs (so the initial charge density is zero everywhere):
    positions from an isotropic Gaussian of width sigma truncated at trunc_sigmas*sigma
    (rejection), Maxwellian velocities at Te and Ti.
    Returns (x [n,3], u_e [n,3], u_i [n,3])."""
    g = _rng(seed)
    x = np.empty((0, 3))
    lim2 = (trunc_sigmas * sigma) ** 2
    while x.shape[0] < n:
        cand = g.normal(0.0, sigma, size=(int(1.2 * (n - x.shape[0])) + 16, 3))
        cand = cand[np.sum(cand * cand, axis=1) <= lim2]
        x = np.concatenate([x, cand], axis=0)
    x = x[:n] + np.asarray(center)
    ve = g.normal(0.0, thermal_sigma_v(Te_eV, m_e), size=(n, 3))
    vi = g.normal(0.0, thermal_sigma_v(Ti_eV, m_i), size=(n, 3))

    def mom(v):
        return v / np.sqrt(1.0 - np.sum(v * v, axis=1) / SPEED_OF_LIGHT ** 2)[:, None]

    return x, mom(ve), mom(vi)


def uniform_box_particles(n, lo, hi, sigma_v, seed):
    """Positions uniform in the box [lo, hi], Gaussian momenta (per component sigma_v)."""
    g = _rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    x = lo + (hi - lo) * g.random((n, 3))
    u = g.normal(0.0, sigma_v, size=(n, 3))
    return x, u


def uniform_cylinder_particles(n, radius, z_lo, z_hi, sigma_v, seed):
    g = _rng(seed)
    r = radius * np.sqrt(g.random(n))
    th = 2.0 * math.pi * g.random(n)
    z = z_lo + (z_hi - z_lo) * g.random(n)
    x = np.column_stack([r * np.cos(th), r * np.sin(th), z])
    u = g.normal(0.0, sigma_v, size=(n, 3))
    return x, u


def random_field_dofs(n, scale, seed):
    """Random values for edge or face degrees of freedom (test fixtures)."""
    return _rng(seed).normal(0.0, scale, size=n)

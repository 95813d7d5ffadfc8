"""Oracle: the seeded disk source of a beam (Sec. IV-B injects electrons through a disk on
the z = 0 wall every step), drawn from a counter-based generator so that any particle of
any step can be reproduced on its own.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011): ten rounds of
    (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57, the key (k0, k1) advanced by (0x9E3779B9,
0xBB67AE85) before every round but the first.

Particle j of injection k of species s, with key (seed mod 2^32, seed div 2^32), takes the
three blocks of counter (j, k mod 2^32, k div 2^32, 4 s + b), b = 0, 1, 2: twelve words
w_0..w_11, six uniforms u_i = ((w_2i >> 5) 2^26 + (w_2i+1 >> 6) + 1/2) 2^-53 in (0, 1):
* position on the disk: radius R sqrt(u_0), angle 2 pi u_1, in the plane spanned by
  e1 = unit(n x a) and e2 = n x e1 (n the unit normal; a = x-axis unless |n_x| >= 0.9,
  then the y-axis), around the centre;
* three standard normals by Box-Muller: sqrt(-2 ln u_2) (cos 2 pi u_3, sin 2 pi u_3) and
  sqrt(-2 ln u_4) cos 2 pi u_5;
* velocity v = v0 n + sigma (N_0, N_1, N_2), with the drift speed v0 from the kinetic
  energy (gamma_0 = 1 + K e / (m c^2)) and the per-component thermal spread sigma =
  sqrt(T e / m) (T in eV); the particle carries u = gamma v (Boris) or v (Adams-Bashforth).
"""
from __future__ import annotations

import numpy as np

from .constants import C_LIGHT, Q_E

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint64 array [..., 4] of 32-bit words; key: [..., 2].  Returns [..., 4]."""
    c = np.asarray(ctr, dtype=np.uint64) & MASK
    k = np.asarray(key, dtype=np.uint64) & MASK
    c = [c[..., i].copy() for i in range(4)]
    k0 = np.broadcast_to(k[..., 0], c[0].shape).copy()
    k1 = np.broadcast_to(k[..., 1], c[0].shape).copy()
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & MASK
            k1 = (k1 + np.uint64(W1)) & MASK
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniforms(n, k, species, seed):
    """The six uniforms of particles 0..n-1 of injection k of a species: [n, 6]."""
    j = np.arange(n, dtype=np.uint64)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    words = []
    for b in range(3):
        ctr = np.stack([j, np.full(n, k & 0xFFFFFFFF, np.uint64), np.full(n, (k >> 32) & 0xFFFFFFFF, np.uint64),
                        np.full(n, 4 * species + b, np.uint64)], axis=1)
        words.append(philox4x32_10(ctr, key))
    w = np.concatenate(words, axis=1)                      # [n, 12]
    hi = (w[:, 0::2] >> np.uint64(5)).astype(np.float64)
    lo = (w[:, 1::2] >> np.uint64(6)).astype(np.float64)
    return (hi * 67108864.0 + lo + 0.5) * 2.0 ** -53


def plane_basis(normal):
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1)
    return n, e1, np.cross(n, e1)


def disk_batch(spec, k, species, mass, relativistic_u=True):
    """Positions x [n, 3] and u [n, 3] of injection k.  spec: dict with center, normal,
    radius, kinetic_eV, thermal_eV, per_step, seed."""
    n = int(spec["per_step"])
    U = uniforms(n, int(k), int(species), int(spec["seed"]))
    nrm, e1, e2 = plane_basis(spec["normal"])
    r = spec["radius"] * np.sqrt(U[:, 0])
    phi = 2.0 * np.pi * U[:, 1]
    x = np.asarray(spec["center"], dtype=np.float64) + r[:, None] * (np.cos(phi)[:, None] * e1 +
                                                                     np.sin(phi)[:, None] * e2)
    a = np.sqrt(-2.0 * np.log(U[:, 2]))
    b = np.sqrt(-2.0 * np.log(U[:, 4]))
    N = np.stack([a * np.cos(2.0 * np.pi * U[:, 3]), a * np.sin(2.0 * np.pi * U[:, 3]),
                  b * np.cos(2.0 * np.pi * U[:, 5])], axis=1)
    g0 = 1.0 + spec["kinetic_eV"] * Q_E / (mass * C_LIGHT ** 2)
    v0 = C_LIGHT * np.sqrt(1.0 - 1.0 / (g0 * g0))
    sigma = np.sqrt(spec["thermal_eV"] * Q_E / mass)
    v = v0 * nrm + sigma * N
    if relativistic_u:
        v = v / np.sqrt(1.0 - np.sum(v * v, axis=1) / C_LIGHT ** 2)[:, None]
    return x, v

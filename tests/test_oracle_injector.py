"""Pins for the oracle's seeded disk source (oracle/injector.py).

* Philox4x32-10 against the known-answer vectors published with the generator
  (Random123: counter/key all zeros, all ones, and the digits of pi).
* The draws: uniforms in (0, 1) with mean 1/2 and variance 1/12; positions on the disk
  (in the plane, inside the radius, E[r^2] = R^2 / 2, uniform angle); velocities with the
  drift v0 n from the kinetic energy and per-component standard deviation sqrt(kT/m).
* Counter-based: a batch is reproducible, and batches of different steps or species differ.
"""
import math

import numpy as np
import pytest

from oracle import injector as inj
from oracle.constants import C_LIGHT, M_E, Q_E


@pytest.mark.parametrize("ctr,key,want", [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
])
def test_philox_known_answers(ctr, key, want):
    got = inj.philox4x32_10(np.array([ctr], dtype=np.uint64), np.array([key], dtype=np.uint64))[0]
    assert [int(v) for v in got] == want


def test_uniforms():
    U = inj.uniforms(200_000, 3, 1, 12345)
    assert U.min() > 0.0 and U.max() < 1.0
    assert np.allclose(U.mean(axis=0), 0.5, atol=4e-3)
    assert np.allclose(U.var(axis=0), 1 / 12, atol=2e-3)
    # the six columns are uncorrelated
    c = np.corrcoef(U.T)
    assert np.abs(c - np.eye(6)).max() < 1e-2


SPEC = dict(center=[0.0, 0.0, 0.0], normal=[0.0, 0.0, 1.0], radius=0.01, kinetic_eV=1000.0, thermal_eV=1.0,
            per_step=100_000, seed=99)


def test_disk_positions_and_velocities():
    x, u = inj.disk_batch(SPEC, 0, 0, M_E, relativistic_u=False)
    assert np.all(x[:, 2] == 0.0)
    r = np.hypot(x[:, 0], x[:, 1])
    assert r.max() <= 0.01
    assert np.mean(r ** 2) == pytest.approx(0.01 ** 2 / 2, rel=1e-2)
    ang = np.arctan2(x[:, 1], x[:, 0])
    hist, _ = np.histogram(ang, bins=8, range=(-math.pi, math.pi))
    assert np.abs(hist / len(x) - 1 / 8).max() < 5e-3
    g0 = 1 + 1000.0 * Q_E / (M_E * C_LIGHT ** 2)
    v0 = C_LIGHT * math.sqrt(1 - 1 / g0 ** 2)
    sig = math.sqrt(Q_E / M_E)
    n = len(u)
    assert u[:, 2].mean() == pytest.approx(v0, abs=4 * sig / math.sqrt(n))
    assert np.abs(u[:, :2].mean(axis=0)).max() < 4 * sig / math.sqrt(n)
    assert np.allclose(u.std(axis=0), sig, rtol=1e-2)
    # gamma v for the Boris pusher
    _, ug = inj.disk_batch(SPEC, 0, 0, M_E)
    g = 1 / np.sqrt(1 - np.sum(u ** 2, axis=1) / C_LIGHT ** 2)
    assert np.allclose(ug, g[:, None] * u, rtol=1e-15)


def test_tilted_plane_basis():
    spec = dict(SPEC, normal=[1.0, 2.0, -2.0], center=[0.1, 0.2, 0.3], per_step=1000)
    x, u = inj.disk_batch(spec, 5, 2, M_E, relativistic_u=False)
    n = np.array([1.0, 2.0, -2.0]) / 3.0
    assert np.abs((x - spec["center"]) @ n).max() < 1e-15
    assert np.linalg.norm(x - spec["center"], axis=1).max() <= 0.01 * (1 + 1e-15)


def test_counter_based_batches():
    a = inj.disk_batch(dict(SPEC, per_step=100), 7, 0, M_E)
    b = inj.disk_batch(dict(SPEC, per_step=100), 7, 0, M_E)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # a longer batch of the same step starts with the same particles
    c = inj.disk_batch(dict(SPEC, per_step=150), 7, 0, M_E)
    assert np.array_equal(c[0][:100], a[0])
    for other in (inj.disk_batch(dict(SPEC, per_step=100), 8, 0, M_E),
                  inj.disk_batch(dict(SPEC, per_step=100), 7, 1, M_E),
                  inj.disk_batch(dict(SPEC, per_step=100, seed=100), 7, 0, M_E)):
        assert not np.any(np.all(other[0] == a[0], axis=1))

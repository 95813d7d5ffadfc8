"""Pins for the oracle's push, path tracking and current deposit (Sec. III-B, III-C).

* Boris: exact invariants and closed forms of the discrete rotation.
* Tracking: cell-exit points against the paper's bisection search on the path parameter
  (Alg. 2, loop read as "while |t_s - t_f| > tol") and against dense point location.
* Deposit: per-piece Whitney-1 path integral against 5-point Gauss-Legendre quadrature of
  W1 . dr, and D^T (deposit) = q w (lambda_end - lambda_start) (charge continuity for a
  single path, eq. (gaussredo)).
"""
import math

import numpy as np
import pytest

from oracle import fem
from oracle.constants import C_LIGHT, M_E, Q_E
from oracle.mesh import Mesh
from oracle.particles import CMesh, boris, deposit_path, trace
from paper_2102_06248_amd import inputs


# ---------------------------------------------------------------- Boris

def test_boris_pure_magnetic_rotation():
    B = np.array([0.0, 0.0, 0.1])
    u0 = np.array([2.0e7, -1.0e7, 3.0e6])
    dt = 1e-11
    g = math.sqrt(1 + u0 @ u0 / C_LIGHT ** 2)
    u = boris(-Q_E, M_E, dt, np.zeros(3), B, u0)
    # |u| conserved, parallel component unchanged, perpendicular rotated by 2 atan(w dt/2)
    assert np.isclose(np.linalg.norm(u), np.linalg.norm(u0), rtol=1e-15)
    assert u[2] == pytest.approx(u0[2], rel=1e-15)
    om = Q_E * 0.1 / (g * M_E)
    th = math.atan2(u[1], u[0]) - math.atan2(u0[1], u0[0])
    th = (th + math.pi) % (2 * math.pi) - math.pi
    # electron (q<0) in +z field gyrates counter-clockwise seen from +z
    assert th == pytest.approx(2 * math.atan(om * dt / 2), rel=1e-12)


def test_boris_pure_electric_kick():
    E = np.array([1e3, -2e4, 5e2])
    u0 = np.array([1e5, 2e5, -3e5])
    dt = 2e-11
    u = boris(-Q_E, M_E, dt, E, np.zeros(3), u0)
    assert np.allclose(u, u0 - Q_E * E * dt / M_E, rtol=1e-14)


def test_boris_exb_drift_average():
    """Crossed fields: the time-averaged velocity is the E x B drift E x B / B^2."""
    E = np.array([0.0, 1e3, 0.0])
    B = np.array([0.0, 0.0, 0.05])
    om = Q_E * 0.05 / M_E
    T = 2 * math.pi / om
    nper = 200
    dt = T / nper
    u = np.zeros(3)
    vs = []
    for _ in range(nper * 20):
        u = boris(-Q_E, M_E, dt, E, B, u)
        vs.append(u / math.sqrt(1 + u @ u / C_LIGHT ** 2))
    vd = np.mean(vs, axis=0)
    drift = np.cross(E, B) / (B @ B)
    assert np.allclose(vd, drift, atol=2e-3 * np.linalg.norm(drift))


# ---------------------------------------------------------------- tracking

def _inside(mesh, t, x, tol=1e-12):
    return mesh.barycentric(t, x).min() >= -tol


def _bisect_exit(mesh, t, xs, d, tol=1e-15):
    """Alg. 2: halve [t_s, t_f] keeping t_s inside the start cell."""
    ts, tf = 0.0, 1.0
    th = 0.5
    while abs(ts - tf) > tol:
        if _inside(mesh, t, xs + th * d, 0.0):
            ts = th
        else:
            tf = th
        th = 0.5 * (ts + tf)
    return ts


@pytest.fixture(scope="module")
def jm():
    xyz, tets = inputs.kuhn_cube(3)
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(3), 1 / 3, 0.12, seed=3)
    m = Mesh(xyz, tets)
    return m, CMesh(m)


def test_exit_points_match_bisection_and_dense_location(jm):
    m, cm = jm
    rng = np.random.default_rng(11)
    n_checked = 0
    for _ in range(300):
        t0 = int(rng.integers(m.n_tets))
        xs = rng.dirichlet(np.ones(4)) @ m.xyz[m.tets[t0]]
        d = rng.normal(size=3) * 0.25
        st, t_end, x_end, rec = trace(cm, t0, xs, d)
        # walk the recorded pieces: every crossing point is the bisection exit of the
        # piece's cell, and the cells agree with dense point location along the path
        t, x = t0, xs.copy()
        pts = [p for _, p in rec]
        tets_after = [tt for tt, _ in rec]
        for k, p in enumerate(pts):
            rem = (xs + d) - x
            s = _bisect_exit(m, t, x, rem)
            assert np.allclose(x + s * rem, p, atol=1e-12)
            n_checked += 1
            if tets_after[k] < 0:
                break
            x, t = p, tets_after[k]
        if st == 0:
            assert np.allclose(x_end, xs + d, atol=1e-14)
            assert _inside(m, t_end, x_end, 1e-12)
            # dense sampling of the final piece lies in the final tet
            for a in np.linspace(0, 1, 9):
                y = x + a * (x_end - x)
                assert _inside(m, t_end, y, 1e-11)
    assert n_checked > 200


def test_vertex_and_edge_aimed_paths_terminate(jm):
    m, cm = jm
    rng = np.random.default_rng(5)
    for _ in range(100):
        t0 = int(rng.integers(m.n_tets))
        xs = rng.dirichlet(np.ones(4)) @ m.xyz[m.tets[t0]]
        # aim exactly through a vertex or an edge midpoint of the start tet, and beyond
        if rng.random() < 0.5:
            target = m.xyz[m.tets[t0, rng.integers(4)]]
        else:
            a, b = rng.choice(4, 2, replace=False)
            target = 0.5 * (m.xyz[m.tets[t0, a]] + m.xyz[m.tets[t0, b]])
        d = 1.7 * (target - xs)
        st, t_end, x_end, _ = trace(cm, t0, xs, d)
        assert st in (0, 1)
        if st == 0:
            assert _inside(m, t_end, x_end, 1e-10)


# ---------------------------------------------------------------- deposit

def test_deposit_matches_gauss_legendre_and_continuity(jm):
    m, cm = jm
    rng = np.random.default_rng(21)
    xg, wg = np.polynomial.legendre.leggauss(5)
    sg, wg = 0.5 * (xg + 1), 0.5 * wg
    D = m.D()
    qw = -3.7e-15
    for _ in range(200):
        t0 = int(rng.integers(m.n_tets))
        xs = rng.dirichlet(np.ones(4)) @ m.xyz[m.tets[t0]]
        d = rng.normal(size=3) * 0.2
        dg = np.zeros(m.n_edges)
        st, t_end, x_end = deposit_path(cm, t0, xs, d, qw, dg)
        _, _, _, rec = trace(cm, t0, xs, d)
        # reference: sum over pieces of qw * int W1 . dr by Gauss-Legendre
        ref = np.zeros(m.n_edges)
        pieces = []
        x, t = xs, t0
        for tt, p in rec:
            pieces.append((t, x, p))
            x, t = p, tt
            if tt < 0:
                break
        if not rec or rec[-1][0] >= 0:
            pieces.append((t, x, x_end))
        for (t, a, b) in pieces:
            pts = a + sg[:, None] * (b - a)
            lam = m.barycentric(np.full(len(sg), t), pts)
            W = fem.whitney1(lam, m.grad_lambda[t][None].repeat(len(sg), 0))
            ref[m.tet_edges[t]] += qw * np.einsum("q,qid,d->i", wg, W, b - a)
        assert np.allclose(dg, ref, rtol=1e-12, atol=1e-13 * abs(qw))
        # D^T dg = q w (lambda(end) - lambda(start)) at the nodes
        rho0 = np.zeros(m.n_nodes)
        rho0[m.tets[t0]] = qw * m.barycentric(t0, xs)
        rho1 = np.zeros(m.n_nodes)
        rho1[m.tets[t_end]] = qw * m.barycentric(t_end, x_end)
        if st == 0:
            assert np.allclose(D.T @ dg, rho1 - rho0, atol=1e-14 * abs(qw))

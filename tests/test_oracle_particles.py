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
from oracle.particles import CMesh, boris, deposit_path, gather, push, trace
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


# ---------------------------------------------------------------- gather (C oracle)

def _jittered(n, seed, frac=0.15):
    xyz, tets = inputs.kuhn_cube(n)
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(n), 1 / n, frac, seed=seed)
    return Mesh(xyz, tets)


def _random_points(m, rng, n):
    t = rng.integers(m.n_tets, size=n)
    lam = rng.dirichlet(np.ones(4), size=n)
    x = np.einsum("pk,pkd->pd", lam, m.xyz[m.tets[t]])
    return t, lam, x


@pytest.mark.parametrize("n,seed", [(2, 4), (3, 9)])
def test_c_gather_reproduces_uniform_fields(n, seed):
    """The Whitney-1 interpolant e_ab = E0 . (r_b - r_a) and the Whitney-2 interpolant
    b_f = B0 . (area vector of f) are exact for constant fields (Sec. II-A), so the C
    gather must return E0 and B0 at every point of every tet, on a distorted mesh."""
    m = _jittered(n, seed)
    cm = CMesh(m)
    rng = np.random.default_rng(seed)
    t, _, x = _random_points(m, rng, 500)
    for _ in range(3):
        E0, B0 = rng.normal(size=3) * 1e3, rng.normal(size=3) * 0.1
        E, B = gather(cm, t, x, m.edge_dofs_of_uniform_field(E0), m.face_dofs_of_uniform_field(B0))
        assert np.max(np.abs(E - E0)) <= 1e-13 * np.linalg.norm(E0)
        assert np.max(np.abs(B - B0)) <= 1e-13 * np.linalg.norm(B0)


def test_c_gather_equals_the_whitney_expansion():
    """For arbitrary edge and face unknowns the C gather is the expansion of Sec. II-A,
    E = sum e_i W1_i, B = sum b_f W2_f, evaluated by the Python Whitney bases."""
    m = _jittered(3, 12)
    cm = CMesh(m)
    rng = np.random.default_rng(2)
    t, lam, x = _random_points(m, rng, 800)
    e, b = rng.normal(size=m.n_edges), rng.normal(size=m.n_faces)
    E, B = gather(cm, t, x, e, b)
    lam_x = m.barycentric(t, x)
    assert np.allclose(lam_x, lam, atol=1e-14)
    E_ref, B_ref = fem.eval_E(m, e, t, lam_x), fem.eval_B(m, b, t, lam_x)
    scale_e = np.abs(E_ref).max()
    scale_b = np.abs(B_ref).max()
    assert np.max(np.abs(E - E_ref)) <= 1e-14 * scale_e * 10
    assert np.max(np.abs(B - B_ref)) <= 1e-14 * scale_b * 10


def _planted_lib(tmp_path, old, new):
    """The oracle's C source with one planted mistake, built into tmp_path."""
    import ctypes
    import subprocess

    from oracle import particles as op
    src = open(op._SRC).read()
    assert src.count(old) == 1
    p = tmp_path / "planted.c"
    p.write_text(src.replace(old, new))
    so = tmp_path / "libplanted.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", str(so), str(p), "-lm"])
    lib = ctypes.CDLL(str(so))
    lib.orc_gather.restype = None
    return lib


@pytest.mark.parametrize("old,new", [
    # the sign between the two terms of W1_ab = lambda_a grad lambda_b - lambda_b grad lambda_a
    ("lam[a] * g[3 * c + d] - lam[c] * g[3 * a + d]", "lam[a] * g[3 * c + d] + lam[c] * g[3 * a + d]"),
    # the pairing of lambda with the gradient of the other end of the edge
    ("lam[a] * g[3 * c + d] - lam[c] * g[3 * a + d]", "lam[c] * g[3 * c + d] - lam[a] * g[3 * a + d]"),
    # a dropped cyclic term of W2
    ("lam[i] * cjl[d] + lam[j] * cli[d] + lam[l] * cij[d]", "lam[i] * cjl[d] + lam[j] * cli[d]"),
])
def test_planted_gather_mistakes_fail_the_uniform_field_pin(tmp_path, old, new):
    """The uniform-field pin above catches the plausible slips in the C gather."""
    import ctypes

    from oracle.particles import _p
    lib = _planted_lib(tmp_path, old, new)
    m = _jittered(2, 4)
    cm = CMesh(m)
    rng = np.random.default_rng(4)
    t, _, x = _random_points(m, rng, 200)
    E0, B0 = np.array([1e3, -2e3, 5e2]), np.array([0.02, 0.05, -0.1])
    e, b = m.edge_dofs_of_uniform_field(E0), m.face_dofs_of_uniform_field(B0)
    t64 = np.ascontiguousarray(t, dtype=np.int64)
    x = np.ascontiguousarray(x)
    E, B = np.zeros_like(x), np.zeros_like(x)
    lib.orc_gather(cm.ref, ctypes.c_int64(len(t64)), _p(t64), _p(x), _p(e), _p(b), _p(E), _p(B))
    err = max(np.max(np.abs(E - E0)) / np.linalg.norm(E0), np.max(np.abs(B - B0)) / np.linalg.norm(B0))
    assert err > 1e-3


def test_c_push_in_a_uniform_electric_field_is_the_exact_impulse():
    """Gather + Boris + walk of the C oracle in a uniform E (B = 0): every particle's
    momentum changes by q E dt / m exactly, and the walk ends at x + dt v^{n+1/2}."""
    m = _jittered(3, 7, 0.1)
    cm = CMesh(m)
    rng = np.random.default_rng(8)
    n = 400
    t, _, x = _random_points(m, rng, n)
    u = rng.normal(size=(n, 3)) * 3e7
    E0 = np.array([3e3, -1e3, 2e3])
    e = m.edge_dofs_of_uniform_field(E0)
    b = np.zeros(m.n_faces)
    dt = 2e-9
    x1, u1 = x.copy(), u.copy()
    tet, alive = t.astype(np.int64), np.ones(n, dtype=np.int8)
    dg = np.zeros(m.n_edges)
    rc, st = push(cm, x1, u1, tet, alive, -Q_E, M_E, 1.0, dt, e, b, dg)
    assert rc == 0 and st.n_crossings > 0
    assert np.allclose(u1, u - Q_E * E0 * dt / M_E, rtol=1e-13, atol=1e-7)
    g = np.sqrt(1 + np.sum(u1 ** 2, axis=1) / C_LIGHT ** 2)
    a = alive.astype(bool)
    assert np.count_nonzero(~a) > 0 and np.count_nonzero(a) > n // 2
    assert np.allclose(x1[a], (x + dt * u1 / g[:, None])[a], atol=1e-14)
    assert np.all(m.barycentric(tet[a], x1[a]).min(axis=1) >= -1e-12)


# ---------------------------------------------------------------- point location

def test_locate_matches_brute_force():
    """Mesh.locate (nearest-centroid candidates) against the definition: a point lies in
    tet t when all four barycentric coordinates are >= 0, checked over every tet."""
    m = _jittered(3, 21, 0.2)
    rng = np.random.default_rng(6)
    inside = _random_points(m, rng, 300)[2]
    # points near faces and vertices, and outside the unit cube
    verts = m.xyz[rng.integers(m.n_nodes, size=60)] + rng.normal(size=(60, 3)) * 1e-9
    outside = rng.uniform(-0.3, 1.3, size=(200, 3))
    pts = np.concatenate([inside, verts, outside])
    loc = m.locate(pts)
    lam_all = np.stack([m.barycentric(np.full(len(pts), t), pts) for t in range(m.n_tets)], axis=1)
    minl = lam_all.min(axis=2)                      # [n_pts, n_tets]
    for i in range(len(pts)):
        ok = np.nonzero(minl[i] >= -1e-12)[0]
        if len(ok) == 0:
            assert loc[i] == -1, i
        else:
            assert loc[i] in ok, (i, loc[i], ok)
    assert np.count_nonzero(loc >= 0) >= 300

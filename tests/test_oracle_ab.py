"""Pins for the oracle's Adams-Bashforth pusher, Lagrange path, curved walk and curved-path
deposit (oracle/ab.py).

Checked against what does not come from the module's own formulas: the coefficients the
paper prints for k = 4 and the textbook ones for k = 1..3, exactness on polynomials,
Table I's cyclotron with its closed-form orbit (convergence slope = order, as Sec. IV-A
states), the straight-line closed form of the Whitney-1 path integral, adaptive quadrature
of the same integrand, and discrete charge continuity D^T g = q w (lambda_end -
lambda_start) along paths that cross many cells.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

from oracle import ab
from oracle.mesh import LOCAL_EDGES, Mesh
from paper_2102_06248_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_coefficients_match_the_paper_and_textbook():
    g = json.load(open(os.path.join(GOLDEN, "ab4_coefficients.json")))
    assert ab.ab_coefficients(4) == [Fraction(c, g["denominator"]) for c in g["numerators"]]
    assert ab.ab_coefficients(1) == [Fraction(1)]                              # forward Euler
    assert ab.ab_coefficients(2) == [Fraction(3, 2), Fraction(-1, 2)]
    assert ab.ab_coefficients(3) == [Fraction(23, 12), Fraction(-16, 12), Fraction(5, 12)]
    for k in range(1, 6):
        beta = ab.ab_coefficients(k)
        assert sum(beta) == 1
        # exact on polynomials of degree < k: sum_j beta_j p(-j) = int_0^1 p
        for d in range(k):
            assert sum(b * Fraction(-j) ** d for j, b in enumerate(beta)) == Fraction(1, d + 1)


def _cyclotron_error(order, n_per_period, periods=1):
    g = json.load(open(os.path.join(GOLDEN, "cyclotron_table1.json")))
    q, m, B = g["Q_C"], g["m_kg"], np.array([0.0, 0.0, g["B_z_T"]])
    r0, v0 = np.array(g["r0_m"]), np.array([0.0, g["v0_y_m_per_s"], 0.0])
    w = q * B[2] / m                                  # signed gyrofrequency (rad/s)
    # closed form: v(t) = v0 rotated by -w t about z, r(t) = r0 + integral of v
    def exact(t):
        cs, sn = np.cos(w * t), np.sin(w * t)
        v = np.array([v0[1] * sn, v0[1] * cs, 0.0])
        r = r0 + np.array([v0[1] * (1 - cs) / w, v0[1] * sn / w, 0.0])
        return r, v
    acc = lambda v: (q / m) * np.cross(v, B)
    dt = 2 * np.pi / abs(w) / n_per_period
    n_steps = n_per_period * periods
    hist_r, hist_v = [], []
    for j in range(order):                            # exact start-up history
        r, v = exact(-j * dt)
        hist_r.append(r)
        hist_v.append(v)
    hist_a = [acc(v) for v in hist_v]
    err, ref = 0.0, 0.0
    for n in range(n_steps):
        r_new, v_new = ab.ab_step(hist_r, hist_v, hist_a, dt, order)
        hist_r = [r_new] + hist_r[:order - 1]
        hist_v = [v_new] + hist_v[:order - 1]
        hist_a = [acc(v_new)] + hist_a[:order - 1]
        ra, _ = exact((n + 1) * dt)
        err += np.sum((r_new - ra) ** 2)
        ref += np.sum(ra ** 2)
    return np.sqrt(err / ref)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_cyclotron_converges_at_the_order(order):
    """Table I's cyclotron, mean relative position error over one period: the slope in dt
    equals the order (Sec. IV-A)."""
    ns = [200, 400, 800]
    errs = [_cyclotron_error(order, n) for n in ns]
    slopes = [np.log(errs[i] / errs[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    print(f"AB{order}: errors {['%.2e' % e for e in errs]}, slopes {['%.2f' % s for s in slopes]}")
    assert all(order - 0.15 <= s <= order + 0.3 for s in slopes)


def test_lagrange_path_reproduces_polynomials():
    rng = np.random.default_rng(3)
    coef = rng.normal(size=(4, 3))                   # a cubic path
    p = lambda s: sum(coef[i] * s ** i for i in range(4))
    dp = lambda s: sum(i * coef[i] * s ** (i - 1) for i in range(1, 4))
    path = ab.step_path(p(1.0), [p(0.0), p(-1.0), p(-2.0)])
    for s in np.linspace(-0.3, 1.2, 7):
        assert np.allclose(path(s), p(s), rtol=0, atol=1e-12)
        assert np.allclose(path.deriv(s), dp(s), rtol=0, atol=1e-12)


@pytest.fixture(scope="module")
def mesh():
    xyz, tets = inputs.kuhn_cube(5)
    xyz = inputs.jitter_nodes(xyz, inputs.kuhn_interior_nodes(5), 0.2, 0.1, seed=4)
    return Mesh(xyz, tets)


def test_straight_path_matches_the_closed_form(mesh):
    """k = 1: the path is a straight segment, and each piece's Whitney-1 integral equals
    the closed form lambda_a(start) lambda_b(end) - lambda_a(end) lambda_b(start)."""
    a, b = np.array([0.31, 0.42, 0.27]), np.array([0.66, 0.51, 0.73])
    path = ab.step_path(b, [a])
    tet = int(mesh.locate(a[None])[0])
    pieces, last = ab.walk_curved(mesh, tet, path, n_gl=2)
    assert len(pieces) > 3 and last >= 0
    g = ab.deposit_curved(mesh, pieces, path, 1.0, n_gl=2)
    want = np.zeros(mesh.n_edges)
    for t, sa, sb, p_in, p_out in pieces:
        ls = mesh.barycentric(t, path(sa)) if p_in is None else p_in
        le = mesh.barycentric(t, path(sb)) if p_out is None else p_out
        ea, eb = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
        want[mesh.tet_edges[t]] += ls[ea] * le[eb] - le[ea] * ls[eb]
    assert np.allclose(g, want, rtol=0, atol=1e-13)


def _curved_path(seed):
    rng = np.random.default_rng(seed)
    pts = 0.5 + 0.3 * rng.uniform(-1, 1, size=(5, 3))   # r^{n+1}, r^n, ..., r^{n-3}
    return ab.step_path(pts[0], list(pts[1:]))


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_curved_walk_chains_cells_and_conserves_charge(mesh, seed):
    """A degree-4 path through many cells: consecutive pieces share a face, each crossing
    lies on that face, the quadrature equals adaptive quadrature, and D^T g = q w
    (lambda(end) - lambda(start)) on every node."""
    path = _curved_path(seed)
    tet = int(mesh.locate(path(0.0)[None])[0])
    assert tet >= 0
    pieces, last = ab.walk_curved(mesh, tet, path, n_gl=5)
    assert last >= 0 and len(pieces) >= 4
    for (t0, _, s, _, p_out), (t1, s1, _, p_in, _) in zip(pieces[:-1], pieces[1:]):
        assert s == s1 and t1 in mesh.nbr[t0]
        assert abs(mesh.barycentric(t0, path(s)).min()) < 1e-12
        # the closing face point: on the face, near r(s), the same point in both cells
        k = int(np.argmin(p_out))
        assert p_out[k] == 0.0 and abs(p_out.sum() - 1.0) < 1e-15
        assert np.abs(p_out - mesh.barycentric(t0, path(s))).max() < 1e-12
        x_out = p_out @ mesh.xyz[mesh.tets[t0]]
        assert np.abs(p_in @ mesh.xyz[mesh.tets[t1]] - x_out).max() < 1e-15
        assert sorted(p_in) == sorted(p_out)
    qw = -3.0
    g = ab.deposit_curved(mesh, pieces, path, qw, n_gl=5)
    # adaptive quadrature of the same integrand on each piece's curved part
    for piece in pieces[:3]:
        t, sa, sb = piece[:3]
        grad = mesh.grad_lambda[t]
        ea, eb = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
        def f(s, c):
            lam = mesh.barycentric(t, path(s))
            dl = grad @ path.deriv(s)
            return lam[ea[c]] * dl[eb[c]] - lam[eb[c]] * dl[ea[c]]
        one = ab.piece_integral(mesh, piece, path, n_gl=5)
        for c in range(6):
            ref = integrate.quad(f, sa, sb, args=(c,), epsabs=1e-15, epsrel=1e-13)[0]
            assert abs(one[c] - ref) <= 1e-12
    # charge continuity: D^T g against the change of the nodal charge
    DTg = mesh.D().T @ g
    rho0 = np.zeros(mesh.n_nodes)
    rho1 = np.zeros(mesh.n_nodes)
    np.add.at(rho0, mesh.tets[tet], qw * mesh.barycentric(tet, path(0.0)))
    np.add.at(rho1, mesh.tets[last], qw * mesh.barycentric(last, path(1.0)))
    assert np.abs(DTg - (rho1 - rho0)).max() <= 1e-14 * abs(qw)
    # a wrong quadrature order (too few points) breaks the exactness of the deposit
    g2 = ab.deposit_curved(mesh, pieces, path, qw, n_gl=2)
    assert np.abs(g2 - g).max() > 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("tol", [1e-15, 1e-7])
def test_face_closures_make_continuity_exact_for_any_crossing_tolerance(mesh, tol):
    """With the crossings located only to tol, the closed pieces still give D^T g = q w
    (lambda(end) - lambda(start)) to round-off; without the closures (the curved parts
    alone) the residual is of the size of the crossing error."""
    qw = 2.5
    D = mesh.D()
    for seed in (5, 6, 7, 8):
        path = _curved_path(seed)
        tet = int(mesh.locate(path(0.0)[None])[0])
        pieces, last = ab.walk_curved(mesh, tet, path, n_gl=5, tol=tol)
        if last < 0:
            continue
        rho = np.zeros(mesh.n_nodes)
        np.add.at(rho, mesh.tets[last], qw * mesh.barycentric(last, path(1.0)))
        np.add.at(rho, mesh.tets[tet], -qw * mesh.barycentric(tet, path(0.0)))
        g = ab.deposit_curved(mesh, pieces, path, qw, n_gl=5)
        assert np.abs(D.T @ g - rho).max() <= 1e-14 * abs(qw)
        bare = np.zeros(mesh.n_edges)
        for piece in pieces:
            bare[mesh.tet_edges[piece[0]]] += qw * ab.piece_integral(mesh, piece, path, n_gl=5)
        if tol > 1e-10 and len(pieces) > 1:
            assert np.abs(D.T @ bare - rho).max() > 1e-12 * abs(qw)

"""Pins for the oracle's mesh, Whitney forms and FEM matrices (Sec. II-A).

Each check compares against something other than the oracle's own formula: closed-form
entity counts, exact-sequence identities of the de Rham complex, analytic integrals of
uniform fields, an independent quadrature, and the P1 stiffness matrix.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem
from oracle.constants import EPS0, MU0
from oracle.mesh import LOCAL_EDGES, LOCAL_FACES, Mesh
from paper_2102_06248_amd import inputs


def kuhn_counts(n):
    nodes = (n + 1) ** 3
    edges = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    faces = 6 * n * n * (n + 1) + 6 * n ** 3
    return nodes, edges, faces, 6 * n ** 3


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_kuhn_counts_and_exactness(n):
    m = Mesh(*inputs.kuhn_cube(n))
    assert (m.n_nodes, m.n_edges, m.n_faces, m.n_tets) == kuhn_counts(n)
    assert m.euler_characteristic() == 1
    assert np.count_nonzero(m.boundary_face) == 12 * n * n
    assert np.count_nonzero(m.boundary_node) == (n + 1) ** 3 - (n - 1) ** 3
    D, C, D2 = m.D(), m.C(), m.D2()
    assert abs(C @ D).max() == 0.0          # curl grad = 0
    assert abs(D2 @ C).max() == 0.0         # div curl = 0


def test_prism_cylinder_counts():
    nr, nz = 3, 4
    m = Mesh(*inputs.prism_cylinder(0.05, 0.2, nr, nz))
    n2 = 1 + 3 * nr * (nr + 1)
    assert m.n_nodes == n2 * (nz + 1)
    assert m.n_tets == 18 * nr * nr * nz
    assert m.euler_characteristic() == 1
    assert abs(m.D2() @ m.C()).max() == 0.0
    # total volume of the polygonal cylinder: 6 n_r^2 triangles of the hex-ring disk
    assert np.isclose(m.vol.sum(), np.sum(_hexdisk_area(0.05, nr)) * 0.2, rtol=1e-12)


def _hexdisk_area(radius, nr):
    xy, tris = inputs.hex_disk(radius, nr)
    a, b, c = xy[tris[:, 0]], xy[tris[:, 1]], xy[tris[:, 2]]
    return 0.5 * np.abs((b - a)[:, 0] * (c - a)[:, 1] - (b - a)[:, 1] * (c - a)[:, 0])


def test_neighbours_symmetric(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    for t in range(m.n_tets):
        for k in range(4):
            nb = m.nbr[t, k]
            if nb < 0:
                assert m.boundary_face[m.tet_faces[t, k]]
                continue
            assert t in m.nbr[nb]
            assert len(set(m.tets[t]) & set(m.tets[nb])) == 3


def test_barycentric_definition(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    rng = np.random.default_rng(1)
    for t in range(0, m.n_tets, 7):
        # vertices map to unit vectors; a random point is reconstructed by sum lambda_k r_k
        lam_v = m.barycentric(np.full(4, t), m.xyz[m.tets[t]])
        assert np.allclose(lam_v, np.eye(4), atol=1e-14)
        w = rng.dirichlet(np.ones(4))
        x = w @ m.xyz[m.tets[t]]
        assert np.allclose(m.barycentric(t, x), w, atol=1e-14)


# ---------------------------------------------------------------- Whitney forms

def _gauss_legendre(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def test_whitney1_edge_circulations(kuhn2_jittered):
    """int_{edge j} W1_i . dl = delta_ij (the defining property of edge elements)."""
    m = Mesh(*kuhn2_jittered)
    s, w = _gauss_legendre(4)
    for t in (0, 5, 17, 33):
        g = m.grad_lambda[t]
        for j, (a, b) in enumerate(LOCAL_EDGES):
            lam = np.zeros((len(s), 4))
            lam[:, a] = 1.0 - s
            lam[:, b] = s
            dl = m.xyz[m.tets[t, b]] - m.xyz[m.tets[t, a]]
            circ = np.einsum("q,qid,d->i", w, fem.whitney1(lam, g[None].repeat(len(s), 0)), dl)
            assert np.allclose(circ, np.eye(6)[j], atol=1e-13)


def _triangle_rule():
    # 3-point rule exact for quadratics on a triangle (edge midpoints, weights 1/3)
    return np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]]), np.full(3, 1.0 / 3.0)


def test_whitney2_face_fluxes(kuhn2_jittered):
    """int_{face j} W2_i . dA = delta_ij with dA along the face's canonical normal
    (r_j - r_i) x (r_k - r_i), i < j < k."""
    m = Mesh(*kuhn2_jittered)
    pts, wts = _triangle_rule()
    for t in (0, 9, 26, 40):
        g = m.grad_lambda[t]
        for j, (a, b, c) in enumerate(LOCAL_FACES):
            lam = np.zeros((3, 4))
            lam[:, [a, b, c]] = pts
            r = m.xyz[m.tets[t]]
            area_vec = 0.5 * np.cross(r[b] - r[a], r[c] - r[a])
            W = fem.whitney2(lam, g[None].repeat(3, 0))
            flux = np.einsum("q,qid,d->i", wts, W, area_vec)
            assert np.allclose(flux, np.eye(4)[j], atol=1e-13)


def test_uniform_fields_reproduced(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    rng = np.random.default_rng(2)
    E0, B0 = rng.normal(size=3), rng.normal(size=3)
    e = m.edge_dofs_of_uniform_field(E0)
    b = m.face_dofs_of_uniform_field(B0)
    t = rng.integers(0, m.n_tets, 50)
    lam = rng.dirichlet(np.ones(4), 50)
    assert np.allclose(fem.eval_E(m, e, t, lam), E0, rtol=1e-13, atol=1e-13)
    assert np.allclose(fem.eval_B(m, b, t, lam), B0, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- matrices

def _duffy_rule(n):
    """Collapsed (Duffy) tensor Gauss-Legendre rule on the unit tetrahedron; exact for
    polynomials of degree <= 2n - 3.  Returns barycentric points [q,4], weights (sum 1)."""
    s, w = _gauss_legendre(n)
    P, W = [], []
    for (a, wa), (b, wb), (c, wc) in itertools.product(zip(s, w), zip(s, w), zip(s, w)):
        x = a
        y = b * (1 - a)
        z = c * (1 - a) * (1 - b)
        P.append([1 - x - y - z, x, y, z])
        W.append(wa * wb * wc * (1 - a) ** 2 * (1 - b) * 6.0)
    return np.array(P), np.array(W)


def test_mass_matrix_vs_independent_quadrature(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    P, W = _duffy_rule(4)
    Me = fem.element_mass(m)
    for t in (0, 11, 29):
        g = m.grad_lambda[t]
        Wq = fem.whitney1(P, g[None].repeat(len(P), 0))
        ref = EPS0 * m.vol[t] * np.einsum("q,qid,qjd->ij", W, Wq, Wq)
        assert np.allclose(Me[t], ref, rtol=1e-13, atol=1e-13 * abs(ref).max())


def test_mass_uniform_field_energy(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    M = fem.mass_matrix(m)
    E0 = np.array([0.3, -1.1, 2.0])
    e = m.edge_dofs_of_uniform_field(E0)
    assert np.isclose(e @ (M @ e), EPS0 * (E0 @ E0) * m.vol.sum(), rtol=1e-13)


def test_magnetic_energy_of_uniform_field(kuhn2_jittered):
    """Face fluxes of a uniform B0 carry the energy |B0|^2 Vol / (2 mu0)."""
    from oracle import diagnostics
    m = Mesh(*kuhn2_jittered)
    B0 = np.array([-0.7, 0.25, 1.3])
    b = m.face_dofs_of_uniform_field(B0)
    W = diagnostics.magnetic_energy(fem.face_mass_matrix(m), b)
    assert np.isclose(W, (B0 @ B0) * m.vol.sum() / (2 * MU0), rtol=1e-13)


def test_kinetic_energy_closed_forms():
    from oracle import diagnostics
    from oracle.constants import C_LIGHT, M_E
    # gamma v for v = 0.6 c: gamma = 1.25, kinetic energy 0.25 m c^2 per unit weight
    u = np.array([[0.0, 0.75 * C_LIGHT, 0.0]])
    assert np.isclose(diagnostics.kinetic_energy(u, 3.0, M_E, C_LIGHT), 3.0 * 0.25 * M_E * C_LIGHT ** 2, rtol=1e-14)
    # slow particles: 1/2 m v^2 to O(v^2/c^2)
    v = np.array([[1e3, -2e3, 5e2], [0.0, 0.0, 0.0]])
    ke = diagnostics.kinetic_energy(v, 2.0, M_E, C_LIGHT)
    assert np.isclose(ke, 2.0 * 0.5 * M_E * np.sum(v ** 2), rtol=1e-10)


def test_mass_on_gradients_is_p1_stiffness(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    M, D = fem.mass_matrix(m), m.D()
    L = fem.nodal_stiffness(m)
    assert abs(D.T @ M @ D - L).max() <= 1e-13 * abs(L).max()


def test_curlcurl_identities(kuhn2_jittered):
    m = Mesh(*kuhn2_jittered)
    S = fem.curlcurl_matrix(m)
    D, C = m.D(), m.C()
    assert abs(S @ D).max() <= 1e-12 * abs(S).max()
    Mf = fem.face_mass_matrix(m)
    assert abs(S - C.T @ Mf @ C).max() <= 1e-13 * abs(S).max()
    # E = 1/2 B0 x r has curl B0; its edge interpolant (midpoint rule is exact for a
    # linear field) has piecewise-constant curl B0, so e^T S e = |B0|^2 Vol / mu0.
    B0 = np.array([0.4, 0.2, -0.9])
    mid = 0.5 * (m.xyz[m.edges[:, 0]] + m.xyz[m.edges[:, 1]])
    dl = m.xyz[m.edges[:, 1]] - m.xyz[m.edges[:, 0]]
    e = np.einsum("id,id->i", 0.5 * np.cross(B0, mid), dl)
    assert np.isclose(e @ (S @ e), (B0 @ B0) * m.vol.sum() / MU0, rtol=1e-12)


def test_curlcurl_nullspace_dimension():
    """On interior edges (PEC), null(S) = gradients of interior-node hat functions."""
    m = Mesh(*inputs.kuhn_cube(2))
    ie = m.interior_edges
    S = fem.curlcurl_matrix(m)[ie][:, ie].toarray()
    M = fem.mass_matrix(m)[ie][:, ie].toarray()
    ev = sla.eigh(S, M, eigvals_only=True)
    n_zero = int(np.sum(np.abs(ev) < 1e-8 * ev.max()))
    assert n_zero == len(m.interior_nodes)

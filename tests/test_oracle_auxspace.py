"""Pins for the oracle's nodal auxiliary-space preconditioner and its PCG.

Each check compares against something other than the preconditioner's own formula: the
de Rham identity S G = 0 of the Whitney complex, line integrals of linear fields by an
independent two-point Gauss-Legendre quadrature, symmetry and positivity, and the direct
sparse solve of the Newmark system.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import auxspace, fem, newmark
from oracle.constants import C_LIGHT
from oracle.mesh import Mesh
from oracle.pic import OracleSim
from paper_2102_06248_amd import inputs


def _jittered_kuhn(n, seed, amp=0.15):
    xyz, tets = inputs.kuhn_cube(n)
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    inner = np.all((xyz > 1e-12) & (xyz < 1 - 1e-12), axis=1)
    xyz = xyz.copy()
    xyz[inner] += amp * h * rng.uniform(-1, 1, size=(inner.sum(), 3))
    return xyz, tets


@pytest.fixture(scope="module")
def mesh():
    return Mesh(*_jittered_kuhn(5, 1))


def test_gradients_are_in_the_kernel_of_curl_curl(mesh):
    S = fem.curlcurl_matrix(mesh)
    G = auxspace.gradient_matrix(mesh, np.arange(mesh.n_edges), np.arange(mesh.n_nodes))
    assert abs(S @ G).max() <= 1e-12 * abs(S).max()
    # a planted orientation error (one edge entered with the wrong sign at one node)
    # breaks the identity
    Gb = G.tolil()
    e = G[:, 7].nonzero()[0][0]
    Gb[e, 7] = -Gb[e, 7]
    assert abs(S @ Gb.tocsr()).max() > 1e-3 * abs(S).max()


def test_vector_interpolation_is_exact_on_linear_fields(mesh):
    rng = np.random.default_rng(2)
    c, L = rng.normal(size=3), rng.normal(size=(3, 3))
    field = lambda x: c + x @ L.T
    Pi = auxspace.vector_interpolation_matrix(mesh, np.arange(mesh.n_edges), np.arange(mesh.n_nodes))
    got = Pi @ field(mesh.xyz).ravel()
    # two-point Gauss-Legendre along each edge (exact for the linear integrand)
    a, b = mesh.xyz[mesh.edges[:, 0]], mesh.xyz[mesh.edges[:, 1]]
    t = b - a
    g = 0.5 / np.sqrt(3.0)
    want = 0.5 * np.sum(t * (field(a + (0.5 - g) * t) + field(a + (0.5 + g) * t)), axis=1)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    # uniform fields: the line integral the mesh module gives
    u = rng.normal(size=3)
    assert np.allclose(Pi @ np.tile(u, mesh.n_nodes), mesh.edge_dofs_of_uniform_field(u), rtol=1e-13, atol=1e-15)


def test_restricted_interpolation_drops_wall_nodes(mesh):
    ie, inode = mesh.interior_edges, mesh.interior_nodes
    full = auxspace.vector_interpolation_matrix(mesh, ie, np.arange(mesh.n_nodes))
    cols = np.stack([3 * inode, 3 * inode + 1, 3 * inode + 2], 1).ravel()
    part = auxspace.vector_interpolation_matrix(mesh, ie, inode)
    assert abs(part - full[:, cols]).max() == 0.0


def _newmark_A(m, cfl_ratio):
    sim = OracleSim(m.xyz, m.tets)
    h = np.linalg.norm(m.xyz[m.edges[:, 1]] - m.xyz[m.edges[:, 0]], axis=1).min()
    dt = cfl_ratio * h / C_LIGHT
    A, _, _ = sim.operators(dt, 0.25, 0.5)
    return A


def test_preconditioner_is_symmetric_positive_definite(mesh):
    A = _newmark_A(mesh, 10.0)
    apply, G, Pi, dG, dPi = auxspace.aux_space_preconditioner(A, mesh)
    assert np.all(dG > 0) and np.all(dPi > 0)
    rng = np.random.default_rng(3)
    x, y = rng.normal(size=(2, A.shape[0]))
    bx, by = apply(x), apply(y)
    assert abs(x @ by - y @ bx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(by)
    assert x @ bx > 0 and y @ by > 0
    # G^T A G has no curl-curl part: its diagonal is that of G^T M G
    M = newmark.restrict(fem.mass_matrix(mesh), mesh.interior_edges)
    assert np.allclose(dG, (G.T @ (M @ G)).diagonal(), rtol=1e-9)


@pytest.mark.parametrize("cfl_ratio", [5.0, 20.0])
def test_pcg_matches_the_direct_solve_in_fewer_iterations(mesh, cfl_ratio):
    A = _newmark_A(mesh, cfl_ratio)
    rng = np.random.default_rng(4)
    b = rng.normal(size=A.shape[0])
    x_direct = spla.spsolve(A.tocsc(), b)
    apply = auxspace.aux_space_preconditioner(A, mesh)[0]
    x, it, res = auxspace.pcg(A, b, np.zeros_like(b), apply, tol=1e-10)
    assert res <= 1e-10
    assert np.linalg.norm(x - x_direct) <= 1e-8 * np.linalg.norm(x_direct)
    _, it_j, _ = newmark.pcg_jacobi(A, b, np.zeros_like(b), 1e-10)
    assert it < it_j
    # the same PCG with the Jacobi part alone is the Jacobi PCG of the Newmark module (up
    # to the rounding of r / d against d^-1 r, which moves late iterations a little)
    dA = A.diagonal()
    _, it_same, _ = auxspace.pcg(A, b, np.zeros_like(b), lambda r: r / dA, tol=1e-10)
    assert abs(it_same - it_j) <= max(2, 0.02 * it_j)
    print(f"cfl ratio {cfl_ratio}: aux-space PCG {it} iterations, Jacobi PCG {it_j}")


def _morton_brute(mesh, nodes):
    """Morton order by string interleaving of the 21-bit quantized coordinates."""
    lo, hi = mesh.xyz.min(axis=0), mesh.xyz.max(axis=0)
    keys = []
    for v in nodes:
        q = [int(min(2097151.0, max(0.0, (mesh.xyz[v, d] - lo[d]) / (hi[d] - lo[d]) * 2097151.0)))
             for d in range(3)]
        bits = [format(x, "021b") for x in q]            # most significant bit first
        keys.append("".join(bits[2][i] + bits[1][i] + bits[0][i] for i in range(21)))   # z y x per level
    return [v for _, v in sorted(zip(keys, nodes), key=lambda kv: kv[0])]


def test_morton_order_and_aggregate_locality():
    m = Mesh(*_jittered_kuhn(9, 5, amp=0.02))
    order = auxspace.morton_order(m, m.interior_nodes)
    assert list(order) == _morton_brute(m, m.interior_nodes)
    # a space-filling curve: runs of 8 consecutive nodes of the 8^3 interior lattice are
    # compact (each lies within a small box of lattice cells)
    h = 1.0 / 9
    ext = [np.ptp(m.xyz[order[k:k + 8]], axis=0).max() for k in range(0, len(order), 8)]
    assert np.median(ext) <= 1.2 * h and max(ext) <= 4.2 * h


def test_coarse_vector_level_interpolates_uniform_fields(mesh):
    """One aggregate holding every interior node: its Pi-level basis for component d is
    the field that is e_d at interior nodes (zero at the wall), whose unknowns on edges
    with both ends interior are the line integrals of the uniform field e_d."""
    ie, inode = mesh.interior_edges, auxspace.morton_order(mesh, mesh.interior_nodes)
    Pi = auxspace.vector_interpolation_matrix(mesh, ie, inode)
    P = auxspace.aggregation_matrix(len(inode), len(inode))
    Q = (Pi @ sp.kron(P, sp.identity(3))).toarray()
    both = ~mesh.boundary_node[mesh.edges[ie]].any(axis=1)
    for d in range(3):
        u = np.eye(3)[d]
        assert np.allclose(Q[both, d], mesh.edge_dofs_of_uniform_field(u)[ie][both], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("levels", [(8,), (8, 64)])
def test_multilevel_preconditioner(mesh, levels):
    A = _newmark_A(mesh, 20.0)
    apply1 = auxspace.aux_space_preconditioner(A, mesh)[0]
    apply = auxspace.aux_space_preconditioner(A, mesh, levels=levels)[0]
    rng = np.random.default_rng(6)
    x, y = rng.normal(size=(2, A.shape[0]))
    assert abs(x @ apply(y) - y @ apply(x)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(apply(y))
    assert x @ apply(x) > x @ apply1(x) > 0        # the levels add positive semi-definite terms
    b = rng.normal(size=A.shape[0])
    x_direct = spla.spsolve(A.tocsc(), b)
    xs, it, res = auxspace.pcg(A, b, np.zeros_like(b), apply, tol=1e-10)
    _, it1, _ = auxspace.pcg(A, b, np.zeros_like(b), apply1, tol=1e-10)
    assert res <= 1e-10 and np.linalg.norm(xs - x_direct) <= 1e-8 * np.linalg.norm(x_direct)
    assert it < it1
    print(f"levels {levels}: {it} iterations, one level {it1}")


def test_fp32_preconditioner_is_the_rounded_fp64_one(mesh):
    A = _newmark_A(mesh, 20.0)
    apply64 = auxspace.aux_space_preconditioner(A, mesh, levels=(8, 64))[0]
    apply32 = auxspace.aux_space_preconditioner(A, mesh, levels=(8, 64), dtype=np.float32)[0]
    r = np.random.default_rng(10).normal(size=A.shape[0])
    z64, z32 = apply64(r), apply32(r.astype(np.float32))
    assert z32.dtype == np.float32
    assert np.linalg.norm(z32 - z64) <= 1e-5 * np.linalg.norm(z64)


@pytest.mark.parametrize("cfl_ratio", [5.0, 20.0])
def test_refined_pcg_meets_the_fp64_tolerance(mesh, cfl_ratio):
    """FP32 inner solves with FP64 residuals reach the FP64 stopping rule and the direct
    solve's solution, in a few more iterations than the FP64 PCG; the same refinement
    with its residual formed in FP32 (a planted mistake) stalls far above the tolerance."""
    A = _newmark_A(mesh, cfl_ratio)
    rng = np.random.default_rng(9)
    b = rng.normal(size=A.shape[0])
    x_direct = spla.spsolve(A.tocsc(), b)
    levels = (8, 64)
    apply32 = auxspace.aux_space_preconditioner(A, mesh, levels=levels, dtype=np.float32)[0]
    x, it, passes, res = auxspace.pcg_refined(A, b, np.zeros_like(b), apply32, tol=1e-10, inner_tol=1e-4)
    assert res <= 1e-10 and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - x_direct) <= 1e-8 * np.linalg.norm(x_direct)
    assert passes >= 2          # FP32 alone does not resolve 1e-10: refinement took place
    apply64 = auxspace.aux_space_preconditioner(A, mesh, levels=levels)[0]
    _, it64, _ = auxspace.pcg(A, b, np.zeros_like(b), apply64, tol=1e-10)
    assert it <= 1.3 * it64 + 5
    print(f"cfl ratio {cfl_ratio}: refined {it} iterations in {passes} passes, FP64 PCG {it64}")
    # planted mistake: residuals in FP32
    A32, b32, x32 = A.astype(np.float32), b.astype(np.float32), np.zeros(len(b), dtype=np.float32)
    for _ in range(8):
        r32 = b32 - A32 @ x32
        d, _ = auxspace._pcg_fp32(A32, r32, np.linalg.norm(r32.astype(np.float64)), apply32, 1e-4, 10000)
        x32 = x32 + d
    assert np.linalg.norm(b - A @ x32.astype(np.float64)) > 1e-9 * np.linalg.norm(b)

"""Oracle: Whitney forms and the finite-element matrices of Sec. II-A.

Whitney 1-form of edge (a,b):  W_ab = lambda_a grad lambda_b - lambda_b grad lambda_a,
curl W_ab = 2 grad lambda_a x grad lambda_b.
Whitney 2-form of face (i,j,k): W_ijk = 2 (lambda_i grad l_j x grad l_k
                                         + lambda_j grad l_k x grad l_i
                                         + lambda_k grad l_i x grad l_j).
E = sum_i e_i W1_i, B = sum_f b_f W2_f (Sec. II-A).

Hodge matrices, each written as its defining integral evaluated with a quadrature rule
that is exact for the integrand's polynomial degree:
  [*eps]_ij   = < W1_i, eps0 W1_j >            (edge mass M; degree 2 -> 4-point rule)
  [*mu^-1]_ij = < W2_i, mu0^-1 W2_j >          (face mass; degree 2 -> 4-point rule)
  [*S]        = [curl]^T [*mu^-1] [curl]       (curl-curl; assembled from curl W1 directly)
and the boundary matrix of the surface impedance matrix (Sec. II-A), without its mu^-1:
  K_ij = int over the absorbing faces of (n x W1_i) . (n x W1_j) dS
(degree 2 on each triangle; a 16-point collapsed Gauss rule).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .constants import EPS0, MU0
from .mesh import LOCAL_EDGES, LOCAL_FACES

# Symmetric 4-point rule on the tetrahedron, exact for polynomials of degree <= 2
# (barycentric points (a,b,b,b) and permutations, equal weights 1/4).
_A4 = 0.5854101966249685
_B4 = 0.1381966011250105
QUAD4 = np.array([[_A4, _B4, _B4, _B4], [_B4, _A4, _B4, _B4],
                  [_B4, _B4, _A4, _B4], [_B4, _B4, _B4, _A4]])
QUAD4_W = np.full(4, 0.25)


def whitney1(lam, grad):
    """W1 of the 6 local edges at barycentric point(s) lam [...,4]; grad [...,4,3].
    Returns [..., 6, 3]."""
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    return lam[..., a, None] * grad[..., b, :] - lam[..., b, None] * grad[..., a, :]


def curl_whitney1(grad):
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    return 2.0 * np.cross(grad[..., a, :], grad[..., b, :])


def whitney2(lam, grad):
    """W2 of the 4 local faces (face k opposite vertex k) at lam.  Returns [..., 4, 3]."""
    out = []
    for k in range(4):
        i, j, l = LOCAL_FACES[k]
        w = (lam[..., i, None] * np.cross(grad[..., j, :], grad[..., l, :])
             + lam[..., j, None] * np.cross(grad[..., l, :], grad[..., i, :])
             + lam[..., l, None] * np.cross(grad[..., i, :], grad[..., j, :]))
        out.append(2.0 * w)
    return np.stack(out, axis=-2)


def element_mass(mesh, eps=EPS0):
    """[n_tets, 6, 6] element edge-mass matrices eps * int W1_i . W1_j dV."""
    g = mesh.grad_lambda
    Me = np.zeros((mesh.n_tets, 6, 6))
    for q in range(4):
        W = whitney1(np.broadcast_to(QUAD4[q], (mesh.n_tets, 4)), g)
        Me += QUAD4_W[q] * np.einsum("tid,tjd->tij", W, W)
    return eps * Me * mesh.vol[:, None, None]


def element_curlcurl(mesh, mu=MU0):
    """[n_tets, 6, 6] element matrices mu^-1 int curl W1_i . curl W1_j dV."""
    cw = curl_whitney1(mesh.grad_lambda)
    return np.einsum("tid,tjd->tij", cw, cw) * (mesh.vol / mu)[:, None, None]


def element_face_mass(mesh, mu=MU0):
    g = mesh.grad_lambda
    Fe = np.zeros((mesh.n_tets, 4, 4))
    for q in range(4):
        W = whitney2(np.broadcast_to(QUAD4[q], (mesh.n_tets, 4)), g)
        Fe += QUAD4_W[q] * np.einsum("tid,tjd->tij", W, W)
    return Fe * (mesh.vol / mu)[:, None, None]


def _assemble(local_to_global, Ke, n):
    m = local_to_global.shape[1]
    rows = np.repeat(local_to_global, m, axis=1).ravel()
    cols = np.tile(local_to_global, (1, m)).ravel()
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))


def mass_matrix(mesh):
    """Global edge mass M = [*eps0] over all edges (orientation: every local edge of a
    sorted tet points low -> high id, as the global edge does, so no sign flips)."""
    return _assemble(mesh.tet_edges, element_mass(mesh), mesh.n_edges)


def curlcurl_matrix(mesh):
    """Global S = [curl]^T [*mu^-1] [curl] over all edges."""
    return _assemble(mesh.tet_edges, element_curlcurl(mesh), mesh.n_edges)


def face_mass_matrix(mesh):
    """[*mu^-1] over all faces.  whitney2 of local face k (vertices i<j<l) carries unit
    flux through that face's canonical right-hand normal whatever the tet's orientation
    (both the basis and the normal are pseudovectors), so no sign flips are needed."""
    return _assemble(mesh.tet_faces, element_face_mass(mesh), mesh.n_faces)


def nodal_stiffness(mesh, eps=EPS0):
    """P1 (Whitney-0) stiffness eps int grad lambda_i . grad lambda_j dV, closed form
    (the gradients are constant): eps V grad l_i . grad l_j."""
    g = mesh.grad_lambda
    Ke = eps * np.einsum("tid,tjd->tij", g, g) * mesh.vol[:, None, None]
    return _assemble(mesh.tets, Ke, mesh.n_nodes)


def eval_E(mesh, e, t, lam):
    """E = sum over the 6 edges of tet t of e_i W1_i(lam)."""
    W = whitney1(lam, mesh.grad_lambda[t])
    return np.einsum("...i,...id->...d", e[mesh.tet_edges[t]], W)


def eval_B(mesh, b, t, lam):
    W = whitney2(lam, mesh.grad_lambda[t])
    return np.einsum("...i,...id->...d", b[mesh.tet_faces[t]], W)


# Collapsed (Duffy) 4 x 4 Gauss-Legendre rule on the reference triangle {s, t >= 0,
# s + t <= 1}: exact for polynomials of degree <= 6 there.
def _triangle_rule():
    g, w = np.polynomial.legendre.leggauss(4)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            pts.append((a, b * (1.0 - a)))
            wts.append(wa * wb * (1.0 - a))
    return np.array(pts), np.array(wts)


TRI_PTS, TRI_W = _triangle_rule()       # weights sum to 1/2, the reference area


def boundary_matrix(mesh, faces):
    """K over all edges for the wall faces `faces` (boolean mask or ids): on each face, at
    every quadrature point, the six Whitney-1 functions of the face's tet, crossed with the
    face's unit normal and dotted pairwise.  The tangential trace of an edge function off
    the face vanishes, so only the face's own three edges carry weight."""
    fm = np.zeros(mesh.n_faces, dtype=bool)
    fm[np.asarray(faces)] = True
    rows, cols, vals = [], [], []
    for f in np.nonzero(fm)[0]:
        t = mesh.face_tets[f, 0]
        k = int(np.nonzero(mesh.tet_faces[t] == f)[0][0])
        verts = LOCAL_FACES[k]
        p = mesh.xyz[mesh.faces[f]]
        N = np.cross(p[1] - p[0], p[2] - p[0])
        jac = np.linalg.norm(N)                     # twice the area
        n = N / jac
        lam = np.zeros((len(TRI_W), 4))
        lam[:, verts[0]] = 1.0 - TRI_PTS[:, 0] - TRI_PTS[:, 1]
        lam[:, verts[1]] = TRI_PTS[:, 0]
        lam[:, verts[2]] = TRI_PTS[:, 1]
        W = whitney1(lam, mesh.grad_lambda[t][None])          # [q, 6, 3]
        nW = np.cross(n, W)
        Ke = jac * np.einsum("q,qid,qjd->ij", TRI_W, nW, nW)
        ge = mesh.tet_edges[t]
        rows.append(np.repeat(ge, 6))
        cols.append(np.tile(ge, 6))
        vals.append(Ke.ravel())
    if not rows:
        return sp.csr_matrix((mesh.n_edges, mesh.n_edges))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh.n_edges, mesh.n_edges))

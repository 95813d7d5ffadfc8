"""Oracle: nodal auxiliary-space preconditioner for the Newmark system, and PCG with it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes the Newmark system (M + beta dt^2 S) e^{n+1} = ... (Sec. II-B, III-A) but
not how it is solved.  Jacobi-PCG needs many iterations once dt is well beyond the
explicit limit: the error components that converge slowly are the discrete gradients
(the kernel of S, where only M acts) and the smooth curl fields.  The nodal auxiliary-space
preconditioner of Hiptmair and Xu (SIAM J. Numer. Anal. 45 (2007) 2483-2509) adds a
correction from two nodal spaces to the edge smoother; here every space gets one Jacobi
step, in additive form:

    B = diag(A)^-1 + G diag(G^T A G)^-1 G^T + Pi diag(Pi^T A Pi)^-1 Pi^T,

with, on interior edges (rows) and interior nodes (columns; PEC walls hold the boundary
unknowns at zero):

* G  the discrete gradient: -1 at the tail and +1 at the head of each edge, i.e. the
  incidence matrix D of the mesh restricted to those rows and columns (de Rham: S G = 0);
* Pi the nodal interpolation of piecewise-linear vector fields into Whitney-1 unknowns.
  For a linear field F the edge unknown is its line integral along the edge, which the
  trapezoid rule gives exactly: (r_b - r_a) . (F(r_a) + F(r_b)) / 2, so the entry of Pi
  for edge (a, b) and node n in {a, b}, component d, is (r_b - r_a)_d / 2.

Coarser levels (optional, ``levels``): the one-level form leaves the smooth components of
the two nodal spaces slow.  Each level groups the interior nodes into aggregates of
consecutive nodes in Morton order of their positions (sizes 8, 64, ...), and adds the
same two corrections for the piecewise-constant nodal fields of each aggregate (the
aggregate's summed hat functions for G, and a constant vector over it for Pi), again with
one Jacobi step:  B += sum over levels of Q diag(Q^T A Q)^-1 Q^T, Q = [G P, Pi P3], P the
aggregation (node -> aggregate) matrix.  This is an additive multilevel (BPX-type) scheme
on the auxiliary spaces.  Morton order: each coordinate scaled to [0, 1] over the bounding
box of all nodes, truncated to 21 bits, bits interleaved x, y, z from the lowest; ties
keep node order.

B is symmetric positive definite (a sum of an SPD matrix and symmetric positive
semi-definite ones), so PCG with it converges to the same solution as any other PCG; it
only changes how many iterations that takes.  The stopping rule is the one of
``newmark.pcg_jacobi``: ||r||_2 <= tol ||b||_2 on the updated residual.

Mixed precision (``pcg_refined``): classical iterative refinement (Wilkinson; for CG
inner solves see e.g. Carson and Higham, SIAM J. Sci. Comput. 40 (2018) A817).  The
residual r = b - A x is formed in FP64; the correction d solves A d = r approximately
with the same PCG run in FP32 (A, the preconditioner's inverse diagonals and all
vectors rounded to FP32; inner products and the step lengths alpha, beta in FP64) from
d = 0, until its updated residual is at most max(inner_tol, tol ||b|| / (2 ||r||)) ||r||;
then x += d in FP64, and again until the FP64 residual meets tol ||b||.  Each pass gains
a factor of about inner_tol as long as that exceeds what FP32 can resolve, and the
result satisfies the same stopping rule as the FP64 PCG.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gradient_matrix(mesh, rows, cols):
    """Discrete gradient G = D[rows][:, cols] (edges x nodes, -1 tail, +1 head)."""
    return mesh.D().tocsr()[rows][:, cols].tocsr()


def vector_interpolation_matrix(mesh, rows, nodes):
    """Pi: values of a vector field at `nodes` (3 per node, x y z) -> line integrals of its
    linear interpolant along the edges `rows` (trapezoid rule, exact for linear fields).
    A node outside `nodes` contributes nothing (its field value is taken as zero)."""
    rows = np.asarray(rows)
    nodes = np.asarray(nodes)
    where = -np.ones(mesh.n_nodes, dtype=np.int64)
    where[nodes] = np.arange(len(nodes))
    ends = mesh.edges[rows]
    t = mesh.xyz[ends[:, 1]] - mesh.xyz[ends[:, 0]]
    r_idx, c_idx, vals = [], [], []
    for end in (0, 1):
        k = where[ends[:, end]]
        ok = k >= 0
        for d in range(3):
            r_idx.append(np.nonzero(ok)[0])
            c_idx.append(3 * k[ok] + d)
            vals.append(0.5 * t[ok, d])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(r_idx), np.concatenate(c_idx))),
                         shape=(len(rows), 3 * len(nodes)))


def morton_order(mesh, nodes):
    """`nodes` sorted by the Morton code of their positions (module docstring)."""
    lo, hi = mesh.xyz.min(axis=0), mesh.xyz.max(axis=0)
    ext = hi - lo
    f = np.where(ext > 0, (mesh.xyz[nodes] - lo) / np.where(ext > 0, ext, 1.0), 0.0)
    q = np.minimum(2097151.0, np.maximum(0.0, f * 2097151.0)).astype(np.uint64)
    code = np.zeros(len(nodes), dtype=np.uint64)
    for bit in range(21):
        for d in range(3):
            code |= ((q[:, d] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + d)
    return np.asarray(nodes)[np.argsort(code, kind="stable")]


def aggregation_matrix(n, size):
    """n x ceil(n / size): node k (in Morton order) -> aggregate k // size."""
    k = np.arange(n)
    return sp.csr_matrix((np.ones(n), (k, k // size)), shape=(n, (n + size - 1) // size))


def aux_space_preconditioner(A, mesh, edges=None, nodes=None, levels=(), dtype=np.float64):
    """The additive preconditioner B as a function r -> B r on the unknowns `edges`
    (default: interior edges, the rows of A) with nodal spaces on `nodes` (default:
    interior nodes, taken in Morton order) and aggregation levels of the given sizes.
    With dtype float32, B r is computed in FP32 from the FP32 roundings of the matrices
    and of the inverse diagonals (the diagonals themselves are formed in FP64).
    Returns (apply, G, Pi, dG, dPi) with the fine-level matrices and diagonals."""
    edges = mesh.interior_edges if edges is None else edges
    nodes = morton_order(mesh, mesh.interior_nodes if nodes is None else nodes)
    G = gradient_matrix(mesh, edges, nodes)
    Pi = vector_interpolation_matrix(mesh, edges, nodes)
    dA = A.diagonal()
    dG = (G.T @ (A @ G)).diagonal()
    dPi = (Pi.T @ (A @ Pi)).diagonal()
    coarse = []
    for size in levels:
        P = aggregation_matrix(len(nodes), size)
        P3 = sp.kron(P, sp.identity(3)).tocsr()   # (node, d) -> (aggregate, d)
        for Q in ((G @ P).tocsr(), (Pi @ P3).tocsr()):
            coarse.append((Q, (Q.T @ (A @ Q)).diagonal()))

    def apply(r):
        z = r / dA + G @ ((G.T @ r) / dG) + Pi @ ((Pi.T @ r) / dPi)
        for Q, d in coarse:
            z = z + Q @ ((Q.T @ r) / d)
        return z

    if np.dtype(dtype) == np.float32:
        f = np.float32
        dinv = (1.0 / dA).astype(f)
        terms = [(Q.astype(f).tocsr(), (1.0 / d).astype(f)) for Q, d in [(G, dG), (Pi, dPi)] + coarse]

        def apply32(r):
            r = np.asarray(r, dtype=f)
            z = dinv * r
            for Q, di in terms:
                z = z + Q @ (di * (Q.T @ r))
            return z

        return apply32, G, Pi, dG, dPi
    return apply, G, Pi, dG, dPi


def pcg(A, b, x0, apply_B, tol=1e-10, maxit=10000):
    """Preconditioned CG (Hestenes-Stiefel recurrences), stopping when the updated residual
    satisfies ||r||_2 <= tol ||b||_2.  Returns (x, iterations, true relative residual)."""
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    it = 0
    if np.linalg.norm(r) > tol * bnorm:
        z = apply_B(r)
        p = z.copy()
        rz = r @ z
        while it < maxit:
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            it += 1
            if np.linalg.norm(r) <= tol * bnorm:
                break
            z = apply_B(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
    return x, it, np.linalg.norm(b - A @ x) / bnorm


def _pcg_fp32(A32, b32, bnorm, apply_B32, tol, maxit):
    """The PCG of ``pcg`` from x = 0 with FP32 vectors, FP64 inner products and step
    lengths (rounded to FP32 where they scale a vector); stops when the updated residual
    satisfies ||r||_2 <= tol * bnorm.  Returns (x, iterations)."""
    f = np.float32
    x = np.zeros_like(b32)
    r = b32.copy()
    it = 0
    if np.linalg.norm(r.astype(np.float64)) > tol * bnorm:
        z = apply_B32(r)
        p = z.copy()
        rz = float(r.astype(np.float64) @ z.astype(np.float64))
        while it < maxit:
            q = A32 @ p
            alpha = rz / float(p.astype(np.float64) @ q.astype(np.float64))
            x = x + f(alpha) * p
            r = r - f(alpha) * q
            it += 1
            if np.linalg.norm(r.astype(np.float64)) <= tol * bnorm:
                break
            z = apply_B32(r)
            rz_new = float(r.astype(np.float64) @ z.astype(np.float64))
            p = z + f(rz_new / rz) * p
            rz = rz_new
    return x, it


def pcg_refined(A, b, x0, apply_B32, tol=1e-10, inner_tol=1e-4, max_passes=8, maxit=10000):
    """Mixed-precision iterative refinement around an FP32 PCG (module docstring).
    apply_B32 is the FP32 preconditioner (``aux_space_preconditioner(..., dtype=float32)``).
    Returns (x, total inner iterations, passes, true relative residual)."""
    bnorm = np.linalg.norm(b)
    x = np.array(x0, dtype=np.float64, copy=True)
    if bnorm == 0.0:
        return np.zeros_like(x), 0, 0, 0.0
    A32 = A.astype(np.float32).tocsr()
    total = passes = 0
    while True:
        r = b - A @ x
        rn = np.linalg.norm(r)
        if rn <= tol * bnorm or passes >= max_passes or total >= maxit:
            break
        tol_in = max(inner_tol, 0.5 * tol * bnorm / rn)
        d, it = _pcg_fp32(A32, r.astype(np.float32), rn, apply_B32, tol_in, maxit - total)
        x += d.astype(np.float64)
        total += it
        passes += 1
    return x, total, passes, rn / bnorm

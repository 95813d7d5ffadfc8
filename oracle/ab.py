"""Oracle: the paper's Adams-Bashforth-k particle pusher, its Lagrange-polynomial path, the
cell-by-cell walk along that curved path and the Whitney-1 path integral of each piece.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The library pushes with relativistic
Boris along straight lines; this module is the reference an Adams-Bashforth pusher is to
be tested against, pinned by the tests in tests/test_oracle_ab.py.

Sec. III-B: Newton's equations with the Lorentz force, dv/dt = a = (q/m)(E + v x B),
dr/dt = v (non-relativistic, as the paper writes them), integrated by the k-step
Adams-Bashforth method
    v^{n+1} = v^n + dt sum_{j<k} beta_j a^{n-j},   r^{n+1} = r^n + dt sum_{j<k} beta_j v^{n-j}.
beta_j is the integral over one step of the Lagrange basis polynomial of the past time
t_{n-j} on the k past times t_n, ..., t_{n-k+1} (computed here in exact rational
arithmetic; the paper prints k = 4).  The path over the step is the Lagrange polynomial
through the k + 1 positions r^{n+1}, r^n, ..., r^{n+1-k}, parameterized by s = (t - t_n)/dt
in [0, 1].

Sec. III-C, Alg. 1 and Alg. 2: the path is followed cell by cell.  Where it leaves the
current cell is found by bisection in s between a point inside and the first of the
remaining interval's Gauss-Legendre points (or its end) found outside, until the bracket is
narrower than `tol`; the exit face is the one whose barycentric coordinate is most negative
at the bracket's outer end, and the path continues in the neighbour across it (a wall
face absorbs the particle).  Each piece adds to the time-integrated current the path
integral of the cell's Whitney-1 functions, q w int W_ab(r(s)) . r'(s) ds, by
Gauss-Legendre quadrature with k + 1 points, which is exact: W is linear in r, r(s) has
degree k and r'(s) degree k - 1, so the integrand has degree 2k - 1.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from .mesh import LOCAL_EDGES


def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def ab_coefficients(k):
    """beta_0 .. beta_{k-1} as Fractions: the integral over s in [0, 1] of the Lagrange
    basis polynomials on the nodes s = 0, -1, ..., -(k - 1)."""
    if not 1 <= k:
        raise ValueError("order must be at least 1")
    nodes = [Fraction(-j) for j in range(k)]
    betas = []
    for j in range(k):
        poly, den = [Fraction(1)], Fraction(1)
        for m in range(k):
            if m != j:
                poly = _poly_mul(poly, [-nodes[m], Fraction(1)])
                den *= nodes[j] - nodes[m]
        betas.append(sum(c / (i + 1) for i, c in enumerate(poly)) / den)
    return betas


def ab_step(r_hist, v_hist, a_hist, dt, k):
    """One Adams-Bashforth step of order min(k, len(a_hist)).  r_hist[0] = r^n, v_hist[j] =
    v^{n-j}, a_hist[j] = a^{n-j} (arrays [..., 3]).  Returns (r^{n+1}, v^{n+1})."""
    m = min(k, len(a_hist), len(v_hist))
    beta = [float(b) for b in ab_coefficients(m)]
    r_new = np.asarray(r_hist[0], dtype=np.float64) + dt * sum(beta[j] * np.asarray(v_hist[j]) for j in range(m))
    v_new = np.asarray(v_hist[0], dtype=np.float64) + dt * sum(beta[j] * np.asarray(a_hist[j]) for j in range(m))
    return r_new, v_new


class LagrangePath:
    """r(s) through points[j] at s = nodes[j] (points [m + 1, 3]); r(s) and r'(s)."""

    def __init__(self, nodes, points):
        self.nodes = np.asarray(nodes, dtype=np.float64)
        self.points = np.asarray(points, dtype=np.float64)

    def _basis(self, s):
        x = self.nodes
        n = len(x)
        l = np.ones(n)
        dl = np.zeros(n)
        for j in range(n):
            for m in range(n):
                if m == j:
                    continue
                l[j] *= (s - x[m]) / (x[j] - x[m])
            for i in range(n):
                if i == j:
                    continue
                term = 1.0 / (x[j] - x[i])
                for m in range(n):
                    if m != j and m != i:
                        term *= (s - x[m]) / (x[j] - x[m])
                dl[j] += term
        return l, dl

    def __call__(self, s):
        l, _ = self._basis(s)
        return l @ self.points

    def deriv(self, s):
        _, dl = self._basis(s)
        return dl @ self.points


def step_path(r_new, r_hist):
    """The path of one step: the Lagrange polynomial through r^{n+1} (s = 1), r^n (s = 0),
    r^{n-1} (s = -1), ... for the given history r_hist = [r^n, r^{n-1}, ...]."""
    pts = [np.asarray(r_new, dtype=np.float64)] + [np.asarray(r, dtype=np.float64) for r in r_hist]
    return LagrangePath([1.0 - j for j in range(len(pts))], pts)


def _inside(mesh, t, x, eps):
    return mesh.barycentric(t, x).min() >= -eps


def walk_curved(mesh, tet, path, n_gl, tol=1e-15, eps=1e-13, cap=64):
    """Pieces (tet, s_a, s_b) of path over s in [0, 1] starting in tet; the second value is
    the final tet, or -1 if the path reached a wall (absorbed) or the crossing cap."""
    g, _ = np.polynomial.legendre.leggauss(n_gl)
    pieces = []
    s_a = 0.0
    for _ in range(cap + 1):
        cand = list(s_a + (1.0 - s_a) * 0.5 * (g + 1.0)) + [1.0]
        out = next((s for s in cand if not _inside(mesh, tet, path(s), eps)), None)
        if out is None:
            pieces.append((tet, s_a, 1.0))
            return pieces, tet
        lo, hi = s_a, out
        while hi - lo > tol:
            mid = 0.5 * (lo + hi)
            if _inside(mesh, tet, path(mid), eps):
                lo = mid
            else:
                hi = mid
        s_x = 0.5 * (lo + hi)
        pieces.append((tet, s_a, s_x))
        k = int(np.argmin(mesh.barycentric(tet, path(hi))))
        nb = int(mesh.nbr[tet, k])
        if nb < 0:
            return pieces, -1
        tet, s_a = nb, s_x
    return pieces, -1


def deposit_curved(mesh, pieces, path, qw, n_gl, g=None):
    """Adds q w int W_ab(r(s)) . r'(s) ds over each piece, by Gauss-Legendre quadrature with
    n_gl points, into g (edge vector, created if None); returns g."""
    if g is None:
        g = np.zeros(mesh.n_edges)
    x, w = np.polynomial.legendre.leggauss(n_gl)
    for tet, s_a, s_b in pieces:
        half = 0.5 * (s_b - s_a)
        grad = mesh.grad_lambda[tet]
        acc = np.zeros(6)
        for xq, wq in zip(x, w):
            s = s_a + half * (xq + 1.0)
            lam = mesh.barycentric(tet, path(s))
            dl = grad @ path.deriv(s)                      # d lambda_k / ds
            a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
            acc += wq * (lam[a] * dl[b] - lam[b] * dl[a])
        g[mesh.tet_edges[tet]] += qw * half * acc
    return g

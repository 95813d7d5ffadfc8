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

Closing the pieces at a crossing (a reading: Sec. III-A states that D^T g = q w (lambda
at the end - lambda at the start) holds exactly, while the bisection only brackets the
crossing to within its tolerance, so the point r(s_x) where a piece ends lies near the
face, not on it, and the two cells' barycentric coordinates of that point differ).  Each
piece is closed onto the face: with L the exit cell's coordinates of r(s_x) and k the exit
face, the face point P has P_k = 0 and P_j = L_j + L_k / 3 for the other three; the exit
cell adds the straight segment L -> P, and the next cell starts with the straight segment
from P (the same three numbers on the shared vertices, 0 on its far vertex) to its own
coordinates of r(s_x).  A straight segment from barycentric point A to B in one cell adds
q w (m_a d_b - m_b d_a) to edge (a, b), m = (A + B) / 2 and d = B - A (the integrand is
constant along it, so this is exact).  The closures are of the size of the bisection
tolerance, and the coordinates at the shared face point are identical on both sides, so
the pieces telescope and D^T g = q w (lambda_end - lambda_start) holds to round-off.
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


def face_point(lam, k):
    """The point of face k (opposite local vertex k) closing a piece that ends at barycentric
    point lam: coordinate k set to 0, its value shared equally by the other three."""
    p = np.asarray(lam, dtype=np.float64) + lam[k] / 3.0
    p[k] = 0.0
    return p


def to_neighbour(mesh, tet, nb, p):
    """Barycentric point p of tet, lying on the face shared with nb, in nb's local order
    (matched by global vertex id; 0 on nb's far vertex)."""
    out = np.zeros(4)
    for j in range(4):
        hit = np.nonzero(mesh.tets[tet] == mesh.tets[nb, j])[0]
        if len(hit):
            out[j] = p[hit[0]]
    return out


def walk_curved(mesh, tet, path, n_gl, tol=1e-15, eps=1e-13, cap=64):
    """Pieces (tet, s_a, s_b, p_in, p_out) of path over s in [0, 1] starting in tet: p_in is
    the face point (barycentric, in this tet) the piece starts from after a crossing, p_out
    the face point it closes onto before the next (None at the ends of the path).  The
    second value is the final tet, or -1 if the path reached a wall (absorbed) or the
    crossing cap."""
    g, _ = np.polynomial.legendre.leggauss(n_gl)
    pieces = []
    s_a, p_in = 0.0, None
    for _ in range(cap + 1):
        cand = list(s_a + (1.0 - s_a) * 0.5 * (g + 1.0)) + [1.0]
        out = next((s for s in cand if not _inside(mesh, tet, path(s), eps)), None)
        if out is None:
            pieces.append((tet, s_a, 1.0, p_in, None))
            return pieces, tet
        lo, hi = s_a, out
        while hi - lo > tol:
            mid = 0.5 * (lo + hi)
            if _inside(mesh, tet, path(mid), eps):
                lo = mid
            else:
                hi = mid
        s_x = 0.5 * (lo + hi)
        k = int(np.argmin(mesh.barycentric(tet, path(hi))))
        p_out = face_point(mesh.barycentric(tet, path(s_x)), k)
        pieces.append((tet, s_a, s_x, p_in, p_out))
        nb = int(mesh.nbr[tet, k])
        if nb < 0:
            return pieces, -1
        p_in = to_neighbour(mesh, tet, nb, p_out)
        tet, s_a = nb, s_x
    return pieces, -1


def segment_integral(lam_a, lam_b):
    """int W_ab . dr for the 6 local edges along the straight segment from barycentric point
    lam_a to lam_b of one cell (W . dr = lambda_a d lambda_b - lambda_b d lambda_a is
    constant along it)."""
    m = 0.5 * (np.asarray(lam_a) + np.asarray(lam_b))
    d = np.asarray(lam_b) - np.asarray(lam_a)
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    return m[a] * d[b] - m[b] * d[a]


def piece_integral(mesh, piece, path, n_gl):
    """int W . dr over one piece's curved part (Gauss-Legendre, n_gl points), without the
    closures."""
    tet, s_a, s_b = piece[:3]
    x, w = np.polynomial.legendre.leggauss(n_gl)
    half = 0.5 * (s_b - s_a)
    grad = mesh.grad_lambda[tet]
    acc = np.zeros(6)
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    for xq, wq in zip(x, w):
        s = s_a + half * (xq + 1.0)
        lam = mesh.barycentric(tet, path(s))
        dl = grad @ path.deriv(s)                      # d lambda_k / ds
        acc += wq * (lam[a] * dl[b] - lam[b] * dl[a])
    return half * acc


def deposit_curved(mesh, pieces, path, qw, n_gl, g=None):
    """Adds q w int W_ab . dr over each piece (its curved part by Gauss-Legendre quadrature
    with n_gl points, and its straight closures onto the faces it enters and leaves by) into
    g (edge vector, created if None); returns g."""
    if g is None:
        g = np.zeros(mesh.n_edges)
    for piece in pieces:
        tet, s_a, s_b, p_in, p_out = piece
        acc = piece_integral(mesh, piece, path, n_gl)
        if p_in is not None:
            acc = acc + segment_integral(p_in, mesh.barycentric(tet, path(s_a)))
        if p_out is not None:
            acc = acc + segment_integral(mesh.barycentric(tet, path(s_b)), p_out)
        g[mesh.tet_edges[tet]] += qw * acc
    return g


AB_MAX = 5      # highest order; a particle keeps its last AB_MAX positions and velocities


class Histories:
    """Per particle (by id) of one species: past positions r^n, r^{n-1}, ..., velocities
    v^n, v^{n-1}, ... and accelerations a^{n-1}, a^{n-2}, ... (newest first).  A particle
    without a history starts at order 1 and gains one order per step; all histories
    restart when dt changes (the coefficients assume equally spaced levels)."""

    def __init__(self):
        self.r, self.v, self.a = {}, {}, {}
        self.dt = None

    def forget(self, pid):
        for d in (self.r, self.v, self.a):
            d.pop(pid, None)


def push_species(mesh, ids, x, u, tet, alive, q, m, w, dt, order, e, b, g, hist, cap=64):
    """One Adams-Bashforth step of order `order` for every live particle of a species, in
    place: x (positions), u (velocities), tet, alive; the current of every piece (with its
    face closures) is added to g.  Returns (crossings, absorbed, cap exceeded)."""
    from . import fem

    if hist.dt != dt:
        hist.r.clear()
        hist.v.clear()
        hist.a.clear()
        hist.dt = dt
    n_cross = n_abs = n_cap = 0
    for i in np.nonzero(alive)[0]:
        pid = int(ids[i])
        t = int(tet[i])
        r_h = hist.r.get(pid, [x[i].copy()])
        v_h = hist.v.get(pid, [u[i].copy()])
        a_h = hist.a.get(pid, [])
        lam = mesh.barycentric(t, r_h[0])
        E = fem.eval_E(mesh, e, t, lam)
        B = fem.eval_B(mesh, b, t, lam)
        a_h = [(q / m) * (E + np.cross(v_h[0], B))] + a_h
        k = min(order, len(a_h))
        r_new, v_new = ab_step(r_h, v_h, a_h, dt, order)
        path = step_path(r_new, r_h[:k])
        pieces, last = walk_curved(mesh, t, path, n_gl=k + 1, cap=cap)
        deposit_curved(mesh, pieces, path, q * w, n_gl=k + 1, g=g)
        n_cross += len(pieces) - 1
        if last < 0:
            alive[i] = 0
            hist.forget(pid)
            if len(pieces) > cap:
                n_cap += 1
            else:
                n_abs += 1
            continue
        tet[i] = last
        x[i] = r_new
        u[i] = v_new
        hist.r[pid] = [r_new] + r_h[:AB_MAX - 1]
        hist.v[pid] = [v_new] + v_h[:AB_MAX - 1]
        hist.a[pid] = a_h[:AB_MAX - 1]
    return n_cross, n_abs, n_cap

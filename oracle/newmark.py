"""Oracle: Newmark-beta field update with the time-integrated current as source.

Semi-discrete wave equation (Sec. II-A, eq. (wave_cont)) with PEC walls (no impedance
term):  M d_t^2 e + S e = -d_t j,   M = [*eps0], S = [curl]^T [*mu0^-1] [curl].

Sec. III-A replaces d_t j by d_t^2 G with G^n = int_0^{t_n} j dt (eq. (G)) and gives the
source the same temporal stencil as the mass term, so that applying the weak divergence
reproduces rho^{n+1} - 2 rho^n + rho^{n-1} whatever the integrator.  With the general
three-level Newmark recurrence (Zienkiewicz; Sec. II-B prints the beta = 1/4, gamma = 1/2
case, with misprinted coefficients):

  (M + beta dt^2 S) e^{n+1} = (2M - (1/2 - 2 beta + gamma) dt^2 S) e^n
                              - (M + (1/2 + beta - gamma) dt^2 S) e^{n-1}
                              - (G^{n+1} - 2 G^n + G^{n-1}).

Boundary (PEC, eq. (dirichlet) with Psi_D = 0): tangential E vanishes, so boundary edge
unknowns are 0 and the system is solved on interior edges only.

First-order absorbing faces (eq. (impedanceBC) with Psi_I = 0, differentiated in time and
combined with Faraday's law, Sec. II-A): the boundary term of the weak curl-curl form
becomes a damping term C d_t e, C = Y K with Y = 1 / (mu0 c) the admittance of free space
and K the boundary matrix (oracle/fem.py), and the edges on those faces become unknowns.
The Newmark recurrence of M e'' + C e' + S e = f (velocity term weighted by gamma):
  (M + gamma dt C + beta dt^2 S) e^{n+1} = (2M - (1 - 2 gamma) dt C - (1/2 - 2 beta + gamma)
        dt^2 S) e^n + (-M + (1 - gamma) dt C - (1/2 + beta - gamma) dt^2 S) e^{n-1} - ...
At beta = 1/4, gamma = 1/2 and with no source the energy E^{n+1/2} = 1/2 |e^{n+1} - e^n|_M^2
/ dt^2 + 1/2 |(e^{n+1} + e^n) / 2|_S^2 drops by exactly (e^{n+1} - e^{n-1})^T C (e^{n+1} -
e^{n-1}) / (4 dt) per step.  D^T C vanishes on interior nodes (an edge on a wall face has
both ends on the wall), so the Gauss identities there are untouched.

Faraday (eq. (faraday)) advances the face fluxes: b^{n+1} = b^n - dt C (gamma e^{n+1} +
(1 - gamma) e^n); for gamma = 1/2 this is the trapezoid rule.  D2 C = 0 keeps D2 b fixed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def newmark_operators(M, S, dt, beta, gamma, Cd=None):
    """(A, B1, B2) with A e^{n+1} = B1 e^n + B2 e^{n-1} - Delta^2 G; Cd the damping matrix
    of absorbing faces (None: PEC only)."""
    A = M + (beta * dt * dt) * S
    B1 = 2.0 * M - ((0.5 - 2.0 * beta + gamma) * dt * dt) * S
    B2 = -M - ((0.5 + beta - gamma) * dt * dt) * S
    if Cd is not None:
        A = A + (gamma * dt) * Cd
        B1 = B1 - ((1.0 - 2.0 * gamma) * dt) * Cd
        B2 = B2 + ((1.0 - gamma) * dt) * Cd
    return A.tocsr(), B1.tocsr(), B2.tocsr()


def damped_energy(M, S, e_np1, e_n, dt):
    """E^{n+1/2} = 1/2 |e^{n+1} - e^n|_M^2 / dt^2 + 1/2 |(e^{n+1} + e^n) / 2|_S^2."""
    d, a = e_np1 - e_n, 0.5 * (e_np1 + e_n)
    return 0.5 * float(d @ (M @ d)) / (dt * dt) + 0.5 * float(a @ (S @ a))


def restrict(Mat, idx):
    return Mat[idx][:, idx].tocsr()


def newmark_rhs(B1, B2, e_n, e_nm1, d2G):
    return B1 @ e_n + B2 @ e_nm1 - d2G


def pcg_jacobi(A, b, x0, tol=1e-10, maxit=10000):
    """Jacobi-preconditioned conjugate gradients, stopping when the updated residual
    satisfies ||r||_2 <= tol ||b||_2.  Returns (x, iterations, true relative residual)."""
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    dinv = 1.0 / A.diagonal()
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    it = 0
    if np.linalg.norm(r) > tol * bnorm:
        z = dinv * r
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
            z = dinv * r
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
    true = np.linalg.norm(b - A @ x) / bnorm
    return x, it, true


def faraday(C, b_n, e_np1, e_n, dt, gamma):
    return b_n - dt * (C @ (gamma * e_np1 + (1.0 - gamma) * e_n))


def cg_plain(A, b, tol=1e-14, maxit=100000):
    """Unpreconditioned CG from zero (used for the electrostatic start)."""
    return pcg_jacobi(A, b, np.zeros_like(b), tol, maxit)


def field_energy(M, e, Mf=None, b=None):
    """Electric energy 1/2 e^T M e (+ magnetic 1/2 b^T [*mu^-1] b when given)."""
    w = 0.5 * float(e @ (M @ e))
    if Mf is not None and b is not None:
        w += 0.5 * float(b @ (Mf @ b))
    return w


def dense_check_matrix(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A)

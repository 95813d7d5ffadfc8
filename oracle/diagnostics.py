"""Oracle: nodal charge and the conservation residuals of Sec. III-A.

rho_k = q w lambda_k(x_p) summed over particles (Whitney-0 moment of a point charge,
Sec. II-A delta-function shapes).  With the weak divergence [div] = -D^T:

* continuity  (eqs. (chargeDef), (gaussredo)): rho^{n+1} - rho^n = D^T (G^{n+1} - G^n);
* Gauss       (Sec. II-A, eq. (goodNmB)):       -D^T M e^n = rho^n.

Both are checked on interior nodes (every edge touching an interior node is an interior
edge, so the identities are exact there).  Because e^{n+1} comes from an iterative solve
(Sec. III-A notes the error is "small but not identically zero"), the Gauss residual
r_G = -D^T M e - rho obeys  r_G^{n+1} - 2 r_G^n + r_G^{n-1} = D^T r_cg^{n+1}, with
r_cg = b - A e^{n+1} the solver's residual; that identity is checked to round-off.
"""
from __future__ import annotations

import numpy as np


def nodal_charge(mesh, tet, lam, qw, n_nodes):
    rho = np.zeros(n_nodes)
    if len(tet):
        np.add.at(rho, mesh.tets[tet].ravel(), (qw * lam).ravel())
    return rho


def divergence_T(D, g):
    """D^T g: net edge quantity flowing into each node."""
    return D.T @ g


def continuity_residual(D, rho_new, rho_old, dG, interior_nodes):
    r = (rho_new - rho_old) - D.T @ dG
    return r[interior_nodes]


def gauss_residual(D, M, e, rho, interior_nodes):
    r = -(D.T @ (M @ e)) - rho
    return r[interior_nodes]


def kinetic_energy(u, w, m, c):
    """Sum over particles of w m c^2 (gamma - 1), gamma = sqrt(1 + |u|^2/c^2), u = gamma v
    (relativistic kinetic energy of macro-particles of weight w), written with
    gamma - 1 = (|u|^2/c^2) / (gamma + 1) to avoid cancellation at low speed."""
    q = np.sum(np.asarray(u, dtype=np.float64) ** 2, axis=1) / c ** 2
    return float(w * m * c ** 2 * np.sum(q / (np.sqrt(1.0 + q) + 1.0)))


def magnetic_energy(Mf, b):
    """1/2 b^T [*mu0^-1] b = 1/(2 mu0) int |B|^2 for the Whitney-2 field of the face fluxes b."""
    return 0.5 * float(b @ (Mf @ b))

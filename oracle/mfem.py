"""Oracle: the mixed finite element (MFEM) field update, face fluxes b and edge unknowns e
advanced together, with the time-integrated current G as source.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Semi-discrete system (Sec. II-A, eq. (maxwell_semi), written in SI with PEC walls):
    d_t b + C e = 0                          (Faraday; C the face-edge incidence)
    M d_t e - C^T Mf b = -j                  (Ampere tested with W1; M = [*eps0],
                                              Mf = [*mu0^-1] the Whitney-2 mass)
so that, with K the skew operator of the pair, the energy W = 1/2 (b^T Mf b + e^T M e)
obeys d_t W = -e^T j.

NM-MFEM (Sec. II-B): the three-level Newmark recurrence of Zienkiewicz for a first-order
system (no second-derivative term), beta = 1/4, gamma = 1/2:
    1/2 C_M (X^{n+1} - X^{n-1}) + dt K_M (X^{n+1} + 2 X^n + X^{n-1}) / 4 = (source)
(the printed coefficients and signs are garbled; this is the recurrence they cite).  Sec.
III-A replaces the current by the time derivative of G, which makes the source of the
e-row -1/2 (G^{n+1} - G^{n-1}) (eq. (goodNmB), first form): applying -D^T then gives
1/2 (rho^{n+1} - rho^{n-1}) on both sides.  Eliminating b^{n+1} with the b-row,
    (M + dt^2/4 S) e^{n+1} = M e^{n-1} + dt C^T Mf (b^n + b^{n-1})
                             - dt^2 S (e^n / 2 + e^{n-1} / 4) - (G^{n+1} - G^{n-1}),
    b^{n+1} = b^{n-1} - dt C (e^n + (e^{n+1} + e^{n-1}) / 2),
with S = C^T Mf C: the operator of the wave-equation update at beta = 1/4.  With the
two-step averages y^{n+1/2} = (X^{n+1} + X^n) / 2 the recurrence is the trapezoid rule,
so in vacuum the energy of the averages is conserved.

BD-MFEM: backward differences (backward Euler, a reading: Sec. IV-B names the scheme
only), with the same substitution of the current by the step's increment of G:
    (M + dt^2 S) e^{n+1} = M e^n + dt C^T Mf b^n - (G^{n+1} - G^n),
    b^{n+1} = b^n - dt C e^{n+1};
-D^T gives rho^{n+1} - rho^n on both sides.  In vacuum the energy drops by exactly
1/2 (|b^{n+1} - b^n|^2_Mf + |e^{n+1} - e^n|^2_M) per step.

Gauss drift identities (r_G = -D^T M e - rho, r_cg the solve's residual on interior edges):
NM-MFEM  r_G^{n+1} - r_G^{n-1} = D^T r_cg;   BD-MFEM  r_G^{n+1} - r_G^n = D^T r_cg.
"""
from __future__ import annotations

import numpy as np


def nm_rhs(M, S, CtMf, dt, e_n, e_nm1, b_n, b_nm1, dG_new, dG_old):
    """Right-hand side of the NM-MFEM e-update on all edges (restrict to interior rows)."""
    return (M @ e_nm1 + dt * (CtMf @ (b_n + b_nm1)) - dt * dt * (S @ (0.5 * e_n + 0.25 * e_nm1))
            - (dG_new + dG_old))


def nm_faraday(C, dt, b_nm1, e_np1, e_n, e_nm1):
    return b_nm1 - dt * (C @ (e_n + 0.5 * (e_np1 + e_nm1)))


def bd_rhs(M, CtMf, dt, e_n, b_n, dG_new):
    return M @ e_n + dt * (CtMf @ b_n) - dG_new


def bd_faraday(C, dt, b_n, e_np1):
    return b_n - dt * (C @ e_np1)


def energy(M, Mf, e, b):
    return 0.5 * float(e @ (M @ e) + b @ (Mf @ b))

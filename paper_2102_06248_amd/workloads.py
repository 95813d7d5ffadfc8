"""Synthetic workloads (meshes, particle sets, step parameters) built from ``inputs``.

Stand-ins for the paper's test problems (Sec. IV), whose meshes and data are not
published: an electron beam in a PEC cylinder (Sec. IV-B) and an expanding neutral plasma
(Sec. IV-C), at the sizes given below.  Only input construction lives here.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs

E_CHARGE = inputs.ELEMENTARY_CHARGE
M_E = inputs.ELECTRON_MASS


def c1_single_electron():
    """1 m cube, 6^3 Kuhn cubes (1296 tets), B = 0.1 T z, one electron, v_perp = 1e5 m/s,
    dt = gyroperiod / 50, 2000 steps, all FP64."""
    xyz, tets = inputs.kuhn_cube(6)
    B0, v0 = 0.1, 1e5
    gam = 1.0 / math.sqrt(1.0 - (v0 / inputs.SPEED_OF_LIGHT) ** 2)
    om = E_CHARGE * B0 / (gam * M_E)
    rL = gam * M_E * v0 / (E_CHARGE * B0)
    c = np.full(3, 5.0 / 12.0)
    return dict(name="c1_single_electron", xyz=xyz, tets=tets, B0=[0.0, 0.0, B0],
                species=[dict(q=-E_CHARGE, m=M_E, w=1.0, x=np.array([c + [rL, 0, 0]]),
                              u=np.array([[0.0, gam * v0, 0.0]]))],
                dt=2 * math.pi / om / 50, beta=0.25, gamma=0.5, steps=2000, precision=1)


def c2_beam(n_particles=1_000_000, seed=0, n_rings=12, n_layers=78):
    """Electron beam in a PEC cylinder r = 0.05 m, L = 0.5 m (hex-ring prism mesh,
    12 rings x 78 layers = 202,176 tets); macro-particles uniform on the disk r <= 0.01 m,
    filling z in [0, 0.5) (the steady state of a 0.25 A beam injected at z = 0), 1 keV drift
    along z with a 1 eV Gaussian thermal spread; dt = 1e-10 s; weight from the injection
    rate of 3,750 macro-particles per step carrying 0.25 A.  The beam drifts as a whole,
    so particles sorted by tet stay nearly sorted: re-sorting every 4th step is enough.
    Newmark solve: FP64 residuals around FP32 inner solves that each reduce the residual
    by 1e-5 (two passes per step)."""
    xyz, tets = inputs.prism_cylinder(0.05, 0.5, n_rings, n_layers)
    dt = 1e-10
    per_step = 3750
    w = 0.25 * dt / (per_step * E_CHARGE)
    x, u = inputs.beam_particles(n_particles, 0.01, 0.0, 0.5, 1000.0, 1.0, M_E, seed)
    return dict(name="c2_beam", xyz=xyz, tets=tets, B0=None,
                species=[dict(q=-E_CHARGE, m=M_E, w=w, x=x, u=u)], dt=dt, beta=0.25, gamma=0.5,
                inject_per_step=per_step, precision=0, sort_period=4, solve="mixed", inner_tol=1e-5)


def c2_injection_batch(step, seed=0, per_step=3750):
    """The macro-particles injected at z = 0 in a given step (seeded per step)."""
    return inputs.beam_particles(per_step, 0.01, 0.0, 0.0, 1000.0, 1.0, M_E, seed * 100003 + 7919 + step)


def c3_plasma(n_pairs=8_000_000, n_cells=55, seed=0):
    """Neutral plasma ball: Kuhn mesh of [-4, 4]^3 cm (55^3 cubes, 998,250 tets), electrons
    and protons (mass ratio 1836) co-located in pairs from a Gaussian of width 1 cm
    truncated at 3.9 sigma, Te = 1 eV, Ti = 0.1 eV; peak density 2.5e13 m^-3 sets the
    weight; dt = 0.05 / omega_pe.  Newmark solve: FP64 residuals around FP32 inner solves
    that each reduce the residual by 2e-4 (three passes; 3e-4 and 5e-4 take a fourth pass
    on some steps, and deeper FP32 passes converge more slowly here),
    started from the quadratic extrapolation of the last three fields (the smooth
    expansion makes it a better start than e^n: 144.5 iterations per step against 165.4).
    Each species is re-binned by tet when a 64th of it has left its tet since its last
    re-binning (the electrons every step, the protons every few dozen steps)."""
    xyz, tets = inputs.kuhn_cube(n_cells, lo=(-0.04,) * 3, hi=(0.04,) * 3)
    m_p = inputs.PROTON_ELECTRON_MASS_RATIO * M_E
    x, ue, ui = inputs.gaussian_ball_pairs(n_pairs, 0.01, 3.9, 1.0, 0.1, M_E, m_p, seed)
    n0 = 2.5e13
    total = n0 * (2 * math.pi) ** 1.5 * 0.01 ** 3
    w = total / n_pairs
    eps0 = 8.8541878128e-12
    wpe = math.sqrt(n0 * E_CHARGE ** 2 / (eps0 * M_E))
    return dict(name="c3_plasma", xyz=xyz, tets=tets, B0=None,
                species=[dict(q=-E_CHARGE, m=M_E, w=w, x=x, u=ue), dict(q=E_CHARGE, m=m_p, w=w, x=x, u=ui)],
                dt=0.05 / wpe, beta=0.25, gamma=0.5, precision=0, solve="mixed", inner_tol=2e-4,
                warm_start="extrap2", sort_period=-1)


def c5_plasma(n_pairs=64_000_000, n_cells=110, seed=0):
    """The plasma ball of c3_plasma refined twice over: Kuhn mesh 110^3 of the same 8 cm cube
    (7,986,000 tets), 64M electron/proton pairs (the same plasma, 8x more macro-particles
    of 1/8 the weight), the same dt; FP32 passes of the Newmark solve reduce the residual
    by 2e-3 each (four passes; deeper passes converge more slowly on this mesh and still
    take four, 3e-3 takes five)."""
    return c3_plasma(n_pairs=n_pairs, n_cells=n_cells, seed=seed) | {"name": "c5_plasma", "inner_tol": 2e-3}


WORKLOADS = {"c2_beam": c2_beam, "c3_plasma": c3_plasma, "c5_plasma": c5_plasma}

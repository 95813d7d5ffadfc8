"""Oracle: one whole PIC step, in the cycle order of Sec. II-A.

State at t_n: particles (x^n, u^{n-1/2}), edge field e^n and e^{n-1}, face flux b^n, the
current increment dG^n = G^n - G^{n-1}.  One step:

  (c) move particles with the Lorentz force from e^n, b^n and integrate the current along
      each path: dG^{n+1} = G^{n+1} - G^n                          (Sec. III-B, III-C)
  (a) map the source into the field update: Delta^2 G = dG^{n+1} - dG^n (Sec. III-A)
  (b,d) solve the Newmark system for e^{n+1} (Jacobi-PCG to ||r|| <= tol ||b||) and
      advance b with Faraday                                        (Sec. II-B)

Only differences of G enter the update, so the oracle keeps dG rather than G itself
(G is also accumulated for read-out).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import ab
from . import diagnostics as dg_
from . import fem, mfem, newmark
from .constants import C_LIGHT, MU0
from .mesh import Mesh
from .particles import CMesh, push


class Species:
    def __init__(self, q, m, w):
        self.q, self.m, self.w = float(q), float(m), float(w)
        self.ids = np.zeros(0, dtype=np.int64)
        self.x = np.zeros((0, 3))
        self.u = np.zeros((0, 3))
        self.tet = np.zeros(0, dtype=np.int64)
        self.alive = np.zeros(0, dtype=np.int8)


class OracleSim:
    def __init__(self, xyz, tets, cg_tol=1e-10, cg_maxit=10000, crossing_cap=64, pusher="boris", ab_order=4,
                 field_solver="wave", abc_faces=None):
        """pusher: "boris" (relativistic Boris, straight paths; u = gamma v at t_{n-1/2}) or
        "ab" (the Adams-Bashforth pusher of Sec. III-B of order ab_order with its curved
        paths; u = v at t_n).  field_solver: "wave" (the Newmark wave equation for e, b by
        Faraday), "nm_mfem" or "bd_mfem" (the mixed system, oracle/mfem.py).
        abc_faces: wall faces that absorb (first-order condition, oracle/newmark.py), as
        face ids or "all"; the others stay PEC (wave update only)."""
        assert field_solver in ("wave", "nm_mfem", "bd_mfem")
        assert abc_faces is None or field_solver == "wave"
        self.pusher, self.ab_order, self.field_solver = pusher, ab_order, field_solver
        self.mesh = m = Mesh(xyz, tets)
        self.cmesh = CMesh(m)
        self.cg_tol, self.cg_maxit, self.cap = cg_tol, cg_maxit, crossing_cap
        self.M = fem.mass_matrix(m)
        self.S = fem.curlcurl_matrix(m)
        self.D, self.C, self.D2 = m.D(), m.C(), m.D2()
        self.ie, self.inode = m.interior_edges, m.interior_nodes
        self.Kd = None
        if abc_faces is not None:
            abc = m.boundary_face.copy() if isinstance(abc_faces, str) and abc_faces == "all" else \
                np.isin(np.arange(m.n_faces), np.asarray(abc_faces))
            assert not np.any(abc & ~m.boundary_face), "absorbing faces must be wall faces"
            pec = m.boundary_face & ~abc
            fixed = np.zeros(m.n_edges, dtype=bool)
            fixed[m.face_edges[pec].ravel()] = True
            self.ie = np.nonzero(~fixed)[0]                  # the unknown edges
            self.K = fem.boundary_matrix(m, abc)
            self.Kd = newmark.restrict(self.K / (MU0 * C_LIGHT), self.ie)
        self.Mi = newmark.restrict(self.M, self.ie)
        self.Si = newmark.restrict(self.S, self.ie)
        ne, nf = m.n_edges, m.n_faces
        self.e = np.zeros(ne)
        self.e_prev = np.zeros(ne)
        self.e_prev2 = np.zeros(ne)
        self.b = np.zeros(nf)
        self.b_prev = np.zeros(nf)
        self.dG = np.zeros(ne)
        if field_solver != "wave":
            self.Mf = fem.face_mass_matrix(m)
            self.CtMf = (self.C.T @ self.Mf).tocsr()
        self.G = np.zeros(ne)
        self.species = []
        self.t = 0.0
        self.nstep = 0
        self._ops_key = None
        self._rG = []           # Gauss residual history (interior nodes)
        self.rho = np.zeros(m.n_nodes)

    # ------------------------------------------------------------------ set-up
    def add_species(self, q, m, w):
        sp_ = Species(q, m, w)
        sp_.hist = ab.Histories()
        self.species.append(sp_)
        return len(self.species) - 1

    def upload_particles(self, s, x, u, ids=None):
        sp_ = self.species[s]
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
        if ids is None:
            ids = np.arange(len(sp_.ids), len(sp_.ids) + len(x), dtype=np.int64)
        tet = self.mesh.locate(x)
        ok = (tet >= 0) & np.all(np.isfinite(u), axis=1)
        sp_.ids = np.concatenate([sp_.ids, np.asarray(ids, dtype=np.int64)[ok]])
        sp_.x = np.ascontiguousarray(np.concatenate([sp_.x, x[ok]]))
        sp_.u = np.ascontiguousarray(np.concatenate([sp_.u, u[ok]]))
        sp_.tet = np.ascontiguousarray(np.concatenate([sp_.tet, tet[ok]]))
        sp_.alive = np.ascontiguousarray(np.concatenate([sp_.alive, np.ones(int(ok.sum()), dtype=np.int8)]))
        self.rho = self.charge()
        return int((~ok).sum())

    def set_uniform_B(self, B0):
        self.b = self.mesh.face_dofs_of_uniform_field(B0)
        self.b_prev = self.b.copy()

    def charge(self):
        rho = np.zeros(self.mesh.n_nodes)
        for sp_ in self.species:
            a = sp_.alive.astype(bool)
            if a.any():
                lam = self.mesh.barycentric(sp_.tet[a], sp_.x[a])
                rho += dg_.nodal_charge(self.mesh, sp_.tet[a], lam, sp_.q * sp_.w, self.mesh.n_nodes)
        return rho

    def init_electrostatic(self, tol=1e-14):
        """Electrostatic start: -D^T M (-D phi) = rho on interior nodes (phi = 0 on the
        walls), e^0 = e^{-1} = -D phi, so Gauss holds at the first two time levels."""
        rho = self.charge()
        self.rho = rho
        ni = self.inode
        if not np.any(rho[ni]):
            return 0
        Di = self.D[:, ni]
        L = (Di.T @ self.M @ Di).tocsr()
        phi_i, it, _ = newmark.pcg_jacobi(L, rho[ni], np.zeros(len(ni)), tol, 100000)
        phi = np.zeros(self.mesh.n_nodes)
        phi[ni] = phi_i
        self.e = -(self.D @ phi)
        self.e[self.mesh.boundary_edge] = 0.0
        self.e_prev = self.e.copy()
        self.e_prev2 = self.e.copy()
        return it

    # ------------------------------------------------------------------ the step
    def operators(self, dt, beta, gamma):
        key = (dt, beta, gamma)
        if key != self._ops_key:
            self._ops = newmark.newmark_operators(self.Mi, self.Si, dt, beta, gamma, self.Kd)
            self._ops_key = key
        return self._ops

    def push_particles(self, dt):
        """Particle half of the step; returns (dG^{n+1}, push stats dict)."""
        dG_new = np.zeros(self.mesh.n_edges)
        st = {"n_crossings": 0, "max_crossings": 0, "n_absorbed": 0, "n_cap_exceeded": 0}
        for sp_ in self.species:
            if len(sp_.tet) == 0:
                continue
            if self.pusher == "ab":
                nc, na, ncap = ab.push_species(self.mesh, sp_.ids, sp_.x, sp_.u, sp_.tet, sp_.alive, sp_.q, sp_.m,
                                               sp_.w, dt, self.ab_order, self.e, self.b, dG_new, sp_.hist, self.cap)
                st["n_crossings"] += nc
                st["n_absorbed"] += na
                st["n_cap_exceeded"] += ncap
                continue
            rc, s = push(self.cmesh, sp_.x, sp_.u, sp_.tet, sp_.alive, sp_.q, sp_.m, sp_.w, dt,
                         self.e, self.b, dG_new, self.cap)
            st["n_crossings"] += s.n_crossings
            st["max_crossings"] = max(st["max_crossings"], s.max_crossings)
            st["n_absorbed"] += s.n_absorbed
            st["n_cap_exceeded"] += s.n_cap_exceeded
        return dG_new, st

    def step(self, dt, beta=0.25, gamma=0.5, x0=None, solve=True, source_override=None):
        """Advance one step.  x0: warm start on interior edges (default e^n).
        source_override(dG_new, dG_old) -> interior source vector replaces Delta^2 G (used
        by the negative test that feeds a Newmark-weighted current instead)."""
        rho_old = self.rho
        dG_new, st = self.push_particles(dt)
        ie = self.ie
        A, B1, B2 = self.operators(dt, beta, gamma)
        if source_override is None:
            src = (dG_new - self.dG)[ie]
        else:
            src = source_override(dG_new, self.dG)
        if self.field_solver == "wave":
            rhs = newmark.newmark_rhs(B1, B2, self.e[ie], self.e_prev[ie], src)
        elif self.field_solver == "nm_mfem":
            A = newmark.newmark_operators(self.Mi, self.Si, dt, 0.25, 0.5)[0]
            rhs = mfem.nm_rhs(self.M, self.S, self.CtMf, dt, self.e, self.e_prev, self.b, self.b_prev, dG_new,
                              self.dG)[ie]
        else:
            A = newmark.newmark_operators(self.Mi, self.Si, dt, 1.0, 0.5)[0]
            rhs = mfem.bd_rhs(self.M, self.CtMf, dt, self.e, self.b, dG_new)[ie]
        e_new = np.zeros_like(self.e)
        if solve:
            start = self.e[ie] if x0 is None else x0
            xi, it, res = newmark.pcg_jacobi(A, rhs, start, self.cg_tol, self.cg_maxit)
            e_new[ie] = xi
            r_cg = np.zeros_like(self.e)
            r_cg[ie] = rhs - A @ xi
        else:
            it, res = 0, 0.0
            e_new[:] = self.e
            r_cg = np.zeros_like(self.e)
        if self.field_solver == "wave":
            b_new = newmark.faraday(self.C, self.b, e_new, self.e, dt, gamma)
        elif self.field_solver == "nm_mfem":
            b_new = mfem.nm_faraday(self.C, dt, self.b_prev, e_new, self.e, self.e_prev)
        else:
            b_new = mfem.bd_faraday(self.C, dt, self.b, e_new)

        # commit
        self.e_prev2, self.e_prev, self.e = self.e_prev, self.e, e_new
        self.b_prev, self.b = self.b, b_new
        self.dG = dG_new
        self.G = self.G + dG_new
        self.t += dt
        self.nstep += 1
        self.rho = self.charge()

        # diagnostics
        ni = self.inode
        r_cont = dg_.continuity_residual(self.D, self.rho, rho_old, dG_new, ni)
        r_g = dg_.gauss_residual(self.D, self.M, self.e, self.rho, ni)
        self._rG.append(r_g)
        self._rG = self._rG[-3:]
        qw = max([abs(s.q * s.w) for s in self.species] or [1.0])
        scale = max(np.max(np.abs(self.rho[ni])) if len(ni) else 0.0, qw)
        drift = None
        if len(self._rG) == 3:
            # the Gauss residual's recurrence follows the solver's stencil: wave (1, -2, 1),
            # NM-MFEM (1, 0, -1), BD-MFEM (1, -1, 0), newest first
            c0, c1, c2 = {"wave": (1, -2, 1), "nm_mfem": (-1, 0, 1), "bd_mfem": (0, -1, 1)}[self.field_solver]
            d2 = c0 * self._rG[0] + c1 * self._rG[1] + c2 * self._rG[2]
            drift = float(np.max(np.abs(d2 - (self.D.T @ r_cg)[ni])) / scale) if len(ni) else 0.0
        st.update(cg_iters=it, cg_rel_resid=res, cont_resid_rel=float(np.max(np.abs(r_cont)) / scale) if len(ni) else 0.0,
                  gauss_resid_rel=float(np.max(np.abs(r_g)) / scale) if len(ni) else 0.0,
                  gauss_drift_check_rel=drift, divb_max=float(np.max(np.abs(self.D2 @ self.b))),
                  n_particles=int(sum(int(s.alive.sum()) for s in self.species)), rhs=rhs, r_cont=r_cont)
        return st

    # ------------------------------------------------------------------ read-out
    def particles(self, s):
        sp_ = self.species[s]
        a = sp_.alive.astype(bool)
        lam = self.mesh.barycentric(sp_.tet[a], sp_.x[a]) if a.any() else np.zeros((0, 4))
        return {"id": sp_.ids[a], "x": sp_.x[a], "u": sp_.u[a], "tet": sp_.tet[a], "lam": lam}

    def solve_direct(self, rhs, dt, beta, gamma):
        A, _, _ = self.operators(dt, beta, gamma)
        return spla.spsolve(A.tocsc(), rhs)

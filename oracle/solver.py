"""The DUGKS step on uniform and multi-level velocity spaces (FP64, plain loops).

Scheme (Sec. 2.2): with s = dt/2,
  cell:   W, q~ from g~, h~ (Eqs. W_from_tilde, discrete_W, discrete_q),
          tau = mu(T)/p, q = 2 tau q~ / (2 tau + dt Pr),
          phi_S (Eq. g_h_eq_Pr) with the compatibility correction,
          phi_bar+ = (2tau - s)/(2tau + dt) phi~ + 3s/(2tau + dt) phi_S and
          phi~+ = 4/3 phi_bar+ - 1/3 phi~  (both follow from the definitions
          phi~ = phi - dt/2 Omega, phi_bar+ = phi + s/2 Omega, phi~+ = phi + dt/2 Omega);
  slopes: per index direction a van Leer limited one-sided slope pair,
          combined into a gradient through the two direction vectors
          (reading of Eq. reconstruction for structured meshes); on
          unstructured meshes least squares with Venkatakrishnan's limiter
          (oracle.umesh);
  face:   phi_bar_f = phi_bar+_up + (x_f - x_up - xi s) . sigma_up
          (Eqs. bar_phi_transport, reconstruction; both sides averaged where
          xi . n = 0), W_f and q_bar (Eq. W_from_bar),
          q_f = 2 tau_f q_bar / (2 tau_f + s Pr),
          phi_f = 2tau_f/(2tau_f + s) phi_bar + s/(2tau_f + s) phi_S (Eq. recover_phi),
          F = A_f (xi . n) phi_f;
  update: phi~^{n+1} = phi~+ - dt/|V| sum F (Eq. explicit_update).
Multi-level (Sec. 3.4): neighbours on another level enter the slope after
projection + four-moment mapping correction to the cell's level; cross-level
faces are evaluated on V_int = min(kappa_L, kappa_R) with both sides' phi_bar+
refined and corrected to their own moments (Eq.
interface_state_moment_matching) and slopes refined by inheritance; the
interface flux (Eq. interface_reduced_fluxes) is projected to each native
level and corrected to the common target F_int (Eq.
native_flux_moment_matching).  Adaptation (criterion, clustering, level
switch with Eq. level_switch_conservation) runs at step 0 and every
`interval` steps, before the step.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import kinetic as kin
from . import levels as lv
from .mesh import Mesh
from .umesh import UMesh, lsq_limited_slope
from .quadrature import base_grid

WALL, FARFIELD, OUTFLOW = 1, 2, 3


@dataclasses.dataclass
class AdaptParams:
    C_split: float
    C_merge: float
    eps_merge: float
    tau_clust: float
    flux_test: bool
    interval: int


def van_leer(a, b):
    """vL(a, b) = (sgn a + sgn b)|a||b|/(|a| + |b|), zero when a b <= 0."""
    prod = a * b
    out = np.zeros_like(a)
    pos = prod > 0
    out[pos] = 2.0 * prod[pos] / (a[pos] + b[pos])
    return out


class Solver:
    def __init__(self, problem, compat: int = 4, face_compat: bool = True,
                 adapt: Optional[AdaptParams] = None, dt: Optional[float] = None,
                 map_moments: int = 4, positivity: str = "keep"):
        self.p = problem
        self.unstructured = bool(getattr(problem, "unstructured", False))
        self.mesh = UMesh(problem) if self.unstructured else Mesh(problem)
        self.D = problem.dim
        self.R, self.Pr, self.K = problem.R, problem.Pr, problem.K
        self.omega, self.T_ref = problem.omega, problem.T_ref
        self.mu_ref = kin.mu_ref_from_kn(problem.Kn, problem.rho_ref, problem.T_ref, problem.R,
                                         problem.L_ref, problem.omega)
        self.compat = compat
        self.face_compat = face_compat
        self.map_moments = map_moments
        # positivity check after a distribution mapping (reading R22): "keep"
        # counts violations and keeps the linear result; "exp" replaces it by
        # the exponential correction (level switches and neighbour rows)
        if positivity not in ("keep", "exp"):
            raise ValueError("positivity must be 'keep' or 'exp'")
        if positivity == "exp" and map_moments != 4:
            raise ValueError("the exponential fallback restores the four conserved moments (map_moments 4)")
        self.positivity = positivity
        self.exp_count = 0
        self.exp_fail = 0
        xi, w, nx, ny = base_grid(problem)
        self.xi_base_D = xi
        xi2 = xi if self.D == 2 else np.column_stack([xi[:, 0], np.zeros(len(xi))])
        self.base = lv.BaseGrid(xi2, w, nx, ny)
        self.dt = dt if dt is not None else problem.cfl * self.mesh.hmin / float(
            np.max(np.sqrt(np.sum(xi * xi, axis=1))))
        self.adapt_params = adapt
        if adapt is not None and self.D != 2:
            raise ValueError("multi-level velocity spaces need D = 2")
        self.levels = [lv.Level(self.base, np.zeros(self.base.Nb, np.uint8))] if self.D == 2 else [None]
        self.cell_level = np.zeros(self.mesh.n_cells, np.int64)
        self.bcs = problem.bcs
        self.step_count = 0
        self.neg_count = 0
        self.iface_cache = {}
        self.g = [None] * self.mesh.n_cells
        self.h = [None] * self.mesh.n_cells
        pj = problem
        for c in range(self.mesh.n_cells):
            if self.unstructured:
                self.init_cell(c, pj.rho0[c], np.array([pj.u0[c], pj.v0[c]]), pj.T0[c])
                continue
            i, j = c % self.mesh.ni, c // self.mesh.ni
            self.init_cell(c, pj.rho0[j, i], np.array([pj.u0[j, i], pj.v0[j, i]]), pj.T0[j, i])

    # -- velocity-set helpers -------------------------------------------------
    def vset(self, lev_id):
        """(xi with D columns, w) of a level."""
        if self.D == 1:
            return self.xi_base_D, self.base.w
        L = self.levels[lev_id]
        return L.xi, L.w

    def init_cell(self, c, rho, u, T):
        """Equilibrium start: g~ = g_eq, h~ = h_eq, compatibility-corrected (q = 0)."""
        xi, w = self.vset(self.cell_level[c])
        uD = np.asarray(u, float)[: self.D]
        self.g[c], self.h[c] = kin.model_distribution(xi, w, rho, uD, T, np.zeros(self.D), self.R,
                                                      self.Pr, self.K, self.compat)

    def mu(self, T):
        return kin.viscosity(T, self.mu_ref, self.T_ref, self.omega)

    def macro(self, xi, w, g, h):
        rho, mom, rhoE = kin.conserved(xi, w, g, h)
        rho, u, T = kin.primitive(rho, mom, rhoE, self.R, self.K)
        return rho, u, T

    # -- totals / fields --------------------------------------------------------
    def totals(self):
        """sum |V| (rho, rho u, rho v, rho E)."""
        out = np.zeros(4)
        for c in range(self.mesh.n_cells):
            xi, w = self.vset(self.cell_level[c])
            rho, mom, rhoE = kin.conserved(xi, w, self.g[c], self.h[c])
            m = np.zeros(2)
            m[: self.D] = mom
            out += self.mesh.vol[c] * np.array([rho, m[0], m[1], rhoE])
        return out

    def fields(self):
        """Per cell (rho, u, v, T, qx, qy) from the stored g~, h~ (q as in Eq. discrete_q)."""
        out = np.zeros((self.mesh.n_cells, 6))
        for c in range(self.mesh.n_cells):
            xi, w = self.vset(self.cell_level[c])
            rho, u, T = self.macro(xi, w, self.g[c], self.h[c])
            tau = self.mu(T) / (rho * self.R * T)
            qt = kin.heat_flux(xi, w, self.g[c], self.h[c], u)
            q = 2 * tau * qt / (2 * tau + self.dt * self.Pr)
            uu = np.zeros(2); uu[: self.D] = u
            qq = np.zeros(2); qq[: self.D] = q
            out[c] = [rho, uu[0], uu[1], T, qq[0], qq[1]]
        return out

    # -- multi-level helpers ----------------------------------------------------
    def iface_level(self, la, lb):
        ka, kb = self.levels[la].kappa, self.levels[lb].kappa
        key = lv.interface_kappa(ka, kb).tobytes()
        if key not in self.iface_cache:
            self.iface_cache[key] = lv.Level(self.base, lv.interface_kappa(ka, kb))
        return self.iface_cache[key]

    def map_pair(self, src, dst, g, h, T_tar, target=None, fallback=False):
        """Projection + linear mapping correction (targets = source moments by
        default); fallback: distribution maps that may take the exponential
        correction when the linear one breaks positivity."""
        gp, hp = lv.project(src, dst, g, h)
        if target is None:
            target = lv.moments4(src.xi, src.w, g, h) if self.map_moments == 4 else lv.moments9(src.xi, src.w, g, h)
        if self.map_moments == 0:
            return gp, hp
        if self.map_moments == 4:
            gs, hs = lv.mapping_correct4(dst, gp, hp, target[:4], T_tar, self.R, self.K, self.D)
        else:
            gs, hs = lv.mapping_correct9(dst, gp, hp, target)
        if np.min(gs) < 0 <= np.min(gp):
            self.neg_count += 1
        if fallback:
            gs, hs = self.positivity_fallback(dst, gp, hp, gs, hs, target)
        return gs, hs

    # positivity band (reading R22): values above -POS_EPS max|g^p| count as
    # nonnegative in the positivity check.  A tolerance of the check (a value
    # that small is no physical negative), not a rounding bound; it is pinned
    # on both sides in the tests.
    POS_EPS = 1e-10

    def positivity_fallback(self, dst, gp, hp, gs, hs, target):
        """Exponential correction in place of a linear one that made a
        nonnegative provisional g^p negative somewhere (positivity mode "exp";
        h* = h^p e^{a.phi} keeps the sign of h^p, which the projection itself
        can make negative).  A Newton iteration that does not converge keeps
        the linear result and is counted."""
        if self.positivity != "exp":
            return gs, hs
        eps = self.POS_EPS * np.max(np.abs(gp))
        if np.min(gp) < -eps or np.min(gs) >= -eps:
            return gs, hs
        ge, he, _, ok = lv.mapping_correct_exp(dst, gp, hp, target[:4])
        if not ok:
            self.exp_fail += 1
            return gs, hs
        self.exp_count += 1
        return ge, he

    # -- adaptation -------------------------------------------------------------
    def set_levels(self, kappas, cell_level):
        """Install a level catalogue and remap every cell whose level changes."""
        new_levels = [lv.Level(self.base, k) for k in kappas]
        self._switch(new_levels, np.asarray(cell_level, np.int64))

    def _switch(self, new_levels, new_cell_level):
        for c in range(self.mesh.n_cells):
            old = self.levels[self.cell_level[c]]
            new = new_levels[new_cell_level[c]]
            if old.key() == new.key():
                continue
            g, h = self.g[c], self.h[c]
            rho, u, T = self.macro(old.xi, old.w, g, h)
            gp, hp = lv.project(old, new, g, h)
            if self.map_moments == 0:
                gs, hs = gp, hp
            elif self.map_moments == 4:
                gs, hs = lv.mapping_correct4(new, gp, hp, lv.moments4(old.xi, old.w, g, h), T,
                                             self.R, self.K, self.D)
            else:
                gs, hs = lv.mapping_correct9(new, gp, hp, lv.moments9(old.xi, old.w, g, h))
            if np.min(gs) < 0 <= np.min(gp):
                # positivity check: counted; the linear result is kept unless
                # the exponential fallback is on
                self.neg_count += 1
            if self.map_moments == 4:
                gs, hs = self.positivity_fallback(new, gp, hp, gs, hs, lv.moments4(old.xi, old.w, g, h))
            self.g[c], self.h[c] = gs, hs
        self.levels = new_levels
        self.cell_level = new_cell_level
        self.iface_cache = {}

    def criterion_masks(self):
        ap = self.adapt_params
        return np.array([lv.criterion(self.levels[self.cell_level[c]], self.g[c], self.h[c],
                                      ap.C_split, ap.C_merge, ap.eps_merge, ap.flux_test)
                         for c in range(self.mesh.n_cells)], np.uint8)

    def adapt(self):
        kap = self.criterion_masks()
        kreps, cell_level = lv.cluster_masks(kap, self.adapt_params.tau_clust)
        self.set_levels(kreps, cell_level)
        return kap

    # -- the step ----------------------------------------------------------------
    def cell_stage(self):
        """Per-cell macroscopic state, collision target and phi_bar+."""
        n = self.mesh.n_cells
        dt, s = self.dt, 0.5 * self.dt
        self.cst = [None] * n
        self.fbp = [None] * n
        for c in range(n):
            xi, w = self.vset(self.cell_level[c])
            g, h = self.g[c], self.h[c]
            rho, u, T = self.macro(xi, w, g, h)
            p = rho * self.R * T
            tau = self.mu(T) / p
            qt = kin.heat_flux(xi, w, g, h, u)
            q = 2.0 * tau * qt / (2.0 * tau + dt * self.Pr)
            gS, hS = kin.model_distribution(xi, w, rho, u, T, q, self.R, self.Pr, self.K, self.compat)
            a = (2.0 * tau - s) / (2.0 * tau + dt)
            b = 3.0 * s / (2.0 * tau + dt)
            self.fbp[c] = (a * g + b * gS, a * h + b * hS)
            self.cst[c] = (rho, u, T, tau, q)

    def neighbour_on(self, c, n):
        """phi_bar+ of neighbour n expressed on cell c's level."""
        lc, ln = self.cell_level[c], self.cell_level[n]
        if lc == ln or self.D == 1:
            return self.fbp[n]
        src, dst = self.levels[ln], self.levels[lc]
        return self.map_pair(src, dst, self.fbp[n][0], self.fbp[n][1], self.cst[n][2], fallback=True)

    def slope_stage(self):
        """Limited gradient sigma of phi_bar+ per cell on its native level."""
        m = self.mesh
        self.sig = [None] * m.n_cells
        if self.unstructured:
            for c in range(m.n_cells):
                nv = [None if nb < 0 else self.neighbour_on(c, nb) for (nb, _, _) in m.cell_faces[c]]
                self.sig[c] = [lsq_limited_slope(m, c, self.fbp[c][comp],
                                                 [None if v is None else v[comp] for v in nv])
                               for comp in (0, 1)]
            return
        for c in range(m.n_cells):
            fc = self.fbp[c]
            dirs = [(0, 1)] if self.D == 1 else [(0, 1), (2, 3)]
            s_dir = []
            for (km, kp) in dirs:
                vals = []
                for k in (km, kp):
                    nb = m.nbr[c, k]
                    if nb < 0:
                        vals.append((None, 1.0))
                    else:
                        vals.append((self.neighbour_on(c, nb), float(np.hypot(*m.dnb[c, k]))))
                out = []
                for comp in (0, 1):
                    lo = np.zeros_like(fc[comp]) if vals[0][0] is None else (fc[comp] - vals[0][0][comp]) / vals[0][1]
                    hi = np.zeros_like(fc[comp]) if vals[1][0] is None else (vals[1][0][comp] - fc[comp]) / vals[1][1]
                    out.append(van_leer(lo, hi))
                s_dir.append(out)
            G = m.G[c]
            sg = []
            for comp in (0, 1):
                si = s_dir[0][comp]
                sj = s_dir[1][comp] if self.D == 2 else np.zeros_like(si)
                sg.append(np.stack([G[0, 0] * si + G[0, 1] * sj, G[1, 0] * si + G[1, 1] * sj], axis=1))
            self.sig[c] = sg

    def face_state_flux(self, xi, w, n, area, gbar, hbar):
        """Face W_f, q_f, tau_f, recovered phi_f and the microflux A (xi . n) phi_f."""
        s = 0.5 * self.dt
        nD = n[: self.D]
        rho, u, T = self.macro(xi, w, gbar, hbar)
        tau = self.mu(T) / (rho * self.R * T)
        qb = kin.heat_flux(xi, w, gbar, hbar, u)
        q = 2.0 * tau * qb / (2.0 * tau + s * self.Pr)
        gS, hS = kin.model_distribution(xi, w, rho, u, T, q, self.R, self.Pr, self.K,
                                        self.compat if self.face_compat else 0)
        gf = 2.0 * tau / (2.0 * tau + s) * gbar + s / (2.0 * tau + s) * gS
        hf = 2.0 * tau / (2.0 * tau + s) * hbar + s / (2.0 * tau + s) * hS
        dn = xi @ nD
        return area * dn * gf, area * dn * hf, T

    def extrap(self, xi, fb, sg, dvec):
        """phi_bar+ + (x_f - x_c - xi s) . sigma for g and h."""
        s = 0.5 * self.dt
        out = []
        for comp in (0, 1):
            d0 = dvec[0] - xi[:, 0] * s
            d1 = dvec[1] - (xi[:, 1] * s if self.D == 2 else 0.0)
            out.append(fb[comp] + d0 * sg[comp][:, 0] + d1 * sg[comp][:, 1])
        return out

    @staticmethod
    def upwind(dn, eL, eR):
        return np.where(dn > 0, eL, np.where(dn < 0, eR, 0.5 * (eL + eR)))

    def step(self):
        ap = self.adapt_params
        # reading R23: step 0 and every `interval` steps; interval 0 adapts
        # only when adapt() is called
        if ap is not None and ap.interval > 0 and self.step_count % ap.interval == 0:
            self.adapt()
        m = self.mesh
        dt = self.dt
        self.cell_stage()
        self.slope_stage()
        acc = [[np.zeros_like(self.g[c]), np.zeros_like(self.h[c])] for c in range(m.n_cells)]
        for f in range(m.n_faces):
            L, R = m.fL[f], m.fR[f]
            lL, lR = self.cell_level[L], self.cell_level[R]
            n = m.fn[f]
            if lL == lR or self.D == 1:
                xi, w = self.vset(lL)
                dn = xi @ n[: self.D]
                eL = self.extrap(xi, self.fbp[L], self.sig[L], m.dL[f])
                eR = self.extrap(xi, self.fbp[R], self.sig[R], m.dR[f])
                gbar = self.upwind(dn, eL[0], eR[0])
                hbar = self.upwind(dn, eL[1], eR[1])
                Fg, Fh, _ = self.face_state_flux(xi, w, n, m.fa[f], gbar, hbar)
                acc[L][0] += Fg; acc[L][1] += Fh
                acc[R][0] -= Fg; acc[R][1] -= Fh
            else:
                self.cross_face(f, acc)
        for b in range(m.n_bfaces):
            self.boundary_face(b, acc)
        for c in range(m.n_cells):
            fb = self.fbp[c]
            k = dt / m.vol[c]
            self.g[c] = (4.0 / 3.0) * fb[0] - (1.0 / 3.0) * self.g[c] - k * acc[c][0]
            self.h[c] = (4.0 / 3.0) * fb[1] - (1.0 / 3.0) * self.h[c] - k * acc[c][1]
        self.step_count += 1

    def cross_face(self, f, acc):
        m = self.mesh
        L, R = m.fL[f], m.fR[f]
        A, B = self.levels[self.cell_level[L]], self.levels[self.cell_level[R]]
        I = self.iface_level(self.cell_level[L], self.cell_level[R])
        n = m.fn[f]
        # states refined to V_int and corrected to their own native moments
        stL = self.map_pair(A, I, self.fbp[L][0], self.fbp[L][1], self.cst[L][2])
        stR = self.map_pair(B, I, self.fbp[R][0], self.fbp[R][1], self.cst[R][2])
        sgL = [np.stack([lv.project(A, I, self.sig[L][0][:, d], self.sig[L][1][:, d])[comp]
                         for d in (0, 1)], axis=1) for comp in (0, 1)]
        sgR = [np.stack([lv.project(B, I, self.sig[R][0][:, d], self.sig[R][1][:, d])[comp]
                         for d in (0, 1)], axis=1) for comp in (0, 1)]
        dn = I.xi @ n
        eL = self.extrap(I.xi, stL, sgL, m.dL[f])
        eR = self.extrap(I.xi, stR, sgR, m.dR[f])
        gbar = self.upwind(dn, eL[0], eR[0])
        hbar = self.upwind(dn, eL[1], eR[1])
        Fg, Fh, Tf = self.face_state_flux(I.xi, I.w, n, 1.0, gbar, hbar)
        tgt = lv.moments4(I.xi, I.w, Fg, Fh) if self.map_moments != 9 else lv.moments9(I.xi, I.w, Fg, Fh)
        FA = self.map_pair(I, A, Fg, Fh, Tf, tgt)
        FB = self.map_pair(I, B, Fg, Fh, Tf, tgt)
        area = m.fa[f]
        acc[L][0] += area * FA[0]; acc[L][1] += area * FA[1]
        acc[R][0] -= area * FB[0]; acc[R][1] -= area * FB[1]

    def boundary_face(self, b, acc):
        m = self.mesh
        c = m.bC[b]
        bc = self.bcs[m.bId[b]]
        xi, w = self.vset(self.cell_level[c])
        n = m.bn[b][: self.D]
        dn = xi @ n
        ext = self.extrap(xi, self.fbp[c], self.sig[c], m.bd[b])
        if bc.kind == WALL:
            uw = np.array([bc.u, bc.v])[: self.D]
            g1, h1 = kin.maxwell(xi, 1.0, uw, bc.T, self.R, self.K)
            out, inn = dn > 0, dn < 0
            rho_w = -np.sum((w * dn * ext[0])[out]) / np.sum((w * dn * g1)[inn])
            gf = np.where(dn > 0, ext[0], rho_w * g1)
            hf = np.where(dn > 0, ext[1], rho_w * h1)
        elif bc.kind == FARFIELD:
            ge, he = kin.maxwell(xi, bc.rho, np.array([bc.u, bc.v])[: self.D], bc.T, self.R, self.K)
            gf = np.where(dn > 0, ext[0], ge)
            hf = np.where(dn > 0, ext[1], he)
        elif bc.kind == OUTFLOW:
            gf = np.where(dn > 0, ext[0], self.fbp[c][0])
            hf = np.where(dn > 0, ext[1], self.fbp[c][1])
        else:
            raise ValueError("unknown boundary kind")
        area = m.ba[b]
        acc[c][0] += area * dn * gf
        acc[c][1] += area * dn * hf

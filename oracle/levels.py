"""Representative velocity levels, projection, mapping corrections, criterion, clustering.

Sec. 3.1-3.4 of the paper.  The base grid V_base is an nx x ny tensor grid,
point b = ix + nx*iy.  Its 2x2 blocks (bx, by), bx < nx//2, by < ny//2, carry
a coarsening index kappa in {0, 1, 2, 3} (fine, merged 2x2, 4x4, 8x8).
A candidate 4x4 (8x8) block exists only where all its 2x2 children exist;
rows and columns left over on odd grids stay fine (reading of the block
tiling on odd grids).
"""
from __future__ import annotations

import math

import numpy as np


class BaseGrid:
    def __init__(self, xi, w, nx, ny):
        self.xi = np.asarray(xi, float)
        self.w = np.asarray(w, float)
        self.nx, self.ny = nx, ny
        self.N = nx * ny
        self.nbx, self.nby = nx // 2, ny // 2
        self.Nb = self.nbx * self.nby

    def block_points(self, s, bx, by):
        """Base indices of the aligned 2^s x 2^s block with block coords (bx, by)."""
        size = 1 << s
        ix = np.arange(bx * size, bx * size + size)
        iy = np.arange(by * size, by * size + size)
        return (ix[None, :] + self.nx * iy[:, None]).ravel()

    def block_children2(self, s, bx, by):
        """2x2-block indices inside the 2^s block (s >= 1)."""
        size = 1 << (s - 1)
        cx = np.arange(bx * size, bx * size + size)
        cy = np.arange(by * size, by * size + size)
        return (cx[None, :] + self.nbx * cy[:, None]).ravel()


class Level:
    """A representative velocity space built from a coarsening-index array."""

    def __init__(self, base: BaseGrid, kappa):
        self.base = base
        self.kappa = np.asarray(kappa, dtype=np.uint8).copy()
        check_consistent(base, self.kappa)
        groups = []
        covered = np.zeros(base.N, bool)
        k = self.kappa
        # merged 8x8 blocks
        for oy in range(base.nby // 4):
            for ox in range(base.nbx // 4):
                ch = base.block_children2(3, ox, oy)
                if np.all(k[ch] == 3):
                    groups.append(base.block_points(3, ox, oy))
        for qy in range(base.nby // 2):
            for qx in range(base.nbx // 2):
                ch = base.block_children2(2, qx, qy)
                if np.all(k[ch] == 2):
                    groups.append(base.block_points(2, qx, qy))
        for by in range(base.nby):
            for bx in range(base.nbx):
                if k[bx + base.nbx * by] == 1:
                    groups.append(base.block_points(1, bx, by))
        for g in groups:
            covered[g] = True
        for b in np.nonzero(~covered)[0]:
            groups.append(np.array([b]))
        # canonical order: ascending first (smallest) base index of each point
        groups.sort(key=lambda a: int(a.min()))
        self.members = [np.sort(g) for g in groups]
        self.N = len(groups)
        self.pt_of_base = np.empty(base.N, np.int64)
        self.w = np.empty(self.N)
        self.xi = np.empty((self.N, base.xi.shape[1]))
        for p, g in enumerate(self.members):
            self.pt_of_base[g] = p
            wg = base.w[g]
            self.w[p] = wg.sum()
            self.xi[p] = (wg[:, None] * base.xi[g]).sum(0) / self.w[p]
            if len(g) > 1:
                # reading R34: a component of a merged point that cancels by the
                # grid's symmetry is zero, not the rounding residue of the mean,
                # so that xi . n = 0 on faces along the axes (Eq. reconstruction,
                # reading R6) is decided as in exact arithmetic
                ext = np.max(np.abs(base.xi[g]), axis=0)
                self.xi[p][np.abs(self.xi[p]) <= 1e-12 * ext] = 0.0

    def key(self):
        return self.kappa.tobytes()


def check_consistent(base: BaseGrid, kappa):
    """Parent-child consistency of a kappa array (raises on violation)."""
    k = np.asarray(kappa)
    if k.shape != (base.Nb,):
        raise ValueError("kappa has wrong length")
    for oy in range(base.nby // 4):
        for ox in range(base.nbx // 4):
            ch = k[base.block_children2(3, ox, oy)]
            if np.any(ch == 3) and not np.all(ch == 3):
                raise ValueError("inconsistent 8x8 block")
    if np.any(k > 3):
        raise ValueError("kappa out of range")
    for qy in range(base.nby // 2):
        for qx in range(base.nbx // 2):
            ch = k[base.block_children2(2, qx, qy)]
            if np.any(ch == 2) and not np.all(ch >= 2):
                raise ValueError("inconsistent 4x4 block")
    # 3s or 2s outside eligible parents are not allowed
    for by in range(base.nby):
        for bx in range(base.nbx):
            v = k[bx + base.nbx * by]
            if v == 3 and not (bx < 4 * (base.nbx // 4) and by < 4 * (base.nby // 4)):
                raise ValueError("8x8 merge outside an eligible block")
            if v == 2 and not (bx < 2 * (base.nbx // 2) and by < 2 * (base.nby // 2)):
                raise ValueError("4x4 merge outside an eligible block")


def moments4(xi, w, g, h):
    """(rho, rho u, rho v, rho E) of a reduced pair (Eq. mapping_four_targets)."""
    x2 = np.sum(xi * xi, axis=1)
    return np.array([np.sum(w * g), np.sum(w * xi[:, 0] * g), np.sum(w * xi[:, 1] * g),
                     0.5 * np.sum(w * (x2 * g + h))])


def project(src: Level, dst: Level, g, h):
    """Hierarchical projection P_{src->dst} (Sec. 3.3.2).

    Refinement: children inherit g and H = h + |xi|^2 g from their parent and
    recover h = H - |xi_child|^2 g; coarsening: w-weighted means of g and H
    (Eqs. mapping_g_projection, mapping_energy_projection,
    mapping_h_projection).  A level-to-level transfer goes through the common
    refinement; refining all the way to V_base and coarsening from there gives
    the same result, and that is what is done here.
    """
    base = src.base
    H = h + np.sum(src.xi * src.xi, axis=1) * g
    gb = g[src.pt_of_base]
    Hb = H[src.pt_of_base]
    wb = base.w
    gd = np.zeros(dst.N)
    Hd = np.zeros(dst.N)
    for p, mem in enumerate(dst.members):
        wm = wb[mem]
        gd[p] = np.sum(wm * gb[mem]) / dst.w[p]
        Hd[p] = np.sum(wm * Hb[mem]) / dst.w[p]
    hd = Hd - np.sum(dst.xi * dst.xi, axis=1) * gd
    return gd, hd


def mapping_matrix4(lev: Level):
    """State-independent 4x4 matrix of the four-moment mapping correction.

    Unit weighting chi = 1, g basis [1, xi_x, xi_y, xi_x^2 + xi_y^2]
    (Eq. raw_four_g_basis); the energy row uses psi = xi^2/2 once the coupling
    delta h = (3 - D + K) R T_tar delta g (Eq. raw_four_gh_coupling) has moved
    its T_tar-dependent part to the right-hand side.
    """
    xi, w = lev.xi, lev.w
    x2 = np.sum(xi * xi, axis=1)
    phi = np.column_stack([np.ones_like(x2), xi[:, 0], xi[:, 1], x2])
    psi = np.column_stack([np.ones_like(x2), xi[:, 0], xi[:, 1], 0.5 * x2])
    return (psi * w[:, None]).T @ phi


def mapping_correct4(lev: Level, gp, hp, target, T_tar, R, K, D=2):
    """Four-moment linear mapping correction (Sec. 3.3.2, Eqs. mapping_four_targets ..
    raw_four_gh_coupling): returns (g*, h*) with moments4 equal to target."""
    xi, w = lev.xi, lev.w
    x2 = np.sum(xi * xi, axis=1)
    cK = 3.0 - D + K
    dM = np.asarray(target, float) - moments4(xi, w, gp, hp)
    rhs = dM.copy()
    rhs[3] = dM[3] - 0.5 * cK * R * T_tar * dM[0]
    a = np.linalg.solve(mapping_matrix4(lev), rhs)
    dg = a[0] + a[1] * xi[:, 0] + a[2] * xi[:, 1] + a[3] * x2
    return gp + dg, hp + cK * R * T_tar * dg


def mapping_correct_exp(lev: Level, gp, hp, target, tol=1e-14, max_iter=30):
    """Exponential moment-constrained correction (Sec. 3.3, Eq.
    exponential_moment_correction), the sign-preserving alternative to the
    linear correction the paper proposes for when the linear one turns a
    nonnegative provisional distribution negative.

    g* = g^p exp(a . phi), h* = h^p exp(a . phi), phi = [1, xi_x, xi_y,
    |xi|^2], with a chosen so that the four mapped moments (mass, momentum,
    total energy, Eq. mapping_four_targets) equal the target.  The system
    F(a) = moments4(g^p e^{a.phi}, h^p e^{a.phi}) - target = 0 is solved by
    Newton's method from a = 0, with the Jacobian
        J_km = sum_i w_i (psi_k g^p_i + psi^h_k h^p_i) e^{a.phi_i} phi_m(xi_i),
    psi = [1, xi_x, xi_y, |xi|^2/2], psi^h = [0, 0, 0, 1/2].  The iteration
    stops when every |F_k| <= tol * S_k, S_k = sum_i w_i |psi_k g^p_i +
    psi^h_k h^p_i| e^{a.phi_i} (the size of the terms summed), or after
    max_iter steps.  Returns (g*, h*, a, converged).
    """
    xi, w = lev.xi, lev.w
    x2 = np.sum(xi * xi, axis=1)
    one = np.ones_like(x2)
    phi = np.column_stack([one, xi[:, 0], xi[:, 1], x2])
    psig = np.column_stack([one, xi[:, 0], xi[:, 1], 0.5 * x2])
    psih = np.column_stack([0.0 * one, 0.0 * one, 0.0 * one, 0.5 * one])
    tgt = np.asarray(target, float)[:4]
    a = np.zeros(4)
    converged = False
    for _ in range(max_iter + 1):
        e = np.exp(phi @ a)
        kern = (psig * (w * gp * e)[:, None] + psih * (w * hp * e)[:, None])     # (N, 4)
        F = kern.sum(axis=0) - tgt
        S = np.abs(kern).sum(axis=0)
        if np.all(np.abs(F) <= tol * S):
            converged = True
            break
        J = kern.T @ phi
        a = a - np.linalg.solve(J, F)
    e = np.exp(phi @ a)
    return gp * e, hp * e, a, converged


def moments9(xi, w, g, h):
    """(rho, rho u, rho v, rho E, Gxx, Gyy, Gxy, Jx, Jy) (Eqs. mapping_nine_targets,
    source_second_raw_moments, source_energy_flux_moments)."""
    x2 = np.sum(xi * xi, axis=1)
    E = 0.5 * (x2 * g + h)
    return np.array([np.sum(w * g), np.sum(w * xi[:, 0] * g), np.sum(w * xi[:, 1] * g),
                     np.sum(w * E), np.sum(w * xi[:, 0] ** 2 * g), np.sum(w * xi[:, 1] ** 2 * g),
                     np.sum(w * xi[:, 0] * xi[:, 1] * g), np.sum(w * xi[:, 0] * E),
                     np.sum(w * xi[:, 1] * E)])


def mapping_correct9(lev: Level, gp, hp, target):
    """Nine-moment mapping correction in two blocks (Eqs. raw_six_g_basis,
    raw_three_h_basis, mapping_h_residual_correction)."""
    xi, w = lev.xi, lev.w
    x2 = np.sum(xi * xi, axis=1)
    one = np.ones_like(x2)
    phig = np.column_stack([one, xi[:, 0], xi[:, 1], xi[:, 0] ** 2, xi[:, 1] ** 2, xi[:, 0] * xi[:, 1]])
    Ag = (phig * w[:, None]).T @ phig      # psi_g equals phi_g for these six moments
    m = moments9(xi, w, gp, hp)
    tgt = np.asarray(target, float)
    a = np.linalg.solve(Ag, (tgt - m)[[0, 1, 2, 4, 5, 6]])
    dg = phig @ a
    phih = np.column_stack([one, xi[:, 0], xi[:, 1]])
    Ah = 0.5 * (phih * w[:, None]).T @ phih
    resid = (tgt - m)[[3, 7, 8]] - 0.5 * (phih * (w * x2 * dg)[:, None]).sum(0)
    b = np.linalg.solve(Ah, resid)
    return gp + dg, hp + phih @ b


# ---------------------------------------------------------------------------
# criterion (Sec. 3.2)
# ---------------------------------------------------------------------------

def refine_to_base(lev: Level, g, h):
    """Inheritance of g and H onto V_base (refinement direction of Sec. 3.3.2)."""
    base = lev.base
    H = h + np.sum(lev.xi * lev.xi, axis=1) * g
    gb = g[lev.pt_of_base]
    hb = H[lev.pt_of_base] - np.sum(base.xi * base.xi, axis=1) * gb
    return gb, hb


def indicators(base: BaseGrid, gb, hb):
    """Per-point contributions M1 = w g / rho_tot and M2 = w (h + |xi|^2 g) / (2 E_tot)
    of a distribution on V_base (Eq. M2), signed as written."""
    w, xi = base.w, base.xi
    x2 = np.sum(xi * xi, axis=1)
    rho_tot = np.sum(w * gb)
    E_tot = np.sum(0.5 * w * (hb + x2 * gb))
    return w * gb / rho_tot, 0.5 * w * (hb + x2 * gb) / E_tot


def block_indicator(base: BaseGrid, M1, M2, s, bx, by):
    """I_B = max(sum_B M1, sum_B M2) over the 2^s block (Eq. block-contribution-indicator)."""
    pts = base.block_points(s, bx, by)
    return max(float(np.sum(M1[pts])), float(np.sum(M2[pts])))


def transport_moments(base: BaseGrid, gb, hb):
    """The four transported densities m_r = (g, xi_x g, xi_y g, (h + |xi|^2 g)/2) per point."""
    xi = base.xi
    x2 = np.sum(xi * xi, axis=1)
    return np.stack([gb, xi[:, 0] * gb, xi[:, 1] * gb, 0.5 * (hb + x2 * gb)])


def flux_scale(base: BaseGrid, gb, hb):
    """S_r = max_d sum_i w_i |xi_{i,d}| |m_r(xi_i)| over the whole space (reading of
    the normalisation in Eq. merge-transport-error)."""
    w, xi = base.w, base.xi
    m = transport_moments(base, gb, hb)
    return np.max(np.stack([np.sum(w * np.abs(xi[:, d]) * np.abs(m), axis=1) for d in (0, 1)]), axis=0)


def block_flux_error(base: BaseGrid, gb, hb, S, s, bx, by):
    """eps_B of Eq. merge-transport-error for the 2^s block: the largest normalised
    difference, over the four densities, both axes and both half-ranges, between
    the half-range fluxes sum_{i in B, sgn xi_d >= 0} w xi_d m_r of the fine points
    and that of the block's merged point (w_B = sum w, xi_B the weighted mean,
    g_B and H_B = (h + |xi|^2 g)_B weighted means, as in the coarsening of
    Sec. 3.3.2)."""
    pts = base.block_points(s, bx, by)
    xp = base.xi[pts]
    wp = base.w[pts]
    gp, hp = gb[pts], hb[pts]
    x2 = np.sum(xp * xp, axis=1)
    m = np.stack([gp, xp[:, 0] * gp, xp[:, 1] * gp, 0.5 * (hp + x2 * gp)])     # m_r on the block's points
    WB = wp.sum()
    xB = (wp[:, None] * xp).sum(0) / WB
    gB = np.sum(wp * gp) / WB
    HB = np.sum(wp * (hp + x2 * gp)) / WB
    mB = np.array([gB, xB[0] * gB, xB[1] * gB, 0.5 * HB])
    err = 0.0
    for d in (0, 1):
        for sgn in (1.0, -1.0):
            sel = sgn * xp[:, d] >= 0
            Ff = np.sum((wp * xp[:, d])[None, :] * m * sel[None, :], axis=1)
            Fm = WB * xB[d] * mB if sgn * xB[d] >= 0 else np.zeros(4)
            err = max(err, float(np.max(np.abs(Ff - Fm) / S)))
    return err


def criterion(lev: Level, g, h, C_split, C_merge, eps_merge, flux_test):
    """Per-cell coarsening index kappa on V_base's 2x2 blocks.

    Indicators M1, M2 (Eq. M2) on the stored distribution refined to V_base;
    I_B = max(sum M1, sum M2) (Eq. block-contribution-indicator); hysteresis
    (Eq. block-hysteresis-rule) against the cell's current level; optional
    transport-error test (Eqs. merge-transport-error,
    combined-merge-condition) with S_r = max_d sum_i w |xi_d| |m_r| over the
    whole space (reading); blocks examined 8x8 -> 4x4 -> 2x2.
    """
    base = lev.base
    prev = lev.kappa
    gb, hb = refine_to_base(lev, g, h)
    M1, M2 = indicators(base, gb, hb)
    S = flux_scale(base, gb, hb)
    kappa = np.zeros(base.Nb, np.uint8)

    def merges(s, bx, by):
        I = block_indicator(base, M1, M2, s, bx, by)
        prev_merged = bool(np.all(prev[base.block_children2(s, bx, by)] >= s))
        cand = I < C_merge or (C_merge <= I <= C_split and prev_merged)
        if cand and flux_test:
            cand = block_flux_error(base, gb, hb, S, s, bx, by) <= eps_merge
        return cand

    def set_k(s, bx, by, val):
        kappa[base.block_children2(s, bx, by)] = val

    def visit(s, bx, by):
        if merges(s, bx, by):
            set_k(s, bx, by, s)
            return
        if s == 1:
            return
        for cy in (2 * by, 2 * by + 1):
            for cx in (2 * bx, 2 * bx + 1):
                visit(s - 1, cx, cy)

    n8x, n8y = base.nbx // 4, base.nby // 4
    n4x, n4y = base.nbx // 2, base.nby // 2
    for oy in range(n8y):
        for ox in range(n8x):
            visit(3, ox, oy)
    for qy in range(n4y):
        for qx in range(n4x):
            if qx < 2 * n8x and qy < 2 * n8y:
                continue
            visit(2, qx, qy)
    for by in range(base.nby):
        for bx in range(base.nbx):
            if bx < 2 * n4x and by < 2 * n4y:
                continue
            visit(1, bx, by)
    return kappa


def tail_check(lev: Level, g, h, kappa_prop, C_split):
    """Tail-mass check of a proposed mask (reading of the learned selector's
    safeguard): the proposal is rejected when a block it merges carries
    I_B = max(sum M1, sum M2) > C_split (Eqs. M2, block-contribution-indicator)
    on the cell's distribution, stored on `lev` and refined to V_base.
    Returns (accepted, I_max): I_max the largest I_B over the merged blocks,
    -inf when the mask merges nothing."""
    base = lev.base
    gb, hb = refine_to_base(lev, g, h)
    M1, M2 = indicators(base, gb, hb)
    I_max = -np.inf
    for bb in range(base.Nb):
        s = int(kappa_prop[bb])
        if s == 0:
            continue
        bx, by = bb % base.nbx, bb // base.nbx
        size = 1 << (s - 1)                 # the block's side in 2x2 blocks
        if bx % size or by % size:
            continue                        # visited once, at its first 2x2 block
        I_max = max(I_max, block_indicator(base, M1, M2, s, bx // size, by // size))
    return bool(I_max <= C_split), I_max


# ---------------------------------------------------------------------------
# grouping (Sec. 3.2)
# ---------------------------------------------------------------------------

def graded_distance(ka, kb):
    """d = sum_b |ka - kb| / (3 N_b), in [0, 1]."""
    ka = np.asarray(ka, int)
    kb = np.asarray(kb, int)
    return float(np.sum(np.abs(ka - kb))) / (3.0 * len(ka))


def cluster_masks(kappas, tau):
    """Dedupe, order by frequency, leader clustering, enclosing masks.

    Unique masks are processed in descending order of frequency (ties: the
    lowest first-occurrence cell index).  A pattern joins the nearest
    existing centre (the founding pattern, never updated; ties to the lowest
    cluster id) when the graded distance is at most tau, compared in integers
    as sum|dk| <= floor(tau * 3 N_b + 1e-9); otherwise it founds a cluster.
    kappa_rep = elementwise min over members; clusters with identical
    kappa_rep are merged.  Returns (list of kappa_rep, cell -> level index).
    """
    kappas = np.asarray(kappas, np.uint8)
    n, Nb = kappas.shape
    uniq, first, inv, counts = np.unique(kappas, axis=0, return_index=True,
                                         return_inverse=True, return_counts=True)
    inv = inv.ravel()
    order = sorted(range(len(uniq)), key=lambda u: (-counts[u], first[u]))
    thr = math.floor(tau * 3 * Nb + 1e-9)
    centres = []
    members = []
    cl_of_uniq = np.empty(len(uniq), np.int64)
    for u in order:
        best, bestd = -1, None
        for cid, cu in enumerate(centres):
            d = int(np.sum(np.abs(uniq[u].astype(int) - uniq[cu].astype(int))))
            if bestd is None or d < bestd:
                best, bestd = cid, d
        if best >= 0 and bestd <= thr:
            members[best].append(u)
            cl_of_uniq[u] = best
        else:
            centres.append(u)
            members.append([u])
            cl_of_uniq[u] = len(centres) - 1
    reps = [np.min(uniq[mem], axis=0).astype(np.uint8) for mem in members]
    # merge clusters whose enclosing masks coincide
    level_of_cluster = []
    kreps = []
    for r in reps:
        for lid, k in enumerate(kreps):
            if np.array_equal(k, r):
                level_of_cluster.append(lid)
                break
        else:
            kreps.append(r)
            level_of_cluster.append(len(kreps) - 1)
    cell_level = np.array([level_of_cluster[cl_of_uniq[inv[c]]] for c in range(n)], np.int64)
    return kreps, cell_level


def interface_kappa(ka, kb):
    """V_int of a cross-level face: the common refinement min(kappa_L, kappa_R)."""
    return np.minimum(np.asarray(ka), np.asarray(kb)).astype(np.uint8)

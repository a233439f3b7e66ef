"""Structured finite-volume geometry for the DUGKS update (Sec. 2.2).

Cells (i, j), index c = i + ni * j, are quadrilaterals with nodes
(i, j), (i+1, j), (i+1, j+1), (i, j+1) in counter-clockwise order.  An
x-face sits at node column i between cells (i-1, j) and (i, j) with its
normal pointing to +i; a y-face sits at node row j between (i, j-1) and
(i, j) with its normal pointing to +j.  Periodic directions wrap, with the
period translation applied to the neighbour's centre.  In 1-D (dim = 1) only
x-faces exist.
"""
from __future__ import annotations

import numpy as np


def _poly_area_centroid(px, py):
    """Shoelace area and centroid of a simple polygon."""
    a = 0.0
    cx = 0.0
    cy = 0.0
    n = len(px)
    for k in range(n):
        x0, y0 = px[k], py[k]
        x1, y1 = px[(k + 1) % n], py[(k + 1) % n]
        cr = x0 * y1 - x1 * y0
        a += cr
        cx += (x0 + x1) * cr
        cy += (y0 + y1) * cr
    a *= 0.5
    return a, np.array([cx / (6.0 * a), cy / (6.0 * a)])


class Mesh:
    def __init__(self, problem):
        X, Y = np.asarray(problem.X, float), np.asarray(problem.Y, float)
        self.dim = problem.dim
        self.ni, self.nj = X.shape[1] - 1, X.shape[0] - 1
        ni, nj = self.ni, self.nj
        self.periodic_i, self.periodic_j = problem.periodic_i, problem.periodic_j
        self.n_cells = ni * nj
        self.vol = np.zeros(self.n_cells)
        self.xc = np.zeros((self.n_cells, 2))
        for j in range(nj):
            for i in range(ni):
                px = [X[j, i], X[j, i + 1], X[j + 1, i + 1], X[j + 1, i]]
                py = [Y[j, i], Y[j, i + 1], Y[j + 1, i + 1], Y[j + 1, i]]
                a, cen = _poly_area_centroid(px, py)
                if not a > 0:
                    raise ValueError("cell (%d, %d) is not counter-clockwise" % (i, j))
                self.vol[i + ni * j] = a
                self.xc[i + ni * j] = cen
        # period translations
        Ti = np.array([X[0, ni] - X[0, 0], Y[0, ni] - Y[0, 0]]) if self.periodic_i else None
        Tj = np.array([X[nj, 0] - X[0, 0], Y[nj, 0] - Y[0, 0]]) if self.periodic_j else None

        def node(i, j):
            return np.array([X[j, i], Y[j, i]])

        def face_geom(p0, p1, plus_i):
            t = p1 - p0
            area = float(np.hypot(t[0], t[1]))
            n = np.array([t[1], -t[0]]) / area if plus_i else np.array([-t[1], t[0]]) / area
            return n, area, 0.5 * (p0 + p1)

        # interior faces: L, R, normal L->R, area, centre, x_f - x_L, x_f - x_R
        fL, fR, fn, fa, fc, dL, dR = [], [], [], [], [], [], []
        # boundary faces: cell, bc id, outward normal, area, centre, x_f - x_c
        bC, bId, bn, ba, bc, bd = [], [], [], [], [], []
        self.face_of_cell = -np.ones((self.n_cells, 4), dtype=np.int64)   # W, E, S, N
        self.bface_of_cell = -np.ones((self.n_cells, 4), dtype=np.int64)
        # x-faces
        for j in range(nj):
            for i in range(ni + (0 if self.periodic_i else 1)):
                n, area, cen = face_geom(node(i, j), node(i, j + 1), True)
                if 0 < i < ni or self.periodic_i:
                    L = (i - 1) % ni + ni * j
                    R = i + ni * j
                    xL = self.xc[L] - (Ti if (self.periodic_i and i == 0) else 0.0)
                    fL.append(L); fR.append(R); fn.append(n); fa.append(area); fc.append(cen)
                    dL.append(cen - xL); dR.append(cen - self.xc[R])
                    self.face_of_cell[L, 1] = len(fL) - 1
                    self.face_of_cell[R, 0] = len(fL) - 1
                elif i == 0:
                    c = ni * j
                    bC.append(c); bId.append(int(problem.bc_imin[j])); bn.append(-n); ba.append(area)
                    bc.append(cen); bd.append(cen - self.xc[c])
                    self.bface_of_cell[c, 0] = len(bC) - 1
                else:
                    c = ni - 1 + ni * j
                    bC.append(c); bId.append(int(problem.bc_imax[j])); bn.append(n); ba.append(area)
                    bc.append(cen); bd.append(cen - self.xc[c])
                    self.bface_of_cell[c, 1] = len(bC) - 1
        if self.dim == 2:
            for j in range(nj + (0 if self.periodic_j else 1)):
                for i in range(ni):
                    n, area, cen = face_geom(node(i, j), node(i + 1, j), False)
                    if 0 < j < nj or self.periodic_j:
                        L = i + ni * ((j - 1) % nj)
                        R = i + ni * j
                        xL = self.xc[L] - (Tj if (self.periodic_j and j == 0) else 0.0)
                        fL.append(L); fR.append(R); fn.append(n); fa.append(area); fc.append(cen)
                        dL.append(cen - xL); dR.append(cen - self.xc[R])
                        self.face_of_cell[L, 3] = len(fL) - 1
                        self.face_of_cell[R, 2] = len(fL) - 1
                    elif j == 0:
                        c = i
                        bC.append(c); bId.append(int(problem.bc_jmin[i])); bn.append(-n)
                        ba.append(area); bc.append(cen); bd.append(cen - self.xc[c])
                        self.bface_of_cell[c, 2] = len(bC) - 1
                    else:
                        c = i + ni * (nj - 1)
                        bC.append(c); bId.append(int(problem.bc_jmax[i])); bn.append(n)
                        ba.append(area); bc.append(cen); bd.append(cen - self.xc[c])
                        self.bface_of_cell[c, 3] = len(bC) - 1
        self.fL, self.fR = np.array(fL, np.int64), np.array(fR, np.int64)
        self.fn, self.fa = np.array(fn).reshape(-1, 2), np.array(fa)
        self.fc, self.dL, self.dR = np.array(fc).reshape(-1, 2), np.array(dL).reshape(-1, 2), np.array(dR).reshape(-1, 2)
        self.bC, self.bId = np.array(bC, np.int64), np.array(bId, np.int64)
        self.bn, self.ba = np.array(bn).reshape(-1, 2), np.array(ba)
        self.bcen, self.bd = np.array(bc).reshape(-1, 2), np.array(bd).reshape(-1, 2)
        self.n_faces, self.n_bfaces = len(fL), len(bC)

        # neighbours (W, E, S, N) and centre offsets x_n - x_c (translated)
        self.nbr = -np.ones((self.n_cells, 4), dtype=np.int64)
        self.dnb = np.zeros((self.n_cells, 4, 2))
        for c in range(self.n_cells):
            for k in range(4):
                f = self.face_of_cell[c, k]
                if f < 0:
                    continue
                if self.fL[f] == c and k in (1, 3):
                    n = self.fR[f]
                    self.nbr[c, k] = n
                    self.dnb[c, k] = (self.fc[f] - self.dR[f]) - (self.fc[f] - self.dL[f])
                else:
                    n = self.fL[f]
                    self.nbr[c, k] = n
                    self.dnb[c, k] = (self.fc[f] - self.dL[f]) - (self.fc[f] - self.dR[f])
        # direction vectors between opposite face centres, and their inverse
        self.G = np.zeros((self.n_cells, 2, 2))
        self.hmin = np.inf
        for c in range(self.n_cells):
            i, j = c % ni, c // ni
            cen = {}
            for k in range(4):
                f = self.face_of_cell[c, k]
                b = self.bface_of_cell[c, k]
                if f >= 0:
                    cen[k] = self.xc[c] + (self.dL[f] if self.fL[f] == c and k in (1, 3) else self.dR[f])
                elif b >= 0:
                    cen[k] = self.bcen[b]
            ti = cen[1] - cen[0]
            ti = ti / np.hypot(*ti)
            if self.dim == 2:
                tj = cen[3] - cen[2]
                tj = tj / np.hypot(*tj)
            else:
                tj = np.array([0.0, 1.0])
            self.G[c] = np.linalg.inv(np.array([ti, tj]))
            for k in cen:
                self.hmin = min(self.hmin, 2.0 * float(np.hypot(*(cen[k] - self.xc[c]))))

"""Unstructured finite-volume geometry for the DUGKS update (Sec. 2.2) and the
limited linear reconstruction on such meshes (Eq. reconstruction).

Test infrastructure: plain FP64 code that the parity tests compare the
library against; nothing in the library imports it.

Cells are counter-clockwise triangles or quadrilaterals given by node lists.
An edge shared by two cells is an interior face: its left cell L is the cell
met first in cell order (edges in polygon order), its normal is L's outward
normal, and its centre is the edge midpoint.  An edge of one cell only is a
boundary face with that cell's outward normal and the boundary id the input
lists for it.

Slopes (reading of the reconstruction for meshes without index directions):
unweighted least squares over the face neighbours, a boundary face adding a
zero-gradient ghost at the mirror point x_c + 2 (x_f - x_c), limited with
Venkatakrishnan's function
  V(d+, d-) = (d+^2 + eps^2 + 2 d- d+) / (d+^2 + 2 d-^2 + d- d+ + eps^2),
d- = sigma . (x_f - x_c) at every face centre, d+ the largest (d- > 0) or
smallest (d- < 0) neighbour difference, including zero for the cell itself;
faces with d- = 0 impose nothing; the limiter factor is min(1, min over faces
of V).  eps^2 = (K h)^3 phi_ref^2 with K = 1, h the square root of the cell
area and phi_ref the largest |phi| among the cell and its neighbours: the
classic absolute form (K h)^3 presumes values of order one, while
distribution values span many orders of magnitude, and with it the tails of
a 1000:1 density jump reconstruct negative.
"""
from __future__ import annotations

import numpy as np

VENKAT_K = 1.0


def _poly_area_centroid(px, py):
    """Shoelace area and centroid of a simple polygon."""
    a = cx = cy = 0.0
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


class UMesh:
    kind = "unstructured"

    def __init__(self, problem):
        P = np.asarray(problem.nodes, float)
        ptr, cn = np.asarray(problem.cell_ptr), np.asarray(problem.cell_node)
        self.dim = 2
        self.n_cells = len(ptr) - 1
        n = self.n_cells
        self.vol = np.zeros(n)
        self.xc = np.zeros((n, 2))
        polys = []
        for c in range(n):
            vs = [int(v) for v in cn[ptr[c]:ptr[c + 1]]]
            if len(vs) not in (3, 4):
                raise ValueError("cell %d has %d nodes (3 or 4 supported)" % (c, len(vs)))
            a, cen = _poly_area_centroid(P[vs, 0], P[vs, 1])
            if not a > 0:
                raise ValueError("cell %d is not counter-clockwise" % c)
            self.vol[c], self.xc[c] = a, cen
            polys.append(vs)
        bid = {}
        for a, b, i in np.asarray(problem.bedges).reshape(-1, 3):
            bid[tuple(sorted((int(a), int(b))))] = int(i)
        first = {}
        fL, fR, fn, fa, fc = [], [], [], [], []
        bC, bId, bn, ba, bc = [], [], [], [], []
        # per cell and local edge: ('f', face id) or ('b', boundary face id)
        self.edges = [[None] * len(vs) for vs in polys]
        pending = {}
        for c, vs in enumerate(polys):
            for k in range(len(vs)):
                p0, p1 = P[vs[k]], P[vs[(k + 1) % len(vs)]]
                key = tuple(sorted((vs[k], vs[(k + 1) % len(vs)])))
                t = p1 - p0
                area = float(np.hypot(t[0], t[1]))
                nrm = np.array([t[1], -t[0]]) / area          # outward for a CCW polygon
                if key in pending:
                    f = pending.pop(key)
                    if fR[f] != -1:
                        raise ValueError("edge shared by more than two cells")
                    fR[f] = c
                    self.edges[c][k] = ("f", f)
                elif key in first:
                    raise ValueError("edge shared by more than two cells")
                else:
                    first[key] = c
                    pending[key] = len(fL)
                    fL.append(c); fR.append(-1); fn.append(nrm); fa.append(area); fc.append(0.5 * (p0 + p1))
                    self.edges[c][k] = ("f", len(fL) - 1)
        # edges left unpaired are boundary faces
        keep = np.array([r >= 0 for r in fR], bool)
        newid = -np.ones(len(fL), np.int64)
        newid[keep] = np.arange(int(keep.sum()))
        for key, f in pending.items():
            if key not in bid:
                raise ValueError("edge %s has one cell and no boundary id" % (key,))
            c = fL[f]
            bC.append(c); bId.append(bid[key]); bn.append(fn[f]); ba.append(fa[f]); bc.append(fc[f])
            for k, e in enumerate(self.edges[c]):
                if e == ("f", f):
                    self.edges[c][k] = ("b", len(bC) - 1)
        for c in range(n):
            for k, e in enumerate(self.edges[c]):
                if e[0] == "f":
                    self.edges[c][k] = ("f", int(newid[e[1]]))
        sel = np.nonzero(keep)[0]
        self.fL = np.array(fL, np.int64)[sel]
        self.fR = np.array(fR, np.int64)[sel]
        self.fn = np.array(fn).reshape(-1, 2)[sel]
        self.fa = np.array(fa)[sel]
        self.fc = np.array(fc).reshape(-1, 2)[sel]
        self.dL = self.fc - self.xc[self.fL]
        self.dR = self.fc - self.xc[self.fR]
        self.bC, self.bId = np.array(bC, np.int64), np.array(bId, np.int64)
        self.bn, self.ba = np.array(bn).reshape(-1, 2), np.array(ba)
        self.bcen = np.array(bc).reshape(-1, 2)
        self.bd = self.bcen - self.xc[self.bC] if len(bC) else np.zeros((0, 2))
        self.n_faces, self.n_bfaces = len(self.fL), len(self.bC)
        # per cell: (neighbour or -1, x_f - x_c, least-squares offset)
        self.cell_faces = []
        self.hmin = np.inf
        for c in range(n):
            lst = []
            for (kind, f) in self.edges[c]:
                if kind == "f":
                    nb = int(self.fR[f] if self.fL[f] == c else self.fL[f])
                    fo = self.fc[f] - self.xc[c]
                    lst.append((nb, fo, self.xc[nb] - self.xc[c]))
                else:
                    fo = self.bcen[f] - self.xc[c]
                    lst.append((-1, fo, 2.0 * fo))
                self.hmin = min(self.hmin, 2.0 * float(np.hypot(*fo)))
            self.cell_faces.append(lst)


def venkat(dp, dm, eps2):
    """Venkatakrishnan's function V(d+, d-) with V = 1 where d- = 0."""
    dp, dm = np.broadcast_arrays(np.asarray(dp, float), np.asarray(dm, float))
    num = dp * dp + eps2 + 2.0 * dm * dp
    den = dp * dp + 2.0 * dm * dm + dm * dp + eps2
    out = np.ones_like(dm)
    nz = dm != 0.0
    out[nz] = num[nz] / den[nz]
    return out


def lsq_gradient(mesh, c, fc, nvals):
    """Unlimited least-squares gradient of one quantity of cell c: fc (N,),
    nvals per local face the neighbour values (N,) or None (boundary face,
    zero-gradient ghost at the mirror point).  Returns (N, 2)."""
    A = np.zeros((2, 2))
    rhs = np.zeros((len(fc), 2))
    for (nb, fo, d), v in zip(mesh.cell_faces[c], nvals):
        A += np.outer(d, d)
        if v is not None:
            rhs += np.outer(v - fc, d)
    return rhs @ np.linalg.inv(A).T


def lsq_limited_slope(mesh, c, fc, nvals, eps2=None):
    """Limited gradient of one quantity of cell c at every velocity point.

    fc: (N,) cell values; nvals: per local face of c the neighbour values
    (N,) on c's velocity set, or None for a boundary face (zero-gradient
    ghost).  eps2: override of eps^2 (scalar or (N,)).  Returns sigma (N, 2)."""
    faces = mesh.cell_faces[c]
    A = np.zeros((2, 2))
    rhs = np.zeros((len(fc), 2))
    for (nb, fo, d), v in zip(faces, nvals):
        A += np.outer(d, d)
        if v is not None:
            rhs += np.outer(v - fc, d)
    sig = rhs @ np.linalg.inv(A).T
    if eps2 is None:
        ref = np.abs(fc)
        for v in nvals:
            if v is not None:
                ref = np.maximum(ref, np.abs(v))
        eps2 = (VENKAT_K * np.sqrt(mesh.vol[c])) ** 3 * ref * ref
    dmax = np.zeros(len(fc))
    dmin = np.zeros(len(fc))
    for v in nvals:
        if v is not None:
            dmax = np.maximum(dmax, v - fc)
            dmin = np.minimum(dmin, v - fc)
    psi = np.ones(len(fc))
    for (nb, fo, d) in faces:
        dm = sig @ fo
        dp = np.where(dm > 0, dmax, dmin)
        psi = np.minimum(psi, venkat(dp, dm, eps2))
    return sig * psi[:, None]

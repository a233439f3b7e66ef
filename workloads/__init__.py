"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds problem set-up only: mesh node coordinates, boundary
specifications, initial macroscopic fields, velocity-grid extents and seeded
random perturbations.  It contains none of the scheme's arithmetic (no
quadrature weights, equilibria, moments or corrections); each side computes
those from these inputs with its own code.

Boundary kinds (integers shared by both sides):
  WALL     isothermal diffuse wall at (T, u, v)
  FARFIELD incoming Maxwellian at (rho, u, v, T); also used for inflow slots
  OUTFLOW  zero-gradient extrapolation
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

WALL, FARFIELD, OUTFLOW = 1, 2, 3


@dataclasses.dataclass
class BC:
    kind: int
    rho: float = 1.0
    u: float = 0.0
    v: float = 0.0
    T: float = 1.0


@dataclasses.dataclass
class Problem:
    """A structured-mesh problem: nodes, boundaries, initial state, physics."""

    name: str
    dim: int
    X: np.ndarray            # node x, shape (nj+1, ni+1)
    Y: np.ndarray            # node y, shape (nj+1, ni+1)
    periodic_i: bool
    periodic_j: bool
    bcs: List[BC]            # boundary table; ids below index into it
    bc_imin: np.ndarray      # (nj,) bc id of the face at i = 0
    bc_imax: np.ndarray      # (nj,) bc id of the face at i = ni
    bc_jmin: np.ndarray      # (ni,) bc id of the face at j = 0
    bc_jmax: np.ndarray      # (ni,) bc id of the face at j = nj
    rho0: np.ndarray         # (nj, ni) initial density
    u0: np.ndarray           # (nj, ni)
    v0: np.ndarray           # (nj, ni)
    T0: np.ndarray           # (nj, ni)
    R: float
    Pr: float
    K: int
    omega: float
    T_ref: float
    rho_ref: float
    L_ref: float
    Kn: float
    cfl: float
    vel_kind: str            # 'nc' (Newton-Cotes) or 'gh' (Gauss-Hermite)
    nv: int                  # velocity points per axis
    vmax: float              # half-width of a Newton-Cotes grid
    gh_scale_T: float = 1.0  # temperature whose sqrt(2RT) scales a GH grid

    @property
    def ni(self) -> int:
        return self.X.shape[1] - 1

    @property
    def nj(self) -> int:
        return self.X.shape[0] - 1

    @property
    def n_cells(self) -> int:
        return self.ni * self.nj


def _nodes_rect(x0, x1, y0, y1, ni, nj):
    xs = np.linspace(x0, x1, ni + 1)
    ys = np.linspace(y0, y1, nj + 1)
    X, Y = np.meshgrid(xs, ys)
    return X.copy(), Y.copy()


def sod_1d(n_cells: int = 200, Kn: float = 1e-3, nv: int = 101, vmax: float = 10.0) -> Problem:
    """1-D Sod tube on [0, 1]: left (1, 0, 1), right (0.125, 0, 0.8), R = 1, BGK."""
    X, Y = _nodes_rect(0.0, 1.0, 0.0, 1.0, n_cells, 1)
    xc = 0.5 * (X[0, :-1] + X[0, 1:])
    left = xc < 0.5
    rho = np.where(left, 1.0, 0.125)[None, :]
    T = np.where(left, 1.0, 0.8)[None, :]
    z = np.zeros_like(rho)
    ids1 = np.zeros(1, np.int32)
    return Problem("sod1d", 1, X, Y, False, False, [BC(OUTFLOW)], ids1, ids1.copy(),
                   np.zeros(n_cells, np.int32), np.zeros(n_cells, np.int32),
                   rho, z, z.copy(), T, R=1.0, Pr=1.0, K=0, omega=0.81, T_ref=1.0,
                   rho_ref=1.0, L_ref=1.0, Kn=Kn, cfl=0.5, vel_kind="nc", nv=nv, vmax=vmax)


def cavity(n: int = 64, Kn: float = 0.075, nv: int = 28, vel_kind: str = "gh",
           vmax: float = 4.0, lid_mach: float = 0.16) -> Problem:
    """Lid-driven cavity on [0,1]^2, R = 0.5, T0 = Tw = 1, Shakhov Pr = 2/3."""
    R = 0.5
    X, Y = _nodes_rect(0.0, 1.0, 0.0, 1.0, n, n)
    uw = lid_mach * math.sqrt(5.0 / 3.0 * R * 1.0)
    bcs = [BC(WALL, T=1.0), BC(WALL, u=uw, T=1.0)]
    ones = np.ones((n, n))
    zi = np.zeros(n, np.int32)
    return Problem("cavity", 2, X, Y, False, False, bcs, zi, zi.copy(), zi.copy(),
                   np.ones(n, np.int32), ones.copy(), 0 * ones, 0 * ones, ones.copy(),
                   R=R, Pr=2.0 / 3.0, K=0, omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0,
                   Kn=Kn, cfl=0.5, vel_kind=vel_kind, nv=nv, vmax=vmax, gh_scale_T=1.0)


def cylinder(ntheta: int = 256, nr: int = 128, Kn: float = 0.1, mach: float = 3.0,
             nv: int = 101, vmax: float = 10.0, r_out: float = 11.0, dr1: float = 0.02) -> Problem:
    """O-grid around a unit cylinder, geometric radial spacing, R = 0.5, T_inf = 1.

    Node (i, j) sits at angle -2*pi*i/ntheta and radius r_j so that cells are
    counter-clockwise; i is periodic, j = 0 is the wall, j = nr the far field.
    """
    R = 0.5
    # geometric ratio q with dr1 * (q^nr - 1)/(q - 1) = r_out - 1
    total = r_out - 1.0
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = dr1 * (mid ** nr - 1.0) / (mid - 1.0)
        lo, hi = (mid, hi) if s < total else (lo, mid)
    q = 0.5 * (lo + hi)
    r = 1.0 + dr1 * (q ** np.arange(nr + 1) - 1.0) / (q - 1.0)
    r[-1] = r_out
    th = -2.0 * math.pi * np.arange(ntheta + 1) / ntheta
    X = r[:, None] * np.cos(th)[None, :]
    Y = r[:, None] * np.sin(th)[None, :]
    X[:, -1] = X[:, 0]
    Y[:, -1] = Y[:, 0]
    U = mach * math.sqrt(5.0 / 3.0 * R * 1.0)
    bcs = [BC(WALL, T=1.0), BC(FARFIELD, rho=1.0, u=U, v=0.0, T=1.0)]
    shape = (nr, ntheta)
    z = np.zeros(ntheta, np.int32)
    return Problem("cylinder", 2, X, Y, True, False, bcs, np.zeros(nr, np.int32),
                   np.zeros(nr, np.int32), z, np.ones(ntheta, np.int32),
                   np.ones(shape), np.full(shape, U), np.zeros(shape), np.ones(shape),
                   R=R, Pr=2.0 / 3.0, K=0, omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0,
                   Kn=Kn, cfl=0.5, vel_kind="nc", nv=nv, vmax=vmax)


def jet(ni: int = 512, nj: int = 256, Kn_jet: float = 1e-3, nv: int = 161, vmax: float = 7.0,
        rho_b: float = 0.01) -> Problem:
    """Slot jet into near vacuum on [0,32]x[-8,8]; sonic inflow at |y| <= 0.5, x = 0."""
    R = 0.5
    X, Y = _nodes_rect(0.0, 32.0, -8.0, 8.0, ni, nj)
    uj = math.sqrt(5.0 / 3.0 * R * 1.0)
    bcs = [BC(WALL, T=1.0), BC(FARFIELD, rho=1.0, u=uj, T=1.0),
           BC(FARFIELD, rho=rho_b, T=1.0)]
    yc = 0.5 * (Y[:-1, 0] + Y[1:, 0])
    imin = np.where(np.abs(yc) <= 0.5, 1, 0).astype(np.int32)
    shape = (nj, ni)
    return Problem("jet", 2, X, Y, False, False, bcs, imin, np.full(nj, 2, np.int32),
                   np.full(ni, 2, np.int32), np.full(ni, 2, np.int32),
                   np.full(shape, rho_b), np.zeros(shape), np.zeros(shape), np.ones(shape),
                   R=R, Pr=2.0 / 3.0, K=0, omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0,
                   Kn=Kn_jet, cfl=0.5, vel_kind="nc", nv=nv, vmax=vmax)


def periodic_box(ni: int, nj: int, Lx: float = 1.0, Ly: float = 0.1, Kn: float = 0.1,
                 nv: int = 17, vmax: float = 4.0, kind: str = "uniform", amp: float = 0.2,
                 Pr: float = 2.0 / 3.0) -> Problem:
    """Periodic box: uniform flow (u = 0.1) or a sine density wave (U0 = 0.1, p0 = 0.5)."""
    R = 0.5
    X, Y = _nodes_rect(0.0, Lx, 0.0, Ly, ni, nj)
    xc = 0.5 * (X[:-1, :-1] + X[:-1, 1:])
    shape = (nj, ni)
    if kind == "uniform":
        rho = np.ones(shape)
        T = np.ones(shape)
    else:
        rho = 1.0 + amp * np.sin(2 * math.pi * xc / Lx)
        T = 0.5 / (rho * R)
    z = np.zeros(ni, np.int32)
    return Problem(kind, 2, X, Y, True, True, [BC(OUTFLOW)], np.zeros(nj, np.int32),
                   np.zeros(nj, np.int32), z, z.copy(), rho, np.full(shape, 0.1),
                   np.zeros(shape), T, R=R, Pr=Pr, K=0, omega=0.81, T_ref=1.0, rho_ref=1.0,
                   L_ref=1.0, Kn=Kn, cfl=0.5, vel_kind="nc", nv=nv, vmax=vmax)


def perturb(problem: Problem, seed: int, amp: float = 0.05) -> Problem:
    """Return a copy with seeded smooth-ish random perturbations of rho, u, v, T."""
    rng = np.random.default_rng(seed)
    p = dataclasses.replace(problem)
    shape = problem.rho0.shape
    p.rho0 = problem.rho0 * (1.0 + amp * rng.uniform(-1, 1, shape))
    p.u0 = problem.u0 + amp * rng.uniform(-1, 1, shape)
    p.v0 = problem.v0 + (amp * rng.uniform(-1, 1, shape) if problem.dim == 2 else 0.0)
    p.T0 = problem.T0 * (1.0 + amp * rng.uniform(-1, 1, shape))
    return p


def random_positive_rows(seed: int, n_rows: int, n_cols: int, lo: float = 0.2,
                         hi: float = 1.0) -> np.ndarray:
    """Seeded random positive values, shape (n_rows, n_cols)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n_rows, n_cols))


def random_states(seed: int, n: int, dim: int = 2):
    """Seeded random macroscopic states (rho, u, v, T, qx, qy) for micro tests."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    u = rng.uniform(-0.5, 0.5, n)
    v = rng.uniform(-0.5, 0.5, n) if dim == 2 else np.zeros(n)
    T = rng.uniform(0.6, 1.6, n)
    qx = rng.uniform(-0.05, 0.05, n)
    qy = rng.uniform(-0.05, 0.05, n) if dim == 2 else np.zeros(n)
    return rho, u, v, T, qx, qy


def random_kappa(nbx: int, nby: int, seed: int, p8: float = 0.25, p4: float = 0.33,
                 p2: float = 0.5) -> np.ndarray:
    """A seeded random coarsening-index array on nbx x nby 2x2 blocks that is
    parent-child consistent (whole 8x8 / 4x4 merges only where those blocks fit)."""
    rng = np.random.default_rng(seed)
    k = np.zeros((nby, nbx), np.uint8)
    for by in range(nby):
        for bx in range(nbx):
            k[by, bx] = 1 if rng.random() < p2 else 0
    for qy in range(nby // 2):
        for qx in range(nbx // 2):
            if rng.random() < p4:
                k[2 * qy:2 * qy + 2, 2 * qx:2 * qx + 2] = 2
    for oy in range(nby // 4):
        for ox in range(nbx // 4):
            if rng.random() < p8:
                k[4 * oy:4 * oy + 4, 4 * ox:4 * ox + 4] = 3
    return k.ravel()


def patch(problem: Problem, i0: int, j0: int, ni: int = 5, nj: int = 5) -> Problem:
    """The ni x nj cells of a structured problem starting at cell (i0, j0), as a
    problem of its own: the same nodes and physics, outflow on every side, not
    periodic (initial state: the original one on those cells)."""
    sl = (slice(j0, j0 + nj), slice(i0, i0 + ni))
    p = dataclasses.replace(problem)
    p.X = problem.X[j0:j0 + nj + 1, i0:i0 + ni + 1].copy()
    p.Y = problem.Y[j0:j0 + nj + 1, i0:i0 + ni + 1].copy()
    p.periodic_i = p.periodic_j = False
    p.bcs = [BC(OUTFLOW)]
    p.bc_imin = np.zeros(nj, np.int32)
    p.bc_imax = np.zeros(nj, np.int32)
    p.bc_jmin = np.zeros(ni, np.int32)
    p.bc_jmax = np.zeros(ni, np.int32)
    p.rho0, p.u0, p.v0, p.T0 = (problem.rho0[sl].copy(), problem.u0[sl].copy(), problem.v0[sl].copy(),
                                problem.T0[sl].copy())
    return p


def striped_levels(ni: int, nj: int, n_levels: int, axis: int = 0) -> np.ndarray:
    """Cell -> level index in stripes along one mesh axis (cell c = i + ni*j)."""
    i = np.arange(ni)[None, :].repeat(nj, 0)
    j = np.arange(nj)[:, None].repeat(ni, 1)
    idx = i if axis == 0 else j
    n = ni if axis == 0 else nj
    return (idx * n_levels // n).ravel().astype(np.int32)


def block_levels(ni: int, nj: int, n_levels: int, seed: int, block: int = 8) -> np.ndarray:
    """Cell -> level index, seeded uniformly per block x block tile of cells
    (cell c = i + ni*j), so that cross-level faces run along the tile edges."""
    rng = np.random.default_rng(seed)
    tiles = rng.integers(0, n_levels, size=((nj + block - 1) // block, (ni + block - 1) // block))
    i = np.arange(ni)[None, :].repeat(nj, 0)
    j = np.arange(nj)[:, None].repeat(ni, 1)
    return tiles[j // block, i // block].ravel().astype(np.int32)


def point_levels(xc: np.ndarray, n_levels: int, seed: int, h: float) -> np.ndarray:
    """Cell -> level index for cells at centroids xc [n][2], seeded uniformly
    per square of side h of the plane (the unstructured counterpart of
    block_levels)."""
    ij = np.floor(np.asarray(xc) / h).astype(np.int64)
    ij -= ij.min(axis=0)
    rng = np.random.default_rng(seed)
    tab = rng.integers(0, n_levels, size=tuple(ij.max(axis=0) + 1))
    return tab[ij[:, 0], ij[:, 1]].astype(np.int32)


def mlp_init_params(K: int, seed: int, H: int = 64, NF: int = 10) -> np.ndarray:
    """Seeded He-normal initial weights of the 10 -> H -> H -> K selector, zero
    biases, identity normalisation (mean 0, std 1); flat layout
    W1 [H][NF], b1, W2 [H][H], b2, W3 [K][H], b3, mean [NF], std [NF]."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(H, NF)) * math.sqrt(2.0 / NF)
    W2 = rng.normal(size=(H, H)) * math.sqrt(2.0 / H)
    W3 = rng.normal(size=(K, H)) * math.sqrt(2.0 / H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(K),
                           np.zeros(NF), np.ones(NF)])


# ---------------------------------------------------------------------------
# unstructured meshes
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class UProblem:
    """An unstructured-mesh problem: polygons (triangles or quadrilaterals,
    counter-clockwise), the boundary id of every edge that belongs to one cell
    only, initial state per cell, physics as in Problem."""

    name: str
    nodes: np.ndarray        # (n_nodes, 2)
    cell_ptr: np.ndarray     # (n_cells + 1,) int32 offsets into cell_node
    cell_node: np.ndarray    # int32 node ids, 3 or 4 per cell
    bedges: np.ndarray       # (n_bedges, 3) int32: node a, node b, bc id
    bcs: List[BC]
    rho0: np.ndarray         # (n_cells,)
    u0: np.ndarray
    v0: np.ndarray
    T0: np.ndarray
    R: float
    Pr: float
    K: int
    omega: float
    T_ref: float
    rho_ref: float
    L_ref: float
    Kn: float
    cfl: float
    vel_kind: str
    nv: int
    vmax: float
    gh_scale_T: float = 1.0
    dim: int = 2
    unstructured: bool = True

    @property
    def n_cells(self) -> int:
        return len(self.cell_ptr) - 1

    def centroids(self) -> np.ndarray:
        """Vertex means of the cells (set-up only: seeding and region tests)."""
        out = np.zeros((self.n_cells, 2))
        for c in range(self.n_cells):
            out[c] = self.nodes[self.cell_node[self.cell_ptr[c]:self.cell_ptr[c + 1]]].mean(axis=0)
        return out


def two_cavity(n: int = 48, nv: int = 101, vmax: float = 7.0, Kn_left: float = 1e-3,
               ratio: float = 1e-3, seed: int = 0, jitter: float = 0.15) -> UProblem:
    """Gas expansion between two square cavities (side 1) joined by a channel of
    length 1 and width 1/8: left cavity [-1.5,-0.5]x[-0.5,0.5], channel
    [-0.5,0.5]x[-1/16,1/16], right cavity [0.5,1.5]x[-0.5,0.5].  Lattice
    spacing 1/n (n a multiple of 16); cavity squares are cut into two
    triangles along a seeded random diagonal, channel squares stay
    quadrilaterals, and every node off the boundary is moved by a seeded
    uniform offset of at most jitter/n per axis.  Diffuse walls at T = 1;
    gas at rest, T = 1, rho = 1 for x < 0 and `ratio` for x > 0 (R = 0.5, so
    sqrt(2 R T_w) = 1)."""
    if n % 16 != 0:
        raise ValueError("n must be a multiple of 16")
    h = 1.0 / n
    ni, nj = 3 * n, n
    half = n // 16
    def inside(i, j):            # lattice square (i, j) by its lower-left corner
        if i < 0 or j < 0 or i >= ni or j >= nj:
            return 0
        if i < n or i >= 2 * n:
            return 1             # cavity
        return 2 if (n // 2 - half) <= j < (n // 2 + half) else 0
    rng = np.random.default_rng(seed)
    node_id = -np.ones((nj + 1, ni + 1), np.int64)
    sq = [(i, j, inside(i, j)) for j in range(nj) for i in range(ni) if inside(i, j)]
    for (i, j, _) in sq:
        for (a, b) in ((i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)):
            node_id[b, a] = 0
    pts = []
    for b in range(nj + 1):
        for a in range(ni + 1):
            if node_id[b, a] == 0:
                node_id[b, a] = len(pts)
                pts.append((-1.5 + a * h, -0.5 + b * h))
    nodes = np.array(pts)
    # boundary edges: lattice edges with a domain square on one side only
    bedges = []
    on_bnd = np.zeros(len(nodes), bool)
    for (i, j, _) in sq:
        for (di, dj, a0, a1) in ((0, -1, (i, j), (i + 1, j)), (1, 0, (i + 1, j), (i + 1, j + 1)),
                                 (0, 1, (i + 1, j + 1), (i, j + 1)), (-1, 0, (i, j + 1), (i, j))):
            if not inside(i + di, j + dj):
                p, q = node_id[a0[1], a0[0]], node_id[a1[1], a1[0]]
                bedges.append((p, q, 0))
                on_bnd[p] = on_bnd[q] = True
    off = rng.uniform(-jitter * h, jitter * h, size=nodes.shape)
    off[on_bnd] = 0.0
    nodes = nodes + off
    cells = []
    for (i, j, kind) in sq:
        a, b = node_id[j, i], node_id[j, i + 1]
        c, d = node_id[j + 1, i + 1], node_id[j + 1, i]
        if kind == 2:
            cells.append((a, b, c, d))
        elif rng.random() < 0.5:
            cells.append((a, b, c)); cells.append((a, c, d))
        else:
            cells.append((a, b, d)); cells.append((b, c, d))
    cell_ptr = np.zeros(len(cells) + 1, np.int32)
    cell_ptr[1:] = np.cumsum([len(c) for c in cells])
    cell_node = np.array([v for c in cells for v in c], np.int32)
    xc = np.array([nodes[list(c)].mean(axis=0) for c in cells])
    left = xc[:, 0] < 0.0
    nc = len(cells)
    R = 0.5
    return UProblem("two_cavity", nodes, cell_ptr, cell_node, np.array(bedges, np.int32).reshape(-1, 3),
                    [BC(WALL, T=1.0)], np.where(left, 1.0, ratio), np.zeros(nc), np.zeros(nc), np.ones(nc),
                    R=R, Pr=2.0 / 3.0, K=0, omega=0.81, T_ref=1.0, rho_ref=1.0, L_ref=1.0, Kn=Kn_left,
                    cfl=0.5, vel_kind="nc", nv=nv, vmax=vmax)


def as_unstructured(problem: Problem, split: str = "none", seed: int = 0) -> UProblem:
    """A structured problem as an unstructured one: the same nodes, each
    quadrilateral kept ("none"), cut along its (i,j)-(i+1,j+1) diagonal
    ("diag") or along a seeded random diagonal ("random").  Cell order: (i, j)
    row-major, the two triangles of a cut cell in a row.  A direction periodic
    in i whose seam nodes coincide (an O-grid) is closed by sharing those
    nodes; other periodic meshes are not supported."""
    if problem.periodic_j or problem.dim != 2:
        raise ValueError("needs a 2-D problem not periodic in j")
    ni, nj = problem.ni, problem.nj
    if problem.periodic_i and not (np.allclose(problem.X[:, 0], problem.X[:, ni])
                                   and np.allclose(problem.Y[:, 0], problem.Y[:, ni])):
        raise ValueError("periodic in i without coinciding seam nodes")
    nodes = np.stack([problem.X.ravel(), problem.Y.ravel()], axis=1)
    wrap = problem.periodic_i
    nid = lambda i, j: j * (ni + 1) + (0 if (wrap and i == ni) else i)
    rng = np.random.default_rng(seed)
    cells, src = [], []
    for j in range(nj):
        for i in range(ni):
            a, b, c, d = nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)
            if split == "none":
                cells.append((a, b, c, d)); src.append(i + ni * j)
            elif split == "diag" or rng.random() < 0.5:
                cells += [(a, b, c), (a, c, d)]; src += [i + ni * j] * 2
            else:
                cells += [(a, b, d), (b, c, d)]; src += [i + ni * j] * 2
    bedges = []
    for j in range(nj if not wrap else 0):
        bedges.append((nid(0, j + 1), nid(0, j), int(problem.bc_imin[j])))
        bedges.append((nid(ni, j), nid(ni, j + 1), int(problem.bc_imax[j])))
    for i in range(ni):
        bedges.append((nid(i, 0), nid(i + 1, 0), int(problem.bc_jmin[i])))
        bedges.append((nid(i + 1, nj), nid(i, nj), int(problem.bc_jmax[i])))
    cell_ptr = np.zeros(len(cells) + 1, np.int32)
    cell_ptr[1:] = np.cumsum([len(c) for c in cells])
    src = np.array(src)
    f = lambda a: np.asarray(a).ravel()[src].copy()
    return UProblem(problem.name + "_u", nodes, cell_ptr, np.array([v for c in cells for v in c], np.int32),
                    np.array(bedges, np.int32), list(problem.bcs), f(problem.rho0), f(problem.u0),
                    f(problem.v0), f(problem.T0), R=problem.R, Pr=problem.Pr, K=problem.K,
                    omega=problem.omega, T_ref=problem.T_ref, rho_ref=problem.rho_ref, L_ref=problem.L_ref,
                    Kn=problem.Kn, cfl=problem.cfl, vel_kind=problem.vel_kind, nv=problem.nv,
                    vmax=problem.vmax, gh_scale_T=problem.gh_scale_T)


def cell_neighbours(p: UProblem):
    """Cells sharing an edge with each cell (set-up only: patch extraction)."""
    owner = {}
    for c in range(p.n_cells):
        vs = p.cell_node[p.cell_ptr[c]:p.cell_ptr[c + 1]]
        for k in range(len(vs)):
            key = tuple(sorted((int(vs[k]), int(vs[(k + 1) % len(vs)]))))
            owner.setdefault(key, []).append(c)
    nb = [[] for _ in range(p.n_cells)]
    for cs in owner.values():
        if len(cs) == 2:
            nb[cs[0]].append(cs[1]); nb[cs[1]].append(cs[0])
    return nb


def upatch(p: UProblem, centre: int, hops: int = 2):
    """The cells within `hops` edge-neighbour steps of `centre`, as a problem of
    its own (edges to cells left out become outflow boundaries; the original
    boundary edges keep their ids).  Returns (problem, cells), cells[k] being
    the original id of the patch's cell k (centre first)."""
    nb = cell_neighbours(p)
    cells, seen, front = [centre], {centre}, [centre]
    for _ in range(hops):
        nxt = []
        for c in front:
            for n in nb[c]:
                if n not in seen:
                    seen.add(n); cells.append(n); nxt.append(n)
        front = nxt
    used = sorted({int(v) for c in cells for v in p.cell_node[p.cell_ptr[c]:p.cell_ptr[c + 1]]})
    remap = {v: k for k, v in enumerate(used)}
    polys = [[remap[int(v)] for v in p.cell_node[p.cell_ptr[c]:p.cell_ptr[c + 1]]] for c in cells]
    orig_b = {tuple(sorted((int(a), int(b)))): int(i) for a, b, i in p.bedges}
    count = {}
    for poly in polys:
        for k in range(len(poly)):
            key = tuple(sorted((poly[k], poly[(k + 1) % len(poly)])))
            count[key] = count.get(key, 0) + 1
    bcs = list(p.bcs) + [BC(OUTFLOW)]
    inv = {k: v for v, k in remap.items()}
    bedges = []
    for poly in polys:
        for k in range(len(poly)):
            a, b = poly[k], poly[(k + 1) % len(poly)]
            if count[tuple(sorted((a, b)))] == 1:
                bid = orig_b.get(tuple(sorted((inv[a], inv[b]))), len(bcs) - 1)
                bedges.append((a, b, bid))
    cell_ptr = np.zeros(len(polys) + 1, np.int32)
    cell_ptr[1:] = np.cumsum([len(q) for q in polys])
    idx = np.array(cells)
    q = dataclasses.replace(p, name=p.name + "_patch", nodes=p.nodes[used].copy(), cell_ptr=cell_ptr,
                            cell_node=np.array([v for poly in polys for v in poly], np.int32),
                            bedges=np.array(bedges, np.int32).reshape(-1, 3), bcs=bcs,
                            rho0=p.rho0[idx].copy(), u0=p.u0[idx].copy(), v0=p.v0[idx].copy(),
                            T0=p.T0[idx].copy())
    return q, idx

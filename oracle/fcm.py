"""Finite cell discretisation, assembly and d/c partition (oracle; FP64).

Follows Section "Spatial Discretization" (indicator alpha, Eqs. Mglobal, K
and f; space-tree quadrature on cut cells; GLL quadrature of the mass on
uncut cells; Gauss-Legendre quadrature of the stiffness on every cell) and
Section "Partitioning of the Degrees of Freedom" (Eqs. MStructure,
KStructure, Kd, Kc, f_xStructure).

Readings where the paper is silent (each also listed in the design notes):
  * a cell is *crossed* by a ball j when d_min < r_j < d_max, with d_min /
    d_max the smallest / largest distance from the centre to the cell box;
    a cell is *empty* when some ball contains it (d_max <= r_j) or when it
    is crossed and its fill ratio is below 1e-10 (Section "Perforated
    plate"); it is *cut* when crossed and not empty, *uncut* otherwise;
  * the space tree bisects a box in every direction while the box is
    crossed and its level is below the depth; every leaf carries the
    (p+1)^d Gauss-Legendre rule (Section "Perforated plate");
  * a point is fictitious when it lies strictly inside some ball;
  * a point source x_s gives f_x,i = alpha(x_s) N_i(x_s) (Eq. f with a
    Dirac load).

Nodes are numbered on the full structured node grid, x fastest; inactive
nodes (those of empty cells only) carry no rows or columns.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .basis import gauss_legendre, gll, lagrange, lagrange_deriv

EMPTY, CUT, UNCUT = 0, 1, 2
ETA_EMPTY = 1e-10


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
class BallUnion:
    """Physical domain = box minus the union of open balls."""

    def __init__(self, centers, radii, dim):
        self.r = np.asarray(radii, dtype=np.float64).reshape(-1)
        if len(self.r):
            self.c = np.asarray(centers, dtype=np.float64).reshape(len(self.r), -1)[:, :dim]
        else:
            self.c = np.zeros((0, dim))
        self.dim = dim

    def fictitious(self, X):
        X = np.asarray(X, dtype=np.float64)
        out = np.zeros(len(X), dtype=bool)
        for cj, rj in zip(self.c, self.r):
            out |= np.sum((X - cj) ** 2, axis=1) < rj * rj
        return out

    def _dists(self, lo, hi):
        lo, hi = np.asarray(lo), np.asarray(hi)
        near = np.clip(self.c, lo, hi)
        dmin = np.sqrt(np.sum((self.c - near) ** 2, axis=1))
        far = np.where(np.abs(self.c - lo) > np.abs(self.c - hi), lo, hi)
        dmax = np.sqrt(np.sum((self.c - far) ** 2, axis=1))
        return dmin, dmax

    def crossed(self, lo, hi) -> bool:
        if len(self.r) == 0:
            return False
        dmin, dmax = self._dists(lo, hi)
        return bool(np.any((dmin < self.r) & (self.r < dmax)))

    def inside(self, lo, hi) -> bool:
        if len(self.r) == 0:
            return False
        _, dmax = self._dists(lo, hi)
        return bool(np.any(dmax <= self.r))


class HalfSpace:
    """Physical iff x[axis] < level (the single-cell cut of Section
    "Critical time step analysis of cut cells")."""

    def __init__(self, axis, level):
        self.axis, self.level = axis, level

    def fictitious(self, X):
        return np.asarray(X)[:, self.axis] >= self.level

    def crossed(self, lo, hi) -> bool:
        return lo[self.axis] < self.level < hi[self.axis]

    def inside(self, lo, hi) -> bool:
        return lo[self.axis] >= self.level


def alpha(geom, X, alpha_f):
    return np.where(geom.fictitious(X), alpha_f, 1.0)


# --------------------------------------------------------------------------
# space tree and quadrature
# --------------------------------------------------------------------------
def tree_leaves(geom, lo, hi, depth) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Leaves of the space tree refined towards the boundary."""
    leaves = []
    dim = len(lo)

    def rec(lo, hi, level):
        if level < depth and geom.crossed(lo, hi):
            mid = 0.5 * (lo + hi)
            for corner in itertools.product((0, 1), repeat=dim):
                c = np.array(corner)
                clo = np.where(c == 0, lo, mid)
                chi = np.where(c == 0, mid, hi)
                rec(clo, chi, level + 1)
        else:
            leaves.append((lo.copy(), hi.copy()))

    rec(np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64), 0)
    return leaves


def tensor_rule(x1, w1, dim):
    """Tensor-product points (x fastest) and weights from a 1D rule."""
    pts = np.array(list(itertools.product(*([x1] * dim))))[:, ::-1]
    wts = np.prod(np.array(list(itertools.product(*([w1] * dim)))), axis=1)
    return pts, wts


def leaf_points(leaves, p, dim):
    """(p+1)^dim Gauss-Legendre points on every leaf, physical coordinates."""
    xg, wg = gauss_legendre(p + 1)
    ref, wref = tensor_rule(xg, wg, dim)
    X, W = [], []
    for lo, hi in leaves:
        half = 0.5 * (hi - lo)
        X.append(lo + (ref + 1.0) * half)
        W.append(wref * np.prod(half))
    return np.concatenate(X), np.concatenate(W)


# --------------------------------------------------------------------------
# element matrices
# --------------------------------------------------------------------------
def element_basis(p, lo, h, X):
    """Tensor Lagrange basis on GLL nodes of the cell [lo, lo+h]:
    values B (m, n^d) and physical gradients G (m, n^d, d); local node
    index a + n b (+ n^2 c), x fastest."""
    xi = 2.0 * (np.asarray(X) - lo) / np.asarray(h) - 1.0
    return element_basis_ref(p, h, xi)


def element_basis_ref(p, h, xi):
    """As element_basis, at reference coordinates xi in [-1, 1]^d."""
    nodes, _ = gll(p)
    dim = len(h)
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    vals = [lagrange(nodes, xi[:, k]) for k in range(dim)]
    ders = [lagrange_deriv(nodes, xi[:, k]) * (2.0 / h[k]) for k in range(dim)]
    n = p + 1
    m = len(xi)
    B = np.ones((m, n ** dim))
    G = np.ones((m, n ** dim, dim))
    for loc, idx in enumerate(itertools.product(range(n), repeat=dim)):
        idx = idx[::-1]                   # idx[0] is the x index (fastest)
        for k in range(dim):
            B[:, loc] *= vals[k][:, idx[k]]
            for g in range(dim):
                G[:, loc, g] *= (ders[k][:, idx[k]] if g == k else vals[k][:, idx[k]])
    return B, G


def quadrature_matrices(p, lo, h, X, W, dens, kappa, xi=None):
    """M_ij = sum_q W_q dens_q N_i N_j and K_ij = sum_q W_q kappa_q grad N_i . grad N_j
    (points X in physical coordinates, or xi in reference coordinates)."""
    B, G = element_basis(p, lo, h, X) if xi is None else element_basis_ref(p, h, xi)
    M = B.T @ (B * (W * dens)[:, None])
    K = np.zeros_like(M)
    for g in range(G.shape[2]):
        K += G[:, :, g].T @ (G[:, :, g] * (W * kappa)[:, None])
    return M, K


def uncut_element_matrices(p, h, rho, kappa):
    """Uncut cell: mass by GLL quadrature (diagonal), stiffness by
    (p+1)^d-point Gauss-Legendre quadrature (Section "Spatial
    Discretization", last paragraph)."""
    dim = len(h)
    lo = np.zeros(dim)
    h = np.asarray(h, dtype=np.float64)
    xl, wl = gll(p)
    ref, wref = tensor_rule(xl, wl, dim)
    Xm = lo + (ref + 1.0) * 0.5 * h
    Wm = wref * np.prod(0.5 * h)
    M, _ = quadrature_matrices(p, lo, h, Xm, Wm, np.full(len(Wm), rho), np.zeros(len(Wm)),
                               xi=ref)
    xg, wg = gauss_legendre(p + 1)
    ref, wref = tensor_rule(xg, wg, dim)
    Xk = lo + (ref + 1.0) * 0.5 * h
    Wk = wref * np.prod(0.5 * h)
    _, K = quadrature_matrices(p, lo, h, Xk, Wk, np.zeros(len(Wk)), np.full(len(Wk), kappa))
    return M, K


def cut_element_matrices(geom, p, lo, h, depth, rho, kappa, alpha_f):
    """Cut cell: consistent M and K by Gauss-Legendre points on the leaves of
    the space tree, with alpha scaling density and stiffness."""
    lo = np.asarray(lo, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    leaves = tree_leaves(geom, lo, lo + h, depth)
    X, W = leaf_points(leaves, p, len(lo))
    a = alpha(geom, X, alpha_f)
    M, K = quadrature_matrices(p, lo, h, X, W, rho * a, kappa * a)
    return M, K


def fill_ratio(geom, p, lo, h, depth):
    lo = np.asarray(lo, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    leaves = tree_leaves(geom, lo, lo + h, depth)
    X, W = leaf_points(leaves, p, len(lo))
    return float(np.sum(W * (~geom.fictitious(X))) / np.prod(h))


def omega_max(K, M):
    """sqrt of the largest eigenvalue of K x = lambda M x (Section "Critical
    time step analysis of cut cells")."""
    return float(np.sqrt(scipy.linalg.eigh(K, M, eigvals_only=True)[-1]))


# --------------------------------------------------------------------------
# mesh, classification and assembly
# --------------------------------------------------------------------------
@dataclass
class Discretisation:
    dim: int
    p: int
    n_cells: Tuple[int, ...]
    grid: Tuple[int, ...]
    h: np.ndarray
    flags: np.ndarray            # per cell: EMPTY / CUT / UNCUT (x fastest)
    M: sp.csr_matrix             # full-grid size, inactive rows empty
    K: sp.csr_matrix
    fx: np.ndarray               # spatial load vector (full grid)
    Id: np.ndarray               # diagonal (explicit) dofs, grid indices ascending
    Ic: np.ndarray               # cut (implicit) dofs, grid indices ascending
    dt_crit_uncut: float
    dt: float

    @property
    def n_grid(self):
        return int(np.prod(self.grid))

    @property
    def active(self):
        return np.union1d(self.Id, self.Ic)


def geometry_of(w):
    return BallUnion(w.hole_centers, w.hole_radii, w.dim)


def cell_box(w, cell_idx):
    h = np.array(w.h)
    lo = np.array(cell_idx, dtype=np.float64) * h
    return lo, h


def cell_nodes(grid, p, cell_idx):
    """Global node ids of a cell's (p+1)^d nodes, local order x fastest."""
    dim = len(cell_idx)
    n = p + 1
    ids = []
    for idx in itertools.product(range(n), repeat=dim):
        idx = idx[::-1]
        g = 0
        stride = 1
        for k in range(dim):
            g += (cell_idx[k] * p + idx[k]) * stride
            stride *= grid[k]
        ids.append(g)
    return np.array(ids, dtype=np.int64)


def all_cells(n_cells):
    dim = len(n_cells)
    return [tuple(reversed(c)) for c in itertools.product(*[range(n) for n in reversed(n_cells)])]


def cell_flag(w, geom, cidx, forced=False):
    """Flag of one cell (its index tuple, x first) following the reading in
    the module doc; forced: an uncut cell treated as cut."""
    lo, h = cell_box(w, cidx)
    if geom.inside(lo, lo + h):
        return EMPTY
    if geom.crossed(lo, lo + h):
        eta = fill_ratio(geom, w.p, lo, h, w.tree_depth)
        return EMPTY if eta < ETA_EMPTY else CUT
    return CUT if forced else UNCUT


def classify(w, geom=None):
    """Per-cell flags (x fastest) following the reading in the module doc."""
    geom = geom or geometry_of(w)
    cells = all_cells(w.n_cells)
    flags = np.full(len(cells), UNCUT, dtype=np.int8)
    forced = set(int(i) for i in (w.forced_cut if w.forced_cut is not None else []))
    for cid, cidx in enumerate(cells):
        flags[cid] = cell_flag(w, geom, cidx, cid in forced)
    return flags


def uncut_dt(w):
    """Cell-wise critical step of an uncut cell times the CFL factor."""
    kappa = w.rho * w.c ** 2
    Me, Ke = uncut_element_matrices(w.p, w.h, w.rho, kappa)
    dtc = 2.0 / omega_max(Ke, Me)
    return dtc, w.cfl * dtc


def point_source(w, geom, grid):
    """f_x for a Dirac load at w.source (global basis evaluated there)."""
    xs = np.asarray(w.source[:w.dim], dtype=np.float64)
    h = np.array(w.h)
    cidx = tuple(int(min(max(np.floor(xs[k] / h[k]), 0), w.n_cells[k] - 1)) for k in range(w.dim))
    lo = np.array(cidx) * h
    B, _ = element_basis(w.p, lo, h, xs[None, :])
    fx = np.zeros(int(np.prod(grid)))
    fx[cell_nodes(grid, w.p, cidx)] = alpha(geom, xs[None, :], w.alpha_f)[0] * B[0]
    return fx, cidx


def sample_points(w, u, points):
    """The finite element field with nodal values u (grid vector) at physical
    points: the cell that contains each point (the lower one on a cell
    face), then the tensor Lagrange basis of Section "Spatial
    discretisation" at the point.  A point in an empty cell is an error."""
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    grid = tuple(w.grid_nodes)
    flags = classify(w)
    out = np.empty(len(pts))
    for r, x in enumerate(pts):
        cidx = tuple(min(int(np.floor(x[k] / w.h[k])), w.n_cells[k] - 1) for k in range(w.dim))
        cid = sum(cidx[k] * int(np.prod(w.n_cells[:k])) for k in range(w.dim))
        if flags[cid] == EMPTY:
            raise ValueError(f"point {x} lies in an empty cell")
        lo, h = cell_box(w, cidx)
        B, _ = element_basis(w.p, lo, h, x[None, :])
        out[r] = B[0] @ np.asarray(u)[cell_nodes(grid, w.p, cidx)]
    return out


def hrz_lump(Me):
    """HRZ lumping (Hinton, Rock and Zienkiewicz) of an element mass matrix:
    its diagonal, scaled so that the lumped matrix keeps the element's total
    mass, the sum of all entries of the consistent matrix."""
    d = np.diag(Me).copy()
    return np.diag(d * (Me.sum() / d.sum()))


def assemble(w) -> Discretisation:
    """Global M, K, f_x and the d/c partition for a workload."""
    geom = geometry_of(w)
    grid = tuple(w.grid_nodes)
    ng = int(np.prod(grid))
    kappa = w.rho * w.c ** 2
    flags = classify(w, geom)
    cells = all_cells(w.n_cells)
    Mu, Ku = uncut_element_matrices(w.p, w.h, w.rho, kappa)
    rows, cols, mv, kv = [], [], [], []
    ncell_nodes = (w.p + 1) ** w.dim
    uncut_nodes = []
    cut_nodes = []
    for cid, cidx in enumerate(cells):
        if flags[cid] == EMPTY:
            continue
        nodes = cell_nodes(grid, w.p, cidx)
        if flags[cid] == UNCUT:
            uncut_nodes.append(nodes)
            continue
        lo, h = cell_box(w, cidx)
        Me, Ke = cut_element_matrices(geom, w.p, lo, h, w.tree_depth, w.rho, kappa, w.alpha_f)
        if getattr(w, "cut_mass", "consistent") == "hrz":
            Me = hrz_lump(Me)
        cut_nodes.append(nodes)
        rows.append(np.repeat(nodes, ncell_nodes))
        cols.append(np.tile(nodes, ncell_nodes))
        mv.append(Me.ravel())
        kv.append(Ke.ravel())
    if uncut_nodes:
        U = np.array(uncut_nodes)
        rows.append(np.repeat(U, ncell_nodes, axis=1).ravel())
        cols.append(np.tile(U, (1, ncell_nodes)).ravel())
        mv.append(np.tile(Mu.ravel(), len(U)))
        kv.append(np.tile(Ku.ravel(), len(U)))
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        M = sp.coo_matrix((np.concatenate(mv), (r, c)), shape=(ng, ng)).tocsr()
        K = sp.coo_matrix((np.concatenate(kv), (r, c)), shape=(ng, ng)).tocsr()
    else:
        M = sp.csr_matrix((ng, ng))
        K = sp.csr_matrix((ng, ng))
    M.eliminate_zeros()
    K.eliminate_zeros()
    Ic = np.unique(np.concatenate(cut_nodes)) if cut_nodes else np.zeros(0, np.int64)
    act = np.unique(np.concatenate(cut_nodes + uncut_nodes)) if (cut_nodes or uncut_nodes) \
        else np.zeros(0, np.int64)
    Id = np.setdiff1d(act, Ic)
    fx, _ = point_source(w, geom, grid)
    dtc, dt = uncut_dt(w)
    return Discretisation(dim=w.dim, p=w.p, n_cells=tuple(w.n_cells), grid=grid,
                          h=np.array(w.h), flags=flags, M=M, K=K, fx=fx, Id=Id, Ic=Ic,
                          dt_crit_uncut=dtc, dt=dt)


def c_components(disc: Discretisation):
    """Connected components of the implicit block (graph of K^cc and M^cc)."""
    import scipy.sparse.csgraph as csg
    Ic = disc.Ic
    A = (abs(disc.K[Ic][:, Ic]) + abs(disc.M[Ic][:, Ic])).tocsr()
    n, lab = csg.connected_components(A, directed=False)
    return n, lab


def sumfact_stiffness(w, disc):
    """K u by cells instead of the assembled matrix: every uncut cell's
    contribution by sum factorisation of the exact 1D matrices (2D:
    kappa [(h_y/h_x) M U K^T + (h_x/h_y) K U M^T] on the cell's nodal values
    U[b, a]; 3D: the three-term analogue), every cut cell's by its dense
    element matrix, summed node by node in cell order.  The same operator as
    the assembled K with another rounding (the form the device kernels
    compute the uncut part in); returns a function u -> K u on the grid."""
    p, dim = w.p, w.dim
    n = p + 1
    kappa = w.rho * w.c ** 2
    xl, _ = gll(p)
    xg, wg = gauss_legendre(n)
    from .basis import lagrange, lagrange_deriv
    Nq, Dq = lagrange(xl, xg), lagrange_deriv(xl, xg)
    Mh = (Nq * wg[:, None]).T @ Nq
    Kh = (Dq * wg[:, None]).T @ Dq
    h = np.asarray(w.h, dtype=np.float64)
    grid = tuple(w.grid_nodes)
    ng = int(np.prod(grid))
    cells = all_cells(w.n_cells)
    uncut = [c for cid, c in enumerate(cells) if disc.flags[cid] == UNCUT]
    cut = [c for cid, c in enumerate(cells) if disc.flags[cid] == CUT]
    ids_u = np.array([cell_nodes(grid, p, c) for c in uncut], dtype=np.int64).reshape(len(uncut), -1)
    geom = geometry_of(w)
    cut_data = []
    for c in cut:
        lo, hh = cell_box(w, c)
        Me, Ke = cut_element_matrices(geom, p, lo, hh, w.tree_depth, w.rho, kappa, w.alpha_f)
        cut_data.append((cell_nodes(grid, p, c), Ke))
    if dim == 2:
        sx, sy = kappa * h[1] / h[0], kappa * h[0] / h[1]
    else:
        sx = kappa * h[1] * h[2] / (2.0 * h[0])
        sy = kappa * h[0] * h[2] / (2.0 * h[1])
        sz = kappa * h[0] * h[1] / (2.0 * h[2])

    def apply(u):
        parts_i, parts_v = [], []
        if len(uncut):
            if dim == 2:
                U = u[ids_u].reshape(-1, n, n)                    # [e, b, a]
                Y = sx * np.einsum("ij,ejk,lk->eil", Mh, U, Kh) + sy * np.einsum("ij,ejk,lk->eil", Kh, U, Mh)
            else:
                U = u[ids_u].reshape(-1, n, n, n)                 # [e, c, b, a]
                Y = (sx * np.einsum("ci,bj,ak,eijk->ecba", Mh, Mh, Kh, U)
                     + sy * np.einsum("ci,bj,ak,eijk->ecba", Mh, Kh, Mh, U)
                     + sz * np.einsum("ci,bj,ak,eijk->ecba", Kh, Mh, Mh, U))
            parts_i.append(ids_u.ravel())
            parts_v.append(Y.reshape(len(uncut), -1).ravel())
        for nodes, Ke in cut_data:
            parts_i.append(nodes)
            parts_v.append(Ke @ u[nodes])
        if not parts_i:
            return np.zeros(ng)
        return np.bincount(np.concatenate(parts_i), weights=np.concatenate(parts_v), minlength=ng)

    return apply

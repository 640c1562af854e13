"""Interface-fitted tensor-product mesh of quadrilaterals / hexahedra.

Section 2.2 asks for a mesh of quads or hexes whose cells do not cut the
fluid-solid interface.  The channel is split per axis into level-0 segments
whose ends include the faces of the elastic bar; a level-l mesh bisects every
level-0 cell l times per axis, so every level of the hierarchy is
interface-fitted and each 2x2 (2x2x2) block of level-l cells is one level
(l-1) cell.

Numbering: node (i, j[, k]) has index i + (nx+1) j (+ (nx+1)(ny+1) k);
cell (i, j[, k]) has index i + nx j (+ nx ny k); the local node a of a cell
sits at offset (a & 1, (a >> 1) & 1, (a >> 2) & 1).
"""
from __future__ import annotations

import itertools

import numpy as np


class Mesh:
    """degree 1: Q1 cells with 2^d vertex nodes; degree 2 (Section 2.2's Q2): the same
    cells with (3)^d nodes each, the vertices plus the edge, face and cell midpoints, so
    that the nodes of a level-l Q2 mesh are the vertices of the level-(l + 1) mesh.
    Local node a of a cell sits at offset (digit r of a in base degree + 1) / degree on
    axis r."""

    def __init__(self, p: dict, level: int | None = None, degree: int = 1):
        self.dim = d = p["dim"]
        self.level = p["level"] if level is None else level
        self.degree = degree
        axes = []
        for ax in p["segments"][:d]:
            pts = []
            for (lo, hi, n) in ax:
                nl = n * 2 ** self.level
                pts.extend(lo + (hi - lo) * np.arange(nl) / nl)
            pts.append(ax[-1][1])
            axes.append(np.asarray(pts, dtype=np.float64))
        self.axes = axes                                       # cell vertices per axis
        self.shape = tuple(len(a) - 1 for a in axes)          # cells per axis
        if degree == 2:
            naxes = []
            for a in axes:
                na = np.empty(2 * a.size - 1)
                na[0::2] = a
                na[1::2] = 0.5 * (a[:-1] + a[1:])
                naxes.append(na)
        else:
            naxes = axes
        self.naxes = naxes                                     # node coordinates per axis
        self.nshape = tuple(len(a) for a in naxes)             # nodes per axis
        self.n_nodes = int(np.prod(self.nshape))
        self.n_cells = int(np.prod(self.shape))
        self.nloc = (degree + 1) ** d

        # node coordinates [n_nodes, d]
        grids = np.meshgrid(*naxes, indexing="ij")
        self.X = np.stack([g.ravel(order="F") for g in grids], axis=1)
        # node multi-index
        nidx = np.meshgrid(*[np.arange(n) for n in self.nshape], indexing="ij")
        self.node_ijk = np.stack([g.ravel(order="F") for g in nidx], axis=1)

        # cells: multi-index, connectivity, sizes
        cidx = np.meshgrid(*[np.arange(n) for n in self.shape], indexing="ij")
        self.cell_ijk = np.stack([g.ravel(order="F") for g in cidx], axis=1)
        self.conn = np.zeros((self.n_cells, self.nloc), dtype=np.int64)
        for a in range(self.nloc):
            off = [(a // (degree + 1) ** q) % (degree + 1) for q in range(d)]
            self.conn[:, a] = self.node_index(degree * self.cell_ijk + np.asarray(off))
        self.h = np.stack([np.diff(axes[q])[self.cell_ijk[:, q]] for q in range(d)], axis=1)
        self.x0 = np.stack([axes[q][self.cell_ijk[:, q]] for q in range(d)], axis=1)

        # solid cells: cell centre inside the bar box
        lo = np.asarray(p["solid_lo"][:d])
        hi = np.asarray(p["solid_hi"][:d])
        centre = self.x0 + 0.5 * self.h
        self.solid = np.all((centre > lo) & (centre < hi), axis=1)
        self.fluid = ~self.solid

        # node classes N_S (nodes of solid cells), N_F (nodes of fluid cells)
        self.in_NS = np.zeros(self.n_nodes, dtype=bool)
        self.in_NS[self.conn[self.solid].ravel()] = True
        self.in_NF = np.zeros(self.n_nodes, dtype=bool)
        self.in_NF[self.conn[self.fluid].ravel()] = True

        # boundary node flags
        X = self.X
        L = np.asarray([a[-1] for a in axes])
        tol = 1e-12
        self.on_inflow = np.abs(X[:, 0]) < tol
        self.on_outflow = np.abs(X[:, 0] - L[0]) < tol
        self.on_wall = np.zeros(self.n_nodes, dtype=bool)
        for q in range(1, d):
            self.on_wall |= (np.abs(X[:, q]) < tol) | (np.abs(X[:, q] - L[q]) < tol)
        self.L = L

        # outflow faces: cells in the last x-column
        self.outflow_cells = np.nonzero(self.cell_ijk[:, 0] == self.shape[0] - 1)[0]

    def node_index(self, ijk: np.ndarray) -> np.ndarray:
        ijk = np.asarray(ijk)
        idx = ijk[..., 0].astype(np.int64)
        stride = self.nshape[0]
        for q in range(1, self.dim):
            idx = idx + stride * ijk[..., q]
            stride *= self.nshape[q]
        return idx

    def n_dofs(self) -> int:
        return self.n_nodes * (2 * self.dim + 1)


def local_offsets(dim: int) -> np.ndarray:
    """Offsets of the 2**dim local nodes of a cell (bit q of a -> axis q)."""
    return np.asarray([[(a >> q) & 1 for q in range(dim)] for a in range(2 ** dim)])


def child_positions(dim: int):
    return list(itertools.product((0, 1), repeat=dim))

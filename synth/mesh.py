"""Structured triangular meshes for the synthetic workloads.

Input generation only: this module builds node coordinates and connectivity
and holds none of the method's arithmetic.  Both the CPU oracle and the GPU
library receive its arrays.

Conventions (a reading of the paper, which uses "standard nodal DG" on a
simplex mesh without fixing a node order, Section 2.3):

* geometry nodes form a row-major grid with spacing h/q, so that for q = 2
  every mid-edge node (including the cell centre on the diagonal) is a grid
  node;
* each cell (i, j) is split along its SW->NE diagonal into a lower triangle
  (v00, v10, v11) and an upper triangle (v00, v11, v01), both counter-clockwise;
* elements are numbered cell-major (row j, column i), lower triangle first;
* element nodes: the three vertices, then (q = 2) the mid-edge nodes of
  edges 0, 1, 2 where edge f joins vertex f and vertex (f + 1) % 3;
* face f of an element is edge f; ``elem_nbr[e, f]`` is the neighbouring
  element or ``-tag`` with tags 1 left (x = 0), 2 right (x = Lx),
  3 bottom (y = 0), 4 top (y = Ly).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    nx: int
    ny: int
    Lx: float
    Ly: float
    q: int                    # geometry (and solution) polynomial degree
    X: np.ndarray             # [n_gnode, 2] reference node coordinates
    elem_gnodes: np.ndarray   # [n_elem, n_gn] int32
    elem_nbr: np.ndarray      # [n_elem, 3] int32, neighbour or -tag

    @property
    def n_elem(self) -> int:
        return self.elem_gnodes.shape[0]

    @property
    def n_gnode(self) -> int:
        return self.X.shape[0]

    @property
    def n_gn(self) -> int:
        return self.elem_gnodes.shape[1]

    def node_coords(self) -> np.ndarray:
        """[n_elem, n_gn, 2] reference coordinates of every element node."""
        return self.X[self.elem_gnodes]


def structured_mesh(nx: int, ny: int, Lx: float, Ly: float, q: int) -> Mesh:
    if q not in (1, 2):
        raise ValueError("q must be 1 or 2")
    gx, gy = q * nx + 1, q * ny + 1
    ii, jj = np.meshgrid(np.arange(gx), np.arange(gy), indexing="xy")
    X = np.stack([ii.ravel() * (Lx / (q * nx)), jj.ravel() * (Ly / (q * ny))], axis=1)

    def gid(a, b):
        return b * gx + a

    n_gn = 3 if q == 1 else 6
    elem = np.zeros((2 * nx * ny, n_gn), dtype=np.int32)
    nbr = np.zeros((2 * nx * ny, 3), dtype=np.int32)
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            v00 = (q * i, q * j)
            v10 = (q * (i + 1), q * j)
            v11 = (q * (i + 1), q * (j + 1))
            v01 = (q * i, q * (j + 1))
            for t, verts in enumerate(((v00, v10, v11), (v00, v11, v01))):
                e = 2 * c + t
                nodes = [gid(*v) for v in verts]
                if q == 2:
                    for f in range(3):
                        a, b = verts[f], verts[(f + 1) % 3]
                        nodes.append(gid((a[0] + b[0]) // 2, (a[1] + b[1]) // 2))
                elem[e] = nodes
            lo, up = 2 * c, 2 * c + 1
            nbr[lo, 0] = -3 if j == 0 else 2 * ((j - 1) * nx + i) + 1
            nbr[lo, 1] = -2 if i == nx - 1 else 2 * (j * nx + i + 1) + 1
            nbr[lo, 2] = up
            nbr[up, 0] = lo
            nbr[up, 1] = -4 if j == ny - 1 else 2 * ((j + 1) * nx + i)
            nbr[up, 2] = -1 if i == 0 else 2 * (j * nx + i - 1)
    return Mesh(nx, ny, float(Lx), float(Ly), q, X, elem, nbr)

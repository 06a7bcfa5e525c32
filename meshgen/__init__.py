"""Seeded synthetic inputs for finite element assembly: meshes, coefficients, upstream gradients.

This module is shared by the tests, the benchmark and the CPU oracle's callers.  It holds
no part of the assembly method itself: no Jacobians, no basis functions, no quadrature,
no sparsity pattern.  It only lays out structured meshes in the shapes the paper's
experiments use (structured grids of P1 triangles, Section 6) and the 3D tetrahedral
meshes of the same kind, perturbs interior nodes, and draws random coefficients.

Conventions (all arrays are numpy, C-contiguous):

* ``coords``: float64, structure-of-arrays ``[dim][n_nodes]``.
* ``conn``: int32, structure-of-arrays ``[npe][n_elems]`` (npe = 3 for P1 triangles,
  4 for P1 tetrahedra, 10 for P2 tetrahedra).
* Nodes are numbered lexicographically with x fastest.  Elements are cell-major: all
  elements of one grid cell are consecutive and cells are numbered with x fastest.
* 2D cells are split along the (i,j)-(i+1,j+1) diagonal into two triangles, which gives
  at most 7 nonzeros per matrix row (the MAX_NZ the paper quotes for its 2D example,
  Section 5, sparse variant).
* 3D cells are split into the 6 Kuhn (Freudenthal) tetrahedra along the cube's
  (0,0,0)-(1,1,1) diagonal: tetrahedron p visits the corners 000 -> +e_{p0} -> +e_{p1} -> 111.
* P2 meshes live on the (2n+1)^3 half grid.  Local node order: the 4 vertices, then the
  edge nodes of edges (01, 02, 03, 12, 13, 23).  Edge nodes sit at the midpoints of their
  (possibly jittered) end vertices, so every element stays affine.
* Jitter: each coordinate of each interior vertex gets an independent U[-a*h, a*h] shift
  (default a = 0.2); boundary vertices stay put, so the domain is exactly [0,1]^dim.
"""

from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Mesh",
    "square_tri",
    "cube_tet",
    "coefficients",
    "upstream_grads",
    "batch_plan",
    "KUHN_PERMS",
    "P2_EDGES",
]

# Axis orders of the 6 Kuhn tetrahedra of a unit cube.
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
# Local vertex pairs of the P2 edge nodes, in local order 4..9.
P2_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


@dataclasses.dataclass
class Mesh:
    dim: int
    order: int
    n: int  # cells per side
    coords: np.ndarray  # float64 [dim][n_nodes]
    conn: np.ndarray  # int32 [npe][n_elems]

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[1])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[1])

    @property
    def npe(self) -> int:
        return int(self.conn.shape[0])

    @property
    def h(self) -> float:
        return 1.0 / self.n


def _rng(seed: int, stream: int) -> np.random.Generator:
    # Independent PCG64 streams per purpose so that, e.g., coefficients do not change
    # when the jitter amplitude does.
    return np.random.default_rng([int(seed), int(stream)])


def _jitter(grid_pts: np.ndarray, n: int, amp: float, seed: int) -> np.ndarray:
    """grid_pts: int [dim][nv] lattice coordinates in 0..n.  Returns float64 [dim][nv]."""
    dim, nv = grid_pts.shape
    h = 1.0 / n
    x = grid_pts.astype(np.float64) * h
    if amp > 0.0:
        interior = np.all((grid_pts > 0) & (grid_pts < n), axis=0)
        idx = np.nonzero(interior)[0]
        d = _rng(seed, 1).uniform(-amp * h, amp * h, size=(idx.size, dim))
        x[:, idx] += d.T
    return x


def square_tri(n: int, jitter: float = 0.2, seed: int = 0) -> Mesh:
    """Unit square, n x n cells, 2 P1 triangles per cell."""
    m = n + 1
    jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    grid = np.stack([ii.ravel(), jj.ravel()])  # node id = i + m*j
    coords = _jitter(grid, n, jitter, seed)
    cj, ci = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    v00 = ci + m * cj
    v10 = v00 + 1
    v11 = v00 + 1 + m
    v01 = v00 + m
    t0 = np.stack([v00, v10, v11])
    t1 = np.stack([v00, v11, v01])
    conn = np.empty((3, 2 * n * n), dtype=np.int32)
    conn[:, 0::2] = t0
    conn[:, 1::2] = t1
    return Mesh(2, 1, n, np.ascontiguousarray(coords), conn)


def _kuhn_corners():
    """Corner offsets (4 x 3 ints) of the 6 Kuhn tetrahedra."""
    out = []
    for p in KUHN_PERMS:
        c = [np.zeros(3, dtype=np.int64)]
        for ax in p:
            nxt = c[-1].copy()
            nxt[ax] += 1
            c.append(nxt)
        out.append(np.stack(c))
    return np.stack(out)  # [6][4][3]


def cube_tet(n: int, order: int = 1, jitter: float = 0.2, seed: int = 0) -> Mesh:
    """Unit cube, n^3 cells, 6 Kuhn tetrahedra per cell, Lagrange order 1 or 2."""
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    corners = _kuhn_corners()  # [6][4][3]
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cell = np.stack([ci.ravel(), cj.ravel(), ck.ravel()])  # [3][ncell], x fastest
    ncell = cell.shape[1]
    # lattice positions of the 4 vertices of every element [4][3][E]; element = 6*cell + t
    vpos = np.empty((4, 3, ncell * 6), dtype=np.int64)
    for t in range(6):
        vpos[:, :, t::6] = cell[None, :, :] + corners[t][:, :, None]

    if order == 1:
        m = n + 1
        vid = vpos[:, 0, :] + m * (vpos[:, 1, :] + m * vpos[:, 2, :])
        kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
        grid = np.stack([ii.ravel(), jj.ravel(), kk.ravel()])
        coords = _jitter(grid, n, jitter, seed)
        return Mesh(3, 1, n, np.ascontiguousarray(coords), np.ascontiguousarray(vid.astype(np.int32)))

    # P2 on the half grid: node id x + m (y + m z) for half-grid position (x, y, z); the
    # id is linear in the position, so an edge node's id is the mean of its end vertices'
    m = 2 * n + 1
    E = vpos.shape[2]
    hid = np.empty((10, E), dtype=np.int64)
    hid[:4] = 2 * (vpos[:, 0, :] + m * (vpos[:, 1, :] + m * vpos[:, 2, :]))
    for k, (a, b) in enumerate(P2_EDGES):
        hid[4 + k] = (hid[a] + hid[b]) // 2
    # vertex coordinates: jitter on the vertex lattice
    mv = n + 1
    kk, jj, ii = np.meshgrid(np.arange(mv), np.arange(mv), np.arange(mv), indexing="ij")
    vgrid = np.stack([ii.ravel(), jj.ravel(), kk.ravel()])
    vx = _jitter(vgrid, n, jitter, seed)
    # every half-grid node is a vertex (all coordinates even) or the midpoint of the
    # edge between pos - s and pos + s, s = its odd coordinates: all Kuhn edges run along
    # 0/1 directions
    hz, hy, hx = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    pos = np.stack([hx.ravel(), hy.ravel(), hz.ravel()])
    odd = pos & 1
    lo = (pos - odd) // 2
    hi = (pos + odd) // 2
    vlo = lo[0] + mv * (lo[1] + mv * lo[2])
    vhi = hi[0] + mv * (hi[1] + mv * hi[2])
    is_vertex = ~odd.any(axis=0)
    coords = np.where(is_vertex[None, :], vx[:, vlo], 0.5 * (vx[:, vlo] + vx[:, vhi]))
    return Mesh(3, 2, n, np.ascontiguousarray(coords), np.ascontiguousarray(hid.astype(np.int32)))


def coefficients(n_elems: int, form: str, seed: int = 0) -> np.ndarray:
    """Per-element coefficients, structure-of-arrays [ncoef][n_elems], float64.

    form "helmholtz": kappa ~ U[0.5, 2]                      -> [1][E]
    form "elasticity": lambda ~ U[0.5, 2], mu ~ U[0.3, 1]    -> [2][E]
    """
    r = _rng(seed, 2)
    if form == "helmholtz":
        return r.uniform(0.5, 2.0, size=(1, n_elems))
    if form == "elasticity":
        lam = r.uniform(0.5, 2.0, size=n_elems)
        mu = r.uniform(0.3, 1.0, size=n_elems)
        return np.stack([lam, mu])
    raise ValueError(form)


def upstream_grads(nnz: int, n_rows: int, seed: int = 0):
    """G ~ N(0,1) on every stored matrix entry and g ~ N(0,1) on every RHS row."""
    r = _rng(seed, 3)
    return r.standard_normal(nnz), r.standard_normal(n_rows)


def batch_plan(n_meshes: int = 512, nmin: int = 6, nmax: int = 32, seed: int = 0):
    """Mixed batch: list of (n, order, form, mesh_seed).

    n ~ U{nmin..nmax}; each mesh is P1 Helmholtz or P2 elasticity with probability 1/2.
    """
    r = _rng(seed, 4)
    ns = r.integers(nmin, nmax + 1, size=n_meshes)
    p2 = r.random(n_meshes) < 0.5
    plan = []
    for k in range(n_meshes):
        if p2[k]:
            plan.append((int(ns[k]), 2, "elasticity", 1000 + k))
        else:
            plan.append((int(ns[k]), 1, "helmholtz", 1000 + k))
    return plan

"""Discrete impedance Helmholtz operator, right-hand side and direct solve.

TEST INFRASTRUCTURE ONLY (see the package header).

The continuous problem is -u'' - k^2 u = f with impedance conditions
d_n u - i k u = g (eq. (lap1), Sec. 1; in 2D the free-space problem of
Sec. 3.1 on the unit square).  The paper discretises it as A u = f
(Sec. 1) with bilinear elements (Sec. 3); this code uses the cell-assembled
second-order finite-difference scheme read as follows:

* nodes x = (p h, q h), 0 <= p, q <= N, h = 1/N, node (p, q) at index
  p*(N+1) + q; every node (boundary ones included) is an unknown;
* the matrix A_D of a box D (a union of cells: the whole square for A, a
  subdomain for the local operator with impedance conditions on its own
  boundary, Sec. 1) is the sum over the cells of D of
    - for each edge (a, b) of the cell: (1/2)/h^2 (e_a - e_b)(e_a - e_b)^T,
    - for each node x of the cell: -(1/4) k(x)^2 on the diagonal,
  plus, for each edge (a, b) on the boundary of D, -(1/2) i k(x)/h at each
  of its two end nodes x;
* 1D: each cell (a, b) adds 1/h^2 (e_a - e_b)(e_a - e_b)^T and -(1/2) k(x)^2 at
  its two nodes, and each end node of D gets -i k(x)/h.

Pins (tests/test_oracle_operator.py): complex symmetry A^T = A; the stencil
values at interior, edge and corner nodes; the Kronecker form of the 2D matrix
built from 1D pieces; the 1D discrete closed form for constant f and its O(h^2)
convergence to the continuous solution of eq. (lap1); a manufactured solution.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def n_nodes(dim: int, n_cells: int) -> int:
    return (n_cells + 1) ** dim


def box_shape(box) -> tuple[int, int]:
    p0, p1, q0, q1 = box
    return p1 - p0 + 1, q1 - q0 + 1


def box_global_indices(box, n_cells: int, dim: int) -> np.ndarray:
    """Global node indices of the nodes of box (p0, p1, q0, q1), local order p-major."""
    p0, p1, q0, q1 = box
    if dim == 1:
        return np.arange(p0, p1 + 1)
    P, Q = np.meshgrid(np.arange(p0, p1 + 1), np.arange(q0, q1 + 1), indexing="ij")
    return (P * (n_cells + 1) + Q).reshape(-1)


def box_matrix(n_cells: int, k_nodes: np.ndarray, box, dim: int) -> sp.csr_matrix:
    """Cell-assembled matrix A_D of box D = (p0, p1, q0, q1) (inclusive node ranges).

    ``k_nodes`` is the wavenumber at every node of the whole grid.  The result is
    indexed by the local nodes of D in p-major order.
    """
    h = 1.0 / n_cells
    p0, p1, q0, q1 = box
    nx, ny = box_shape(box)
    gidx = box_global_indices(box, n_cells, dim)
    kloc = np.asarray(k_nodes, dtype=np.float64)[gidx]
    rows: list[np.ndarray] = []
    cols: list[np.ndarray] = []
    vals: list[np.ndarray] = []

    def add(r, c, v):
        rows.append(np.asarray(r).ravel())
        cols.append(np.asarray(c).ravel())
        vals.append(np.broadcast_to(np.asarray(v, dtype=np.complex128), np.asarray(r).shape).ravel())

    if dim == 1:
        if nx < 2:
            raise ValueError("1D box needs at least two nodes")
        a = np.arange(nx - 1)
        b = a + 1
        w = 1.0 / h ** 2
        add(a, a, w)
        add(b, b, w)
        add(a, b, -w)
        add(b, a, -w)
        add(a, a, -0.5 * kloc[a] ** 2)
        add(b, b, -0.5 * kloc[b] ** 2)
        for x in (0, nx - 1):
            add(np.array([x]), np.array([x]), -1j * kloc[x] / h)
    else:
        if nx < 2 or ny < 2:
            raise ValueError("2D box needs at least two nodes per side")

        def loc(a, c):
            return a * ny + c

        A_, C_ = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="ij")
        A_ = A_.ravel()
        C_ = C_.ravel()
        # cell corners in counter-clockwise order
        corners = [loc(A_, C_), loc(A_ + 1, C_), loc(A_ + 1, C_ + 1), loc(A_, C_ + 1)]
        w = 0.5 / h ** 2
        for s, t in ((0, 1), (1, 2), (2, 3), (3, 0)):
            ia, ib = corners[s], corners[t]
            add(ia, ia, w)
            add(ib, ib, w)
            add(ia, ib, -w)
            add(ib, ia, -w)
        for ic in corners:
            add(ic, ic, -0.25 * kloc[ic] ** 2)
        # boundary edges of D: (cell mask, edge end nodes)
        bnd = [
            (C_ == 0, corners[0], corners[1]),           # bottom side q = q0
            (A_ == nx - 2, corners[1], corners[2]),      # right side p = p1
            (C_ == ny - 2, corners[2], corners[3]),      # top side q = q1
            (A_ == 0, corners[3], corners[0]),           # left side p = p0
        ]
        for mask, ea, eb in bnd:
            for x in (ea[mask], eb[mask]):
                add(x, x, -0.5j * kloc[x] / h)

    n = nx * ny
    A = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)
    ).tocsr()
    A.sum_duplicates()
    return A


def global_box(n_cells: int, dim: int):
    return (0, n_cells, 0, n_cells if dim == 2 else 0)


def global_matrix(n_cells: int, k_nodes: np.ndarray, dim: int) -> sp.csr_matrix:
    """A of the whole domain (Sec. 1: A u = f)."""
    return box_matrix(n_cells, k_nodes, global_box(n_cells, dim), dim)


def boundary_edge_count(n_cells: int, dim: int) -> np.ndarray:
    """Number of boundary facets of the whole domain at each node (2D: edges, 1D: end points)."""
    n = n_cells + 1
    if dim == 1:
        c = np.zeros(n)
        c[0] = c[-1] = 1.0
        return c
    P, Q = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    cx = (P > 0).astype(float) + (P < n - 1)
    cy = (Q > 0).astype(float) + (Q < n - 1)
    on_x = (P == 0) | (P == n - 1)
    on_y = (Q == 0) | (Q == n - 1)
    return (on_y * cx + on_x * cy).reshape(-1)


def rhs_vector(n_cells: int, f: np.ndarray, g: np.ndarray | None, dim: int) -> np.ndarray:
    """Discrete right-hand side b = f + impedance data.

    ``f`` is the discrete source vector of A u = f (Sec. 1).  ``g`` is the
    impedance data at the nodes (zero away from the boundary); it enters through
    the boundary facets of each node: 2D (number of boundary edges)/2 * g/h,
    1D g/h at the two end nodes.
    """
    b = np.array(f, dtype=np.complex128, copy=True)
    if g is None:
        return b
    h = 1.0 / n_cells
    nb = boundary_edge_count(n_cells, dim)
    scale = nb / 2.0 if dim == 2 else nb
    return b + scale * np.asarray(g) / h


def direct_solve(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    """u* = A^{-1} b by sparse LU with partial pivoting (SuperLU), complex128."""
    lu = spla.splu(sp.csc_matrix(A, dtype=np.complex128))
    return lu.solve(np.asarray(b, dtype=np.complex128))

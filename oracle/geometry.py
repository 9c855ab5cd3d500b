"""Hierarchical overlapping box decomposition.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows the decomposition of Sec. 1 (two overlapping intervals, each split
again: Omega_i into Omega_{2i+1}, Omega_{2i+2}) and the notation of Sec. 3
([m_x1 x m_y1, ..., m_xl x m_yl], element-based partition extended outward
by two elements, overlap delta = 4h).  Readings where the paper is silent:

* cuts at level l: M_l = m_1 * ... * m_l boxes per direction, cut j at cell
  floor(j N / M_l); the non-overlapping ("dyadic") boxes are nested;
* a child box extends delta_l/2 cells beyond its dyadic box on every side that
  is interior to the parent's dyadic box; a side on the parent's dyadic
  boundary takes the parent's (overlapping) extent; the result is clipped to
  the parent's extent;
* restricted prolongation P_i (ORAS, Sec. 1): a node of the parent box is
  clamped into the parent's dyadic range and owned by the child whose dyadic
  box holds it, half-open [c_j, c_{j+1}) with the last box closed;
* interface nodes B_i: the nodes of the child box that have a 5-point neighbour
  inside the parent box but outside the child box (the closure of the part of
  the child's boundary interior to the parent, Sec. 2);
* neighbours N(i): the siblings whose closed boxes intersect the closed box i;
* boxes at a level are numbered parent by parent, and inside a parent with the
  x position slow and the y position fast; interface nodes are listed in
  increasing local (p-major) index.

Pins (tests/test_oracle_geometry.py): the owned sets partition every parent box
(sum_i P_i R_i = I exactly); leaves of a hierarchy with equal overlap at every
level equal the boxes of the flat decomposition with the same finest cuts; the
worked 1D example of two subdomains overlapping by 20 cells; interface nodes are
exactly the rows where the local operator differs from the parent operator.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Box:
    level: int
    index: int
    parent: int
    pos: tuple[int, int]               # position (a, b) among the parent's children
    gpos: tuple[int, int]              # position among all boxes of the level
    dyadic: tuple[int, int, int, int]  # cell (== node) coordinates of the non-overlapping box
    ext: tuple[int, int, int, int]     # inclusive node ranges (p0, p1, q0, q1) of the box
    own: tuple[int, int, int, int]     # inclusive node ranges owned under P_i
    interface: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    neighbors: list[int] = field(default_factory=list)
    n_if: int = 0
    children: list[int] = field(default_factory=list)

    @property
    def shape(self) -> tuple[int, int]:
        return self.ext[1] - self.ext[0] + 1, self.ext[3] - self.ext[2] + 1

    @property
    def n(self) -> int:
        a, b = self.shape
        return a * b

    def local_index(self, p, q):
        return (np.asarray(p) - self.ext[0]) * self.shape[1] + (np.asarray(q) - self.ext[2])


@dataclass
class Hierarchy:
    dim: int
    n_cells: int
    m: list[tuple[int, int]]
    overlap: list[int]
    levels: list[list[Box]]  # levels[0] = [root], levels[l] = boxes of level l

    @property
    def depth(self) -> int:
        return len(self.levels) - 1

    def box(self, level: int, index: int) -> Box:
        return self.levels[level][index]


def _cuts(n_cells: int, M: int) -> list[int]:
    return [(j * n_cells) // M for j in range(M + 1)]


def build_hierarchy(dim: int, n_cells: int, m, overlap) -> Hierarchy:
    """Boxes of every level for the decomposition [m_1, ..., m_L] with overlaps delta_l (cells)."""
    m = [tuple(int(v) for v in mm) for mm in m]
    if dim == 1:
        m = [(mm[0], 1) for mm in m]
    overlap = [int(o) for o in overlap]
    if len(overlap) != len(m):
        raise ValueError("one overlap per level")
    if any(o % 2 for o in overlap):
        raise ValueError("overlap must be even (delta/2 cells per side)")
    ny_top = n_cells if dim == 2 else 0
    root = Box(level=0, index=0, parent=-1, pos=(0, 0), gpos=(0, 0), dyadic=(0, n_cells, 0, ny_top),
               ext=(0, n_cells, 0, ny_top), own=(0, n_cells, 0, ny_top))
    levels: list[list[Box]] = [[root]]
    Mx, My = 1, 1
    for lvl, ((mx, my), delta) in enumerate(zip(m, overlap), start=1):
        Mx, My = Mx * mx, My * my
        cx = _cuts(n_cells, Mx)
        cy = _cuts(n_cells, My) if dim == 2 else [0] * (My + 1)
        half = delta // 2
        boxes: list[Box] = []
        for pidx, par in enumerate(levels[-1]):
            PX, PY = par.gpos
            for a in range(mx):
                for b in range(my):
                    I, J = PX * mx + a, PY * my + b
                    dx0, dx1 = cx[I], cx[I + 1]
                    dy0, dy1 = (cy[J], cy[J + 1]) if dim == 2 else (0, 0)
                    P0, P1, Q0, Q1 = par.ext
                    p0 = P0 if a == 0 else max(dx0 - half, P0)
                    p1 = P1 if a == mx - 1 else min(dx1 + half, P1)
                    if dim == 2:
                        q0 = Q0 if b == 0 else max(dy0 - half, Q0)
                        q1 = Q1 if b == my - 1 else min(dy1 + half, Q1)
                    else:
                        q0 = q1 = 0
                    o_p0 = P0 if a == 0 else dx0
                    o_p1 = P1 if a == mx - 1 else dx1 - 1
                    if dim == 2:
                        o_q0 = Q0 if b == 0 else dy0
                        o_q1 = Q1 if b == my - 1 else dy1 - 1
                    else:
                        o_q0 = o_q1 = 0
                    bx = Box(level=lvl, index=len(boxes), parent=pidx, pos=(a, b), gpos=(I, J),
                             dyadic=(dx0, dx1, dy0, dy1), ext=(p0, p1, q0, q1),
                             own=(o_p0, o_p1, o_q0, o_q1))
                    par.children.append(bx.index)
                    boxes.append(bx)
        # interface nodes, neighbours and interface counts
        for bx in boxes:
            par = levels[-1][bx.parent]
            P0, P1, Q0, Q1 = par.ext
            p0, p1, q0, q1 = bx.ext
            sides = [p0 > P0, p1 < P1]
            if dim == 2:
                sides += [q0 > Q0, q1 < Q1]
            bx.n_if = int(sum(sides))
            P, Q = np.meshgrid(np.arange(p0, p1 + 1), np.arange(q0, q1 + 1), indexing="ij")
            on = np.zeros(P.shape, dtype=bool)
            if sides[0]:
                on |= P == p0
            if sides[1]:
                on |= P == p1
            if dim == 2:
                if sides[2]:
                    on |= Q == q0
                if sides[3]:
                    on |= Q == q1
            bx.interface = np.flatnonzero(on.reshape(-1))
            for other in (boxes[c] for c in par.children):
                if other.index == bx.index:
                    continue
                r0, r1, s0, s1 = other.ext
                if r0 <= p1 and p0 <= r1 and s0 <= q1 and q0 <= s1:
                    bx.neighbors.append(other.index)
        levels.append(boxes)
    return Hierarchy(dim=dim, n_cells=n_cells, m=m, overlap=overlap, levels=levels)


def parent_local_indices(parent: Box, child: Box) -> np.ndarray:
    """Indices into the parent's local vector of the child's nodes (the restriction R_i)."""
    p0, p1, q0, q1 = child.ext
    P, Q = np.meshgrid(np.arange(p0, p1 + 1), np.arange(q0, q1 + 1), indexing="ij")
    return parent.local_index(P, Q).reshape(-1)


def owned_mask(child: Box) -> np.ndarray:
    """Boolean mask over the child's local nodes: True where P_i keeps the value."""
    p0, p1, q0, q1 = child.ext
    P, Q = np.meshgrid(np.arange(p0, p1 + 1), np.arange(q0, q1 + 1), indexing="ij")
    o = child.own
    m = (P >= o[0]) & (P <= o[1]) & (Q >= o[2]) & (Q <= o[3])
    return m.reshape(-1)

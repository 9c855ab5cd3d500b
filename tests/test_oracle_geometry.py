"""Pins of the oracle's decomposition geometry (Sec. 1 and the Sec. 3 set-up)."""

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import operator as op

CASES = [
    (1, 2001, [(2, 1)], [20]),
    (1, 64, [(2, 1), (2, 1), (2, 1)], [4, 4, 4]),
    (2, 256, [(4, 4)], [4]),
    (2, 64, [(2, 2), (2, 2), (2, 2)], [8, 8, 8]),
    (2, 70, [(3, 2), (2, 3)], [4, 4]),
    (2, 37, [(3, 3)], [4]),
]


@pytest.mark.parametrize("dim,N,m,ov", CASES)
def test_owned_sets_partition_every_parent(dim, N, m, ov):
    # sum_i P_i R_i = I on every parent box (Sec. 1): each parent node owned exactly once
    H = geo.build_hierarchy(dim, N, m, ov)
    for lvl in range(1, H.depth + 1):
        for p, par in enumerate(H.levels[lvl - 1]):
            count = np.zeros(par.n, dtype=np.int64)
            for c in par.children:
                ch = H.levels[lvl][c]
                idx = geo.parent_local_indices(par, ch)
                count[idx[geo.owned_mask(ch)]] += 1
            assert np.all(count == 1)


def test_two_subdomains_overlap_20_cells():
    H = geo.build_hierarchy(1, 2001, [(2, 1)], [20])
    b0, b1 = H.levels[1]
    assert b0.ext == (0, 1010, 0, 0) and b1.ext == (990, 2001, 0, 0)
    assert list(b0.interface) == [1010] and list(b1.interface + b1.ext[0]) == [990]
    assert b0.neighbors == [1] and b1.neighbors == [0]
    assert b0.n_if == 1 and b1.n_if == 1


def test_c2_box_sizes():
    # 4x4 boxes of 64 cells extended by 2 cells: 67 or 69 nodes per side
    H = geo.build_hierarchy(2, 256, [(4, 4)], [4])
    sides = sorted({s for b in H.levels[1] for s in b.shape})
    assert sides == [67, 69]
    ctr = H.levels[1][5]
    assert ctr.n_if == 4 and ctr.interface.size == 4 * 69 - 4
    assert len(ctr.neighbors) == 8


@pytest.mark.parametrize("dim,N,m_h,m_f,ov", [
    (2, 64, [(2, 2), (2, 2), (2, 2)], [(8, 8)], 4),
    (2, 48, [(2, 2), (3, 3)], [(6, 6)], 4),
    (1, 80, [(2, 1), (2, 1), (2, 1)], [(8, 1)], 6),
])
def test_hierarchy_leaves_equal_flat_boxes(dim, N, m_h, m_f, ov):
    # with equal overlap per level the leaves are the flat boxes and the composed
    # ownership is the flat ownership (needed for "one hierarchical DD iteration is
    # one flat DD iteration", Sec. 3.1)
    Hh = geo.build_hierarchy(dim, N, m_h, [ov] * len(m_h))
    Hf = geo.build_hierarchy(dim, N, m_f, [ov])
    flat = {b.gpos: b for b in Hf.levels[1]}
    L = Hh.depth
    for leaf in Hh.levels[L]:
        fb = flat[leaf.gpos]
        assert leaf.ext == fb.ext
        # composed owned set along the ancestors
        b = leaf
        p0, p1, q0, q1 = leaf.ext
        P, Q = np.meshgrid(np.arange(p0, p1 + 1), np.arange(q0, q1 + 1), indexing="ij")
        keep = np.ones(P.shape, dtype=bool)
        lvl = L
        while lvl >= 1:
            o = b.own
            keep &= (P >= o[0]) & (P <= o[1]) & (Q >= o[2]) & (Q <= o[3])
            b = Hh.levels[lvl - 1][b.parent]
            lvl -= 1
        assert np.array_equal(keep.reshape(-1), geo.owned_mask(fb))


@pytest.mark.parametrize("dim,N,m,ov", CASES[:5])
def test_interface_rows_are_where_local_operator_differs(dim, N, m, ov):
    # B_i selects exactly the rows where A~_i differs from the parent operator (Sec. 2)
    H = geo.build_hierarchy(dim, N, m, ov)
    k = np.random.default_rng(0).uniform(3, 9, size=(N + 1) ** dim)
    for lvl in range(1, H.depth + 1):
        for p, par in enumerate(H.levels[lvl - 1]):
            Ap = op.box_matrix(N, k, par.ext, dim).tocsr()
            for c in par.children[:4]:
                ch = H.levels[lvl][c]
                idx = geo.parent_local_indices(par, ch)
                Ai = op.box_matrix(N, k, ch.ext, dim).tocsr()
                sub = Ap[idx][:, idx]
                full_rows = np.asarray(abs(Ap[idx]).sum(axis=1)).ravel()
                sub_rows = np.asarray(abs(sub).sum(axis=1)).ravel()
                diff = np.asarray(abs(Ai - sub).sum(axis=1)).ravel() + (full_rows - sub_rows)
                rows = np.flatnonzero(diff > 1e-9 * abs(Ap).max())
                assert np.array_equal(rows, ch.interface)
            if p > 2:
                break

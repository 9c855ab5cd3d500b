"""Pins of the oracle's ORAS / randomised-SVD coarse space (Secs. 1-2)."""

import numpy as np
import pytest

import workloads as W
from oracle import krylov
from oracle import operator as op
from oracle.schwarz import Coarse, HierarchicalORAS
from helpers import build_all, omegas, rel


def _solver(dim, N, m, ov, k=None, seed=0, **kw):
    n = (N + 1) ** dim
    if k is None:
        k = np.full(n, 10.0)
    elif np.isscalar(k):
        k = np.full(n, float(k))
    return HierarchicalORAS(dim, N, k, m, ov, **kw)


def _one_step(S, f, u0=None):
    u0 = np.zeros_like(f) if u0 is None else u0
    return u0 + S.precondition(f - S.A @ u0)


# ---------------------------------------------------------------- one-step exactness
def test_1d_two_subdomains_rsvd_basis_exact_in_one_step():
    # Sec. 1: with the a-harmonic extension of the two interface values the
    # error space is two-dimensional and the coarse correction makes the method exact.
    N, k = 2001, 20 * np.pi
    S = build_all(_solver(1, N, [(2, 1)], [20], k=k), rank=1, oversample=10)
    f = W.white_rhs(N + 1, 3)[0]
    us = op.direct_solve(S.A, f)
    assert rel(_one_step(S, f), us) < 1e-10
    u0 = W.white_rhs(N + 1, 4)[0]
    e1 = _one_step(S, f, u0) - us
    assert np.linalg.norm(e1) / np.linalg.norm(u0 - us) < 1e-10


def test_1d_explicit_a_harmonic_basis_exact_in_one_step():
    # C = [P_1 U_1, P_2 U_2], U_i the zero-source solutions with unit impedance data
    # at the interface (eqs. (U1)-(U2)).
    N, k = 500, 12.0
    S = _solver(1, N, [(2, 1)], [20], k=k)
    blocks, idx = [], []
    for c, bx in enumerate(S.H.levels[1]):
        e = np.zeros((bx.n, 1), dtype=complex)
        e[bx.interface] = 1.0
        U = np.linalg.solve(S.mats[1][c].toarray(), e)
        blocks.append(U[S.own[1][c]])
        idx.append(S.R[1][c][S.own[1][c]])
    S.set_coarse(0, 0, Coarse(child_ids=[0, 1], own_idx=idx, blocks=blocks))
    f = W.white_rhs(N + 1, 5)[0]
    assert rel(_one_step(S, f), op.direct_solve(S.A, f)) < 1e-10


@pytest.mark.parametrize("levels", [2, 3])
def test_1d_hierarchy_exact_in_one_step(levels):
    # Sec. 1: if the sub-problems are solved exactly, the method on the parent
    # converges in one step; by recursion the hierarchy is exact in one step.
    N, k = 512, 15.0
    S = build_all(_solver(1, N, [(2, 1)] * levels, [8] * levels, k=k), rank=1, oversample=10)
    f = W.white_rhs(N + 1, 6)[0]
    assert rel(_one_step(S, f), op.direct_solve(S.A, f)) < 1e-9


def _install_full_interface(S, lvl):
    """Coarse blocks C_i = P_i S_i(B_i^T I): every interface column (V_i = I)."""
    for p, par in enumerate(S.H.levels[lvl - 1]):
        idx, blocks = [], []
        for c in par.children:
            m_in = S.H.levels[lvl][c].interface.size
            blocks.append(S.extend(lvl, c, np.eye(m_in, dtype=complex)))
            idx.append(S.R[lvl][c][S.own[lvl][c]])
        S.set_coarse(lvl - 1, p, Coarse(child_ids=list(par.children), own_idx=idx, blocks=blocks))
    S.built[lvl] = True


@pytest.mark.parametrize("N,m", [(16, 2), (24, 3), (30, 4)])
def test_2d_untruncated_interface_space_exact_in_one_step(N, m):
    # all interface modes of every subdomain (V_i = I): after the smoother the
    # error is P_i A~_i^{-1} of data on the interfaces, so it lies in span C and one
    # step is exact (the 2D form of the argument of Sec. 1).
    S = _solver(2, N, [(m, m)], [4], k=8.0)
    _install_full_interface(S, 1)
    f = W.smoothed_gaussian_rhs(N, 7)[0]
    u = _one_step(S, f)
    assert np.linalg.norm(f - S.A @ u) / np.linalg.norm(f) < 1e-10


def test_2d_full_rank_sketch_exact_when_interface_map_is_injective():
    # 2x2 boxes: T_i has full column rank, so a full-width sketch spans every
    # interface mode and the randomised basis is as good as V_i = I.
    S = build_all(_solver(2, 16, [(2, 2)], [4], k=8.0), rank=10**6, oversample=0)
    f = W.smoothed_gaussian_rhs(16, 7)[0]
    u = _one_step(S, f)
    assert np.linalg.norm(f - S.A @ u) / np.linalg.norm(f) < 1e-10


def test_2d_hierarchy_untruncated_exact_in_one_step():
    # exact sub-solves by recursion: level-2 full interface spaces make every
    # level-1 sub-solve exact, then the level-1 full spaces make the root exact.
    S = _solver(2, 32, [(2, 2), (2, 2)], [4, 4], k=8.0)
    _install_full_interface(S, 2)
    _install_full_interface(S, 1)
    f = W.smoothed_gaussian_rhs(32, 8)[0]
    u = _one_step(S, f)
    assert np.linalg.norm(f - S.A @ u) / np.linalg.norm(f) < 1e-9


# ---------------------------------------------------------------- hierarchy = flat
@pytest.mark.parametrize("dim,N,mh,mf,ov", [
    (2, 32, [(2, 2), (2, 2)], [(4, 4)], 4),
    (2, 48, [(2, 2), (2, 2), (3, 3)], [(12, 12)], 2),
    (1, 128, [(2, 1)] * 3, [(8, 1)], 6),
])
def test_hierarchical_equals_flat_without_coarse(dim, N, mh, mf, ov):
    # Sec. 3.1: without coarse correction and with one DD iteration per level, one
    # hierarchical DD iteration is exactly one flat DD iteration.
    k = np.random.default_rng(2).uniform(6, 12, (N + 1) ** dim)
    Sh = build_all(_solver(dim, N, mh, [ov] * len(mh), k=k), rank=0, oversample=0)
    Sf = build_all(_solver(dim, N, mf, [ov], k=k), rank=0, oversample=0)
    r = W.white_rhs((N + 1) ** dim, 9)[0]
    assert rel(Sh.precondition(r), Sf.precondition(r)) < 1e-13


# ---------------------------------------------------------------- randomised SVD
def _brute_T(S, lvl, i):
    """Dense T_i = B_i^o A~_i^{-1} B_i^T from explicit matrices (all rows kept)."""
    box = S.H.levels[lvl][i]
    par = S.H.levels[lvl - 1][box.parent]
    Ainv = np.linalg.inv(S.mats[lvl][i].toarray())
    Bi = np.eye(box.n)[box.interface]
    Ri = np.eye(par.n)[S.R[lvl][i]]
    Pi = Ri.T @ np.diag(S.own[lvl][i].astype(float))
    rows = []
    for j in box.neighbors:
        nb = S.H.levels[lvl][j]
        Bj = np.eye(nb.n)[nb.interface]
        Rj = np.eye(par.n)[S.R[lvl][j]]
        rows.append(Bj @ S.mats[lvl][j].toarray() @ Rj @ Pi)
    return np.vstack(rows) @ Ainv @ Bi.T


def test_full_sketch_reproduces_exact_svd():
    S = _solver(2, 24, [(3, 3)], [4], k=9.0)
    i = 4
    T = _brute_T(S, 1, i)
    sv = np.linalg.svd(T, compute_uv=False)
    m_in = S.H.levels[1][i].interface.size
    om = W.omega_block(1, 1, i, m_in, m_in)
    V, sig = S.rsvd_basis(1, i, 10**6, om)
    assert np.allclose(sig, sv[:sig.size], rtol=0, atol=1e-12 * sv[0])
    # truncated to r with a full sketch: same dominant right singular subspace
    r = 12
    assert sv[r - 1] > 1.05 * sv[r]
    Vr, _ = S.rsvd_basis(1, i, 10**6, om)
    Vr = Vr[:, :r]
    _, _, Vh = np.linalg.svd(T)
    Vb = Vh.conj().T[:, :r]
    assert np.linalg.norm(Vr @ Vr.conj().T - Vb @ Vb.conj().T, 2) < 1e-9


def test_full_sketch_at_upper_level_with_exact_subsolves():
    # a level-1 box whose sub-solve is exact (full level-2 interface spaces):
    # the randomised SVD through the hierarchical sub-solver and its adjoint
    # conj(S_i(conj .)) reproduces the SVD of the brute-force T_i.
    S = _solver(2, 32, [(2, 2), (2, 2)], [4, 4], k=8.0)
    _install_full_interface(S, 2)
    i = 0
    T = _brute_T(S, 1, i)
    sv = np.linalg.svd(T, compute_uv=False)
    m_in = S.H.levels[1][i].interface.size
    _, sig = S.rsvd_basis(1, i, 10**6, W.omega_block(3, 1, i, m_in, m_in))
    n = min(sig.size, 20)
    assert np.allclose(sig[:n], sv[:n], rtol=0, atol=1e-9 * sv[0])


@pytest.mark.parametrize("i", [0, 1, 4])
def test_truncated_sketch_within_hmt_bound(i):
    # Halko-Martinsson-Tropp (SIAM Rev. 2011), simplified bound of Sec. 1.5:
    # ||(I - QQ^*) T|| <= [1 + 11 sqrt(k+p) sqrt(min(m,n))] sigma_{k+1}
    # with probability >= 1 - 6 p^-p (p >= 4).
    S = _solver(2, 24, [(3, 3)], [4], k=9.0)
    k_, p = 6, 6
    m_in = S.H.levels[1][i].interface.size
    Q, _ = S.sketch(1, i, W.omega_block(2, 1, i, m_in, k_ + p))
    T = _brute_T(S, 1, i)
    sv = np.linalg.svd(T, compute_uv=False)
    # the oracle drops structurally zero rows; compare on the kept rows
    nz = np.flatnonzero(np.abs(T).sum(axis=1) > 0)
    Tk = T[nz]
    assert Q.shape[0] == Tk.shape[0]
    err = np.linalg.norm(Tk - Q @ (Q.conj().T @ Tk), 2)
    bound = (1 + 11 * np.sqrt(k_ + p) * np.sqrt(min(T.shape))) * sv[k_]
    assert err <= bound
    assert err >= sv[k_ + p] * (1 - 1e-10)  # no rank-(k+p) projection beats the SVD


def test_adjoint_dot_product_identity():
    S = _solver(2, 24, [(3, 3)], [4], k=9.0)
    rng = np.random.default_rng(3)
    for i in (0, 4, 7):
        box = S.H.levels[1][i]
        x = rng.standard_normal((box.interface.size, 2)) + 1j * rng.standard_normal((box.interface.size, 2))
        Tx, parts = S.apply_T(1, i, x)
        y = rng.standard_normal(Tx.shape) + 1j * rng.standard_normal(Tx.shape)
        Tsy = S.apply_T_adjoint(1, i, y, parts)
        lhs = np.vdot(y, Tx)
        rhs = np.vdot(Tsy, x)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _c2_like():
    S = _solver(2, 48, [(3, 3)], [4], k=12.0)
    return build_all(S, rank=4, oversample=6)


def test_galerkin_orthogonality():
    S = _c2_like()
    cs = S.coarse[0][0]
    r = W.white_rhs(S.A.shape[0], 11)[0]
    u = S.precondition(r)
    C = cs.dense(S.A.shape[0])
    g = C.conj().T @ (r - S.A @ u)
    assert np.linalg.norm(g) <= 1e-11 * np.linalg.norm(C.conj().T @ r)


def test_coarse_correction_depends_only_on_span():
    S = _c2_like()
    r = W.white_rhs(S.A.shape[0], 12)[0]
    u1 = S.precondition(r)
    cs = S.coarse[0][0]
    rng = np.random.default_rng(4)
    blocks = []
    for b in cs.blocks:
        Wm = rng.standard_normal((b.shape[1],) * 2) + 1j * rng.standard_normal((b.shape[1],) * 2)
        blocks.append(b @ Wm)
    S.set_coarse(0, 0, Coarse(child_ids=cs.child_ids, own_idx=cs.own_idx, blocks=blocks))
    assert rel(S.precondition(r), u1) < 1e-11


def test_fixed_point_is_discrete_solution():
    S = _c2_like()
    f = W.smoothed_gaussian_rhs(48, 13)[0]
    u, info = krylov.stationary(lambda x: S.A @ x, S.precondition, f, tol=1e-10, maxit=60)
    assert info.converged
    assert rel(u, op.direct_solve(S.A, f)) < 1e-8


def test_mixed_precision_leaves_converge_to_fp64_solution():
    S = _solver(2, 48, [(3, 3)], [4], k=12.0, leaf_dtype=np.complex64)
    build_all(S, rank=4, oversample=6)
    f = W.smoothed_gaussian_rhs(48, 14)[0]
    u, info = krylov.fgmres(lambda x: S.A @ x, S.precondition, f, tol=1e-8, maxit=100)
    assert info.converged
    assert rel(u, op.direct_solve(S.A, f)) < 1e-7


def test_build_order_enforced():
    S = _solver(2, 32, [(2, 2), (2, 2)], [4, 4], k=8.0)
    with pytest.raises(RuntimeError):
        S.build_coarse(1, 2, 2, omegas(S, 1, 2, 2))


def test_negligible_modes_are_dropped_and_the_step_stays_exact():
    # rank above the interface size with a thin overlap: some interface modes extend to
    # (numerically) nothing on the owned nodes; they are left out of C (A_c stays
    # invertible) and the full interface space still makes one step exact (Sec. 2).
    N = 24
    S = _solver(2, N, [(2, 2)], [2], k=5.0)
    oms = []
    for i in range(4):
        m_in, _, s = S.sizes(1, i, 10**6, 10)
        oms.append(W.omega_block(0, 1, i, m_in, s))
    S.build_coarse(1, 10**6, 10, oms)
    cs = S.coarse[0][0]
    full = sum(S.sizes(1, i, 10**6, 10)[1] for i in range(4))
    assert 0 < cs.size < full
    assert np.linalg.cond(cs.Ac) < 1e12
    f = W.white_rhs((N + 1) ** 2, 15)[0]
    u = S.precondition(f)
    assert np.linalg.norm(f - S.A @ u) / np.linalg.norm(f) < 1e-10

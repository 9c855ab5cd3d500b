"""Pins of the oracle's operator (discretisation of eq. (lap1) and of Sec. 3.1)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operator as op


def _rand_k(n, seed, lo=5.0, hi=15.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


@pytest.mark.parametrize("dim,N", [(1, 17), (2, 9)])
def test_complex_symmetric(dim, N):
    k = _rand_k((N + 1) ** dim, 1)
    A = op.global_matrix(N, k, dim)
    assert abs(A - A.T).max() == 0.0
    box = (2, N - 3, 0, 0) if dim == 1 else (1, N - 2, 3, N)
    Ab = op.box_matrix(N, k, box, dim)
    assert abs(Ab - Ab.T).max() == 0.0


def test_stencil_values_2d_constant_k():
    # Interior 4/h^2 - k^2, off-diagonals -1/h^2; edge 2/h^2 - k^2/2 - ik/h with
    # -1/(2h^2) along the edge and -1/h^2 inward; corner 1/h^2 - k^2/4 - ik/h with
    # -1/(2h^2) to both neighbours.
    N, kk = 8, 7.0
    h = 1.0 / N
    A = op.global_matrix(N, np.full((N + 1) ** 2, kk), 2).toarray()
    n = N + 1

    def g(p, q):
        return p * n + q

    i = g(4, 3)
    assert np.isclose(A[i, i], 4 / h**2 - kk**2)
    for j in (g(3, 3), g(5, 3), g(4, 2), g(4, 4)):
        assert np.isclose(A[i, j], -1 / h**2)
    assert np.count_nonzero(A[i]) == 5
    e = g(0, 4)  # left edge
    assert np.isclose(A[e, e], 2 / h**2 - kk**2 / 2 - 1j * kk / h)
    assert np.isclose(A[e, g(0, 3)], -0.5 / h**2) and np.isclose(A[e, g(0, 5)], -0.5 / h**2)
    assert np.isclose(A[e, g(1, 4)], -1 / h**2)
    c = g(N, N)  # corner
    assert np.isclose(A[c, c], 1 / h**2 - kk**2 / 4 - 1j * kk / h)
    assert np.isclose(A[c, g(N - 1, N)], -0.5 / h**2) and np.isclose(A[c, g(N, N - 1)], -0.5 / h**2)
    assert np.count_nonzero(A[c]) == 3


def test_stencil_values_1d():
    N, kk = 10, 3.0
    h = 1.0 / N
    A = op.global_matrix(N, np.full(N + 1, kk), 1).toarray()
    assert np.isclose(A[4, 4], 2 / h**2 - kk**2)
    assert np.isclose(A[4, 3], -1 / h**2) and np.isclose(A[4, 5], -1 / h**2)
    for e in (0, N):
        assert np.isclose(A[e, e], 1 / h**2 - kk**2 / 2 - 1j * kk / h)
    assert np.isclose(A[0, 1], -1 / h**2)


def _pieces_1d(n_nodes, h):
    """1D stiffness K, lumped mass weights M (1/2 at the ends), end selector E."""
    K = np.zeros((n_nodes, n_nodes))
    for a in range(n_nodes - 1):
        K[a, a] += 1 / h**2
        K[a + 1, a + 1] += 1 / h**2
        K[a, a + 1] -= 1 / h**2
        K[a + 1, a] -= 1 / h**2
    M = np.ones(n_nodes)
    M[0] = M[-1] = 0.5
    E = np.zeros(n_nodes)
    E[0] = E[-1] = 1.0
    return K, np.diag(M), np.diag(E)


@pytest.mark.parametrize("box", [(0, 7, 0, 7), (2, 6, 1, 7), (0, 3, 4, 7)])
def test_kronecker_form_2d(box):
    # With heterogeneous k the cell-assembled 2D matrix equals
    #   K (x) M + M (x) K - diag(k^2) (M (x) M) - (i/h) diag(k) (E (x) M + M (x) E)
    # built from independent 1D pieces on the box.
    N = 7
    h = 1.0 / N
    k = _rand_k((N + 1) ** 2, 3)
    nx, ny = box[1] - box[0] + 1, box[3] - box[2] + 1
    Kx, Mx, Ex = _pieces_1d(nx, h)
    Ky, My, Ey = _pieces_1d(ny, h)
    kb = k[op.box_global_indices(box, N, 2)]
    ref = (np.kron(Kx, My) + np.kron(Mx, Ky) - np.diag(kb**2) @ np.kron(Mx, My)
           - 1j / h * np.diag(kb) @ (np.kron(Ex, My) + np.kron(Mx, Ey)))
    A = op.box_matrix(N, k, box, 2).toarray()
    assert np.allclose(A, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def _closed_form_1d(N, k, f):
    """Discrete solution for constant f with the lumped RHS (ends f/2), g = 0.

    u_j = -f/k^2 + a (mu^j + mu^(N-j)), mu = exp(i theta), cos theta = 1 - (kh)^2/2,
    a = (f/k) / [ (sin theta / h)(1 - mu^N) + k (1 + mu^N) ].
    """
    h = 1.0 / N
    theta = np.arccos(1 - (k * h) ** 2 / 2)
    mu = np.exp(1j * theta)
    a = (f / k) / ((np.sin(theta) / h) * (1 - mu**N) + k * (1 + mu**N))
    j = np.arange(N + 1)
    return -f / k**2 + a * (mu**j + mu ** (N - j))


def test_closed_form_1d():
    N, k, fval = 2001, 20 * np.pi, 1.0
    A = op.global_matrix(N, np.full(N + 1, k), 1)
    b = np.full(N + 1, fval, dtype=complex)
    b[0] = b[-1] = fval / 2
    u = op.direct_solve(A, b)
    ref = _closed_form_1d(N, k, fval)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-10


def test_second_order_convergence_1d():
    # the continuous solution (f/k^2)(-1 + e^{ikx}/2 + e^{ik(1-x)}/2) of eq. (lap1)
    k, fval = 4 * np.pi, 1.0
    errs = []
    for N in (200, 400, 800):
        A = op.global_matrix(N, np.full(N + 1, k), 1)
        b = np.full(N + 1, fval, dtype=complex)
        b[0] = b[-1] = fval / 2
        u = op.direct_solve(A, b)
        x = np.linspace(0, 1, N + 1)
        ue = (fval / k**2) * (-1 + 0.5 * np.exp(1j * k * x) + 0.5 * np.exp(1j * k * (1 - x)))
        errs.append(np.abs(u - ue).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4


def test_impedance_data_1d_plane_wave():
    # f = 0 and impedance data of the discrete plane wave mu^j: the solve returns mu^j.
    N, k = 50, 9.0
    h = 1.0 / N
    theta = np.arccos(1 - (k * h) ** 2 / 2)
    mu = np.exp(1j * theta)
    g = np.zeros(N + 1, dtype=complex)
    g[0] = -1j * (np.sin(theta) / h + k)
    g[N] = 1j * mu**N * (np.sin(theta) / h - k)
    A = op.global_matrix(N, np.full(N + 1, k), 1)
    b = op.rhs_vector(N, np.zeros(N + 1), g, 1)
    u = op.direct_solve(A, b)
    assert np.allclose(u, mu ** np.arange(N + 1), atol=1e-10)


def test_impedance_data_2d_plane_wave():
    # 2D wave mu^p independent of q: on x-sides the 1D data, on y-sides -ik u,
    # at corners the mean of the two (each side carries one boundary edge).
    N, k = 20, 6.0
    h = 1.0 / N
    theta = np.arccos(1 - (k * h) ** 2 / 2)
    mu = np.exp(1j * theta)
    n = N + 1
    P, Q = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v = mu ** P
    gx = np.zeros((n, n), dtype=complex)
    gx[0, :] = -1j * (np.sin(theta) / h + k)
    gx[N, :] = 1j * mu**N * (np.sin(theta) / h - k)
    gy = np.zeros((n, n), dtype=complex)
    gy[:, 0] = -1j * k * v[:, 0]
    gy[:, N] = -1j * k * v[:, N]
    on_x = (P == 0) | (P == N)
    on_y = (Q == 0) | (Q == N)
    g = np.where(on_x & on_y, 0.5 * (gx + gy), gx + gy)
    A = op.global_matrix(N, np.full(n * n, k), 2)
    b = op.rhs_vector(N, np.zeros(n * n), g.reshape(-1), 2)
    u = op.direct_solve(A, b)
    assert np.allclose(u, v.reshape(-1), atol=1e-9)


@pytest.mark.parametrize("dim,N", [(1, 300), (2, 40)])
def test_manufactured_solution(dim, N):
    # the set-up of Sec. 3.1: a random discrete u, f = A u, the solve returns u
    rng = np.random.default_rng(5)
    n = (N + 1) ** dim
    k = _rand_k(n, 7, 10, 30)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = op.global_matrix(N, k, dim)
    x = op.direct_solve(A, A @ u)
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-10
    assert sp.issparse(A)

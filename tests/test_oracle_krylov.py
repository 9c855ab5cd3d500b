"""Pins of the oracle's outer loops (stationary iteration and restarted FGMRES)."""

import numpy as np
import pytest

import workloads as W
from oracle import krylov
from oracle import operator as op
from oracle.schwarz import HierarchicalORAS
from helpers import build_all, rel


def _small():
    N = 12
    S = HierarchicalORAS(2, N, np.full((N + 1) ** 2, 9.0), [(2, 2)], [4])
    build_all(S, rank=2, oversample=3)
    f = W.smoothed_gaussian_rhs(N, 21)[0]
    return S, f


def test_gmres_iterate_minimises_residual_over_krylov_space():
    # GMRES (right preconditioning): u_k = B y_k with y_k minimising ||f - A B y||
    # over K_k(A B, f); compare with a brute-force least-squares solve on an
    # explicitly built, orthonormalised Krylov basis.
    S, f = _small()
    AB = lambda x: S.A @ S.precondition(x)
    for kk in range(1, 7):
        u, info = krylov.fgmres(lambda x: S.A @ x, S.precondition, f, tol=0.0, maxit=kk, restart=50)
        K = [f]
        for _ in range(kk - 1):
            K.append(AB(K[-1]))
        Qk, _ = np.linalg.qr(np.stack(K, axis=1))
        M = np.stack([AB(Qk[:, t]) for t in range(kk)], axis=1)
        c, *_ = np.linalg.lstsq(M, f, rcond=None)
        best = np.linalg.norm(f - M @ c)
        got = np.linalg.norm(f - S.A @ u)
        assert info.iters == kk
        assert abs(got - best) <= 1e-9 * np.linalg.norm(f)


def test_residual_history_non_increasing_within_cycle():
    S, f = _small()
    _, info = krylov.fgmres(lambda x: S.A @ x, S.precondition, f, tol=1e-12, maxit=30, restart=30)
    h = np.array(info.history)
    assert np.all(np.diff(h) <= 1e-14)


def test_full_restart_exact_in_n_steps():
    N = 7
    A = op.global_matrix(N, np.full(N + 1, 5.0), 1)
    f = W.white_rhs(N + 1, 22)[0]
    u, info = krylov.fgmres(lambda x: A @ x, lambda x: x, f, tol=1e-13, maxit=N + 1, restart=N + 1)
    assert info.converged and info.iters <= N + 1
    assert rel(u, op.direct_solve(A, f)) < 1e-10


def test_restarted_gmres_converges_and_reports_true_residual():
    S, f = _small()
    u, info = krylov.fgmres(lambda x: S.A @ x, S.precondition, f, tol=1e-10, maxit=200, restart=3)
    assert info.converged
    assert np.isclose(info.rel_residual, np.linalg.norm(f - S.A @ u) / np.linalg.norm(f), rtol=1e-6)
    assert info.rel_residual < 1e-10


@pytest.mark.parametrize("solver", ["stationary", "fgmres"])
def test_zero_rhs_gives_zero_in_zero_iterations(solver):
    S, f = _small()
    fn = getattr(krylov, solver)
    u, info = fn(lambda x: S.A @ x, S.precondition, np.zeros_like(f), tol=1e-8, maxit=10)
    assert info.iters == 0 and info.converged and np.all(u == 0)


def test_stationary_maxit_reports_not_converged():
    S, f = _small()
    u, info = krylov.stationary(lambda x: S.A @ x, S.precondition, f, tol=1e-30, maxit=2)
    assert info.iters == 2 and not info.converged

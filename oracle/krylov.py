"""Outer loops around the ORAS preconditioner B.

TEST INFRASTRUCTURE ONLY (see the package header).

* Stationary: u_0 = 0, u_{t+1} = u_t + B(f - A u_t) (eqs. (sub1)-(coarse1) of
  Sec. 1 in Richardson form), stopped when ||f - A u||_2 / ||f||_2 < tol.
* Right-preconditioned restarted GMRES on A B y = f, u = B y (Sec. 3 uses
  GMRES on the Schwarz-preconditioned system, zero initial guess, relative
  residual stopping).  Written in the flexible form that keeps Z_j = B v_j, so
  that it also serves a preconditioner that is not exactly linear (complex64
  sub-solves); for a linear B it is GMRES.  Orthogonalisation by classical
  Gram-Schmidt applied twice; the small least-squares problem by Givens
  rotations.  The true residual is recomputed at every restart and at exit.

Pins (tests/test_oracle_krylov.py): on small problems the k-th GMRES iterate
minimises ||f - A B y|| over the Krylov space K_k(A B, f) built by brute
force; residual norms never increase inside a cycle; a restart length of n
reaches the exact solution in n steps.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveInfo:
    iters: int = 0
    rel_residual: float = np.inf
    converged: bool = False
    history: list = field(default_factory=list)  # relative residual after each iteration


def _norm(x):
    return float(np.sqrt(np.sum(np.abs(x) ** 2)))


def stationary(apply_A, apply_B, f, tol=1e-8, maxit=100, u0=None):
    f = np.asarray(f, dtype=np.complex128)
    nf = _norm(f)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.complex128)
    info = SolveInfo()
    if nf == 0.0:
        info.rel_residual = 0.0
        info.converged = True
        return np.zeros_like(f), info
    r = f - apply_A(u)
    rel = _norm(r) / nf
    while True:
        if rel < tol:
            info.converged = True
            break
        if info.iters >= maxit:
            break
        u = u + apply_B(r)
        info.iters += 1
        r = f - apply_A(u)
        rel = _norm(r) / nf
        info.history.append(rel)
    info.rel_residual = rel
    return u, info


def fgmres(apply_A, apply_B, f, tol=1e-8, maxit=500, restart=50):
    """Right-preconditioned restarted (F)GMRES from u = 0."""
    f = np.asarray(f, dtype=np.complex128)
    n = f.shape[0]
    nf = _norm(f)
    u = np.zeros_like(f)
    info = SolveInfo()
    if nf == 0.0:
        info.rel_residual = 0.0
        info.converged = True
        return u, info
    r = f.copy()
    beta = nf
    while True:
        if beta / nf < tol:
            info.converged = True
            break
        if info.iters >= maxit:
            break
        m = min(restart, maxit - info.iters)
        V = np.zeros((n, m + 1), dtype=np.complex128)
        Z = np.zeros((n, m), dtype=np.complex128)
        Hh = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            Z[:, j] = apply_B(V[:, j])
            w = apply_A(Z[:, j])
            # classical Gram-Schmidt, twice
            h1 = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h1
            h2 = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h2
            Hh[:j + 1, j] = h1 + h2
            Hh[j + 1, j] = _norm(w)
            if Hh[j + 1, j] != 0.0:
                V[:, j + 1] = w / Hh[j + 1, j]
            # apply the previous rotations to the new column
            for t in range(j):
                a, b = Hh[t, j], Hh[t + 1, j]
                Hh[t, j] = np.conj(cs[t]) * a + np.conj(sn[t]) * b
                Hh[t + 1, j] = -sn[t] * a + cs[t] * b
            # new rotation zeroing H[j+1, j]
            a, b = Hh[j, j], Hh[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = a / den, b / den
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            info.iters += 1
            j_done = j + 1
            info.history.append(abs(g[j + 1]) / nf)
            if abs(g[j + 1]) / nf < tol:
                break
        y = np.linalg.solve(np.triu(Hh[:j_done, :j_done]), g[:j_done])
        u = u + Z[:, :j_done] @ y
        r = f - apply_A(u)
        beta = _norm(r)
    info.rel_residual = beta / nf
    return u, info

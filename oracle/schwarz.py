"""Two-level and hierarchical ORAS with the randomised-SVD coarse basis.

TEST INFRASTRUCTURE ONLY (see the package header).

What is computed, in the paper's order:

* one ORAS smoothing step, eq. (sub1) of Sec. 1, read in Richardson form
  u~ = u + sum_i P_i A~_i^{-1} R_i (f - A u)  (the literal form drops the
  leading u; both agree for the first step from u = 0);
* the coarse correction, eq. (coarse1): u = u~ + C A_c^{-1} C^H (f - A u~),
  A_c = C^H A C the Galerkin matrix on the range of C;
* the interface map of Sec. 2 in its algebraic form:
  T_i = B_i^o A~_i^{-1} B_i^T with B_ij = B_j A~_j R_j P_i stacked over the
  neighbours j (structurally zero rows left out), and the coarse vectors
  C_i = P_i A~_i^{-1} B_i^T V_i, V_i the dominant right singular vectors of T_i;
* the randomised SVD of Sec. 2 (apply T_i to a few random samples,
  orthogonalise, apply the adjoint T_i^*, then a small SVD), with
  r_i + p samples (Sec. 3 uses n_c + 5);
* the hierarchy of Sec. 1 and Sec. 2: a non-leaf subdomain problem is solved
  by n_i steps of the same two-level method on that subdomain (Sec. 3,
  "number of Schwarz iterations" n_il), from a zero initial guess; its coarse
  basis is built with those inexact solves and therefore carries iterative
  error (Sec. 2, the paragraph after the remarks).

Readings where the paper is silent:

* r_i = min(rank_per_interface * n_if(i), m_in), s_i = min(r_i + p, m_in);
* the adjoint at a non-leaf level is conj(S_i(conj(.))), the same forward
  sub-solver; at a leaf it is the exact solve with A~_i^H;
* QR is Householder (LAPACK), the small SVD is LAPACK's, the Galerkin matrix is
  factored by LU with partial pivoting;
* mixed precision: the leaf factorisations and leaf solves run in complex64;
  everything else (residuals, QR, SVD, A_c, outer vectors) in complex128.

Pins (tests/test_oracle_schwarz.py): one-step exactness in 1D with two
subdomains and the a-harmonic basis (Sec. 1); the same for the 1D hierarchy
with exact sub-solves; one-step exactness in 2D with the untruncated interface
space; hierarchical = flat for one iteration without coarse modes (Sec. 3.1,
the remark on Tab. 2); full-width sketch = exact SVD of a brute-force T_i; the
HMT error bound for truncated sketches; the adjoint dot-product identity;
Galerkin orthogonality; invariance of the correction under C -> C W.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import Box, Hierarchy, build_hierarchy, owned_mask, parent_local_indices
from .operator import box_matrix, global_matrix


# A coarse mode of box i whose extension P_i S_i(B_i^T v) has a norm on the owned
# nodes of at most NEGLIGIBLE times the largest of the box's modes is not used: it
# adds a (numerically) zero column to C and makes A_c singular.
NEGLIGIBLE = 1e-10


@dataclass
class Coarse:
    """Coarse space of one parent problem: blocks C_i on the owned nodes of each child."""
    child_ids: list[int]
    own_idx: list[np.ndarray]      # indices into the parent's local vector
    blocks: list[np.ndarray]       # C_i restricted to its owned nodes, (n_own_i, r_i)
    Ac: np.ndarray | None = None
    lu: tuple | None = None
    V: list[np.ndarray] = field(default_factory=list)
    sigma: list[np.ndarray] = field(default_factory=list)

    @property
    def size(self) -> int:
        return int(sum(b.shape[1] for b in self.blocks))

    def dense(self, n_parent: int) -> sp.csc_matrix:
        """C as a sparse n_parent x n_c matrix (C = (C_i), Sec. 2)."""
        rows, cols, vals = [], [], []
        off = 0
        for idx, blk in zip(self.own_idx, self.blocks):
            r = blk.shape[1]
            rr, cc = np.meshgrid(idx, np.arange(off, off + r), indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(blk.ravel())
            off += r
        if off == 0:
            return sp.csc_matrix((n_parent, 0), dtype=np.complex128)
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n_parent, off))


class HierarchicalORAS:
    """The hierarchical two-level ORAS preconditioner of a problem on the unit interval/square.

    Parameters follow Sec. 3: ``m`` = [m_1, ..., m_L] splits per level, ``overlap``
    = delta/h per level, ``inner_iters`` = n_il for the non-leaf levels 1..L-1.
    """

    def __init__(self, dim, n_cells, k_nodes, m, overlap, inner_iters=None, leaf_dtype=np.complex128):
        self.dim = dim
        self.n_cells = n_cells
        self.k = np.asarray(k_nodes, dtype=np.float64)
        self.H: Hierarchy = build_hierarchy(dim, n_cells, m, overlap)
        L = self.H.depth
        # n_il for the non-leaf levels l = 1..L-1 (Sec. 3); default one iteration
        self.inner_iters = [1] * (L + 1)
        for lvl, v in enumerate(inner_iters or [], start=1):
            self.inner_iters[lvl] = int(v)
        self.leaf_dtype = np.dtype(leaf_dtype)
        self.A = global_matrix(n_cells, self.k, dim)
        # local operators A~_i of every box below the root
        self.mats: list[list[sp.csr_matrix]] = [[self.A]]
        for lvl in range(1, L + 1):
            self.mats.append([box_matrix(n_cells, self.k, b.ext, dim) for b in self.H.levels[lvl]])
        # exact leaf factorisations (SuperLU, partial pivoting)
        self.leaf_lu = [spla.splu(sp.csc_matrix(Ai, dtype=self.leaf_dtype)) for Ai in self.mats[L]]
        # restriction maps R_i (child nodes inside the parent's local vector) and owned masks
        self.R: list[list[np.ndarray]] = [[]]
        self.own: list[list[np.ndarray]] = [[]]
        for lvl in range(1, L + 1):
            self.R.append([parent_local_indices(self.H.levels[lvl - 1][b.parent], b) for b in self.H.levels[lvl]])
            self.own.append([owned_mask(b) for b in self.H.levels[lvl]])
        # coarse spaces of the parent problems at each level 0..L-1 (None = no coarse space)
        self.coarse: list[list[Coarse | None]] = [[None] * len(self.H.levels[lvl]) for lvl in range(L)]
        self.built = [False] * (L + 1)

    # ------------------------------------------------------------------ local solves
    def local_solve(self, lvl: int, i: int, b: np.ndarray) -> np.ndarray:
        """S_i(b): exact solve at a leaf, n_i two-level steps from zero otherwise (Sec. 1, Sec. 3)."""
        b = np.asarray(b, dtype=np.complex128)
        if lvl == self.H.depth:
            x = self.leaf_lu[i].solve(b.astype(self.leaf_dtype))
            return np.asarray(x, dtype=np.complex128)
        A = self.mats[lvl][i]
        u = np.zeros_like(b)
        for _ in range(self.inner_iters[lvl]):
            u = u + self.apply_B(lvl, i, b - A @ u)
        return u

    def local_solve_adjoint(self, lvl: int, i: int, b: np.ndarray) -> np.ndarray:
        """Adjoint sub-solve: exact A~_i^{-H} at a leaf; conj(S_i(conj b)) above (a reading)."""
        b = np.asarray(b, dtype=np.complex128)
        if lvl == self.H.depth:
            x = self.leaf_lu[i].solve(b.astype(self.leaf_dtype), trans="H")
            return np.asarray(x, dtype=np.complex128)
        return np.conj(self.local_solve(lvl, i, np.conj(b)))

    # ------------------------------------------------------------------ one two-level step
    def smoother(self, lvl: int, p: int, r: np.ndarray) -> np.ndarray:
        """sum_i P_i S_i(R_i r) over the children i of parent p at level lvl (eq. (sub1))."""
        par = self.H.levels[lvl][p]
        out = np.zeros_like(r, dtype=np.complex128)
        for c in par.children:
            x = self.local_solve(lvl + 1, c, r[self.R[lvl + 1][c]])
            idx = self.R[lvl + 1][c][self.own[lvl + 1][c]]
            out[idx] = x[self.own[lvl + 1][c]]
        return out

    def coarse_correct(self, lvl: int, p: int, r: np.ndarray, u: np.ndarray) -> np.ndarray:
        """u + C A_c^{-1} C^H (r - A u) for the parent problem p (eq. (coarse1))."""
        cs = self.coarse[lvl][p]
        if cs is None or cs.size == 0:
            return u
        A = self.mats[lvl][p]
        res = r - A @ u
        c = np.concatenate([blk.conj().T @ res[idx] for idx, blk in zip(cs.own_idx, cs.blocks)], axis=0)
        y = sla.lu_solve(cs.lu, c)
        out = u.copy()
        off = 0
        for idx, blk in zip(cs.own_idx, cs.blocks):
            rr = blk.shape[1]
            out[idx] += blk @ y[off:off + rr]
            off += rr
        return out

    def apply_B(self, lvl: int, p: int, r: np.ndarray) -> np.ndarray:
        """One two-level ORAS step on residual r from zero: B_p(r) (eqs. (sub1)-(coarse1))."""
        u = self.smoother(lvl, p, r)
        return self.coarse_correct(lvl, p, r, u)

    def precondition(self, r: np.ndarray) -> np.ndarray:
        """B(r) of the whole problem (root, level 0)."""
        return self.apply_B(0, 0, r)

    # ------------------------------------------------------------------ interface map
    def trace_to_neighbors(self, lvl: int, i: int, X: np.ndarray):
        """Y = B_i^o-applied data: stacked (A~_j R_j P_i X)[B_j] over neighbours j, zero rows dropped.

        Returns (Y, parts) with parts = [(j, kept interface rows of j)] in stacking order.
        """
        box = self.H.levels[lvl][i]
        par = self.H.levels[lvl - 1][box.parent]
        G = np.zeros((par.n, X.shape[1]), dtype=np.complex128)
        own = self.own[lvl][i]
        G[self.R[lvl][i][own]] = X[own]
        ownvec = np.zeros(par.n)
        ownvec[self.R[lvl][i][own]] = 1.0
        blocks, parts = [], []
        for j in box.neighbors:
            nb = self.H.levels[lvl][j]
            Aj = self.mats[lvl][j]
            AjB = Aj[nb.interface]
            struct = (abs(AjB) @ ownvec[self.R[lvl][j]]) > 0
            rows = nb.interface[struct]
            if rows.size == 0:
                continue
            blocks.append((Aj @ G[self.R[lvl][j]])[rows])
            parts.append((j, rows))
        if not blocks:
            return np.zeros((0, X.shape[1]), dtype=np.complex128), parts
        return np.concatenate(blocks, axis=0), parts

    def trace_adjoint(self, lvl: int, i: int, Q: np.ndarray, parts) -> np.ndarray:
        """H = sum_j P_i^T R_j^T A~_j^H B_j^T Q_j, on the nodes of box i."""
        box = self.H.levels[lvl][i]
        par = self.H.levels[lvl - 1][box.parent]
        Hp = np.zeros((par.n, Q.shape[1]), dtype=np.complex128)
        off = 0
        for j, rows in parts:
            nb = self.H.levels[lvl][j]
            Z = np.zeros((nb.n, Q.shape[1]), dtype=np.complex128)
            Z[rows] = Q[off:off + rows.size]
            off += rows.size
            Hp[self.R[lvl][j]] += self.mats[lvl][j].conj().T @ Z
        Hi = Hp[self.R[lvl][i]]
        Hi[~self.own[lvl][i]] = 0.0
        return Hi

    def apply_T(self, lvl: int, i: int, g: np.ndarray):
        """T_i g = B_i^o S_i(B_i^T g) (Sec. 2, algebraic form)."""
        box = self.H.levels[lvl][i]
        rhs = np.zeros((box.n, g.shape[1]), dtype=np.complex128)
        rhs[box.interface] = g
        X = self.local_solve(lvl, i, rhs)
        return self.trace_to_neighbors(lvl, i, X)

    def apply_T_adjoint(self, lvl: int, i: int, y: np.ndarray, parts) -> np.ndarray:
        """T_i^* y = B_i S_i^*((B_i^o)^H y)."""
        box = self.H.levels[lvl][i]
        H = self.trace_adjoint(lvl, i, y, parts)
        W = self.local_solve_adjoint(lvl, i, H)
        return W[box.interface]

    def sizes(self, lvl: int, i: int, rank: int, oversample: int) -> tuple[int, int, int]:
        box = self.H.levels[lvl][i]
        m_in = int(box.interface.size)
        r = min(rank * box.n_if, m_in)
        s = min(r + oversample, m_in) if r > 0 else 0
        return m_in, r, s

    # ------------------------------------------------------------------ randomised SVD
    def sketch(self, lvl: int, i: int, omega: np.ndarray):
        """Orthonormal basis Q of the sampled range T_i Omega_i (Sec. 2: apply T_i to random
        samples, then orthogonalise).  ``omega`` has shape (s_i, m_in)."""
        Om = np.asarray(omega, dtype=np.complex128).T          # m_in x s
        Y, parts = self.apply_T(lvl, i, Om)                    # sample the range of T_i
        Q, _ = np.linalg.qr(Y, mode="reduced")                 # orthogonalise (Householder)
        return Q, parts

    def rsvd_basis(self, lvl: int, i: int, rank: int, omega: np.ndarray):
        """V_i by the randomised SVD of T_i (Sec. 2): sketch, orthogonalise, adjoint, small SVD.

        ``omega`` has shape (s_i, m_in): row t is the t-th Gaussian sample.
        Returns (V_i of shape (m_in, r_i), singular values of the sketch).
        """
        box = self.H.levels[lvl][i]
        m_in = box.interface.size
        r = min(rank * box.n_if, m_in)
        if r == 0:
            return np.zeros((m_in, 0), dtype=np.complex128), np.zeros(0)
        Q, parts = self.sketch(lvl, i, omega)
        Bh = self.apply_T_adjoint(lvl, i, Q, parts)            # B^H = T_i^* Q, m_in x s
        _, sig, Vh = np.linalg.svd(Bh.conj().T, full_matrices=False)  # SVD of B = Q^H T_i
        V = Vh.conj().T[:, :r]
        return V, sig

    def extend(self, lvl: int, i: int, V: np.ndarray) -> np.ndarray:
        """C_i = P_i S_i(B_i^T V_i) on the owned nodes of box i (Sec. 2)."""
        box = self.H.levels[lvl][i]
        rhs = np.zeros((box.n, V.shape[1]), dtype=np.complex128)
        rhs[box.interface] = V
        X = self.local_solve(lvl, i, rhs)
        return X[self.own[lvl][i]]

    def build_coarse(self, lvl: int, rank: int, oversample: int, omegas) -> None:
        """Coarse spaces of every parent at level lvl-1 from the boxes of level lvl.

        Must run bottom-up (level L first): sub-solves at level lvl use the coarse
        spaces of level lvl+1.  ``omegas[i]`` is the (s_i, m_in) Gaussian block of box i.
        """
        L = self.H.depth
        if not (1 <= lvl <= L):
            raise ValueError("level out of range")
        if lvl < L and not self.built[lvl + 1]:
            raise RuntimeError("build_coarse must run from the finest level up")
        for p, par in enumerate(self.H.levels[lvl - 1]):
            own_idx, blocks, Vs, sigs = [], [], [], []
            for c in par.children:
                if rank > 0:
                    V, sig = self.rsvd_basis(lvl, c, rank, omegas[c])
                else:
                    V, sig = np.zeros((self.H.levels[lvl][c].interface.size, 0), dtype=np.complex128), np.zeros(0)
                Ci = self.extend(lvl, c, V) if V.shape[1] else np.zeros((int(self.own[lvl][c].sum()), 0), np.complex128)
                if Ci.shape[1]:
                    norms = np.linalg.norm(Ci, axis=0)
                    keep = norms > NEGLIGIBLE * norms.max()
                    Ci, V = Ci[:, keep], V[:, keep]
                own_idx.append(self.R[lvl][c][self.own[lvl][c]])
                blocks.append(Ci)
                Vs.append(V)
                sigs.append(sig)
            cs = Coarse(child_ids=list(par.children), own_idx=own_idx, blocks=blocks, V=Vs, sigma=sigs)
            self.set_coarse(lvl - 1, p, cs)
        self.built[lvl] = True

    def set_coarse(self, lvl: int, p: int, cs: Coarse) -> None:
        """Install coarse blocks for parent p and form A_c = C^H A C with its LU (eq. (coarse1))."""
        if cs.size == 0:
            self.coarse[lvl][p] = cs
            return
        A = self.mats[lvl][p]
        C = cs.dense(A.shape[0])
        cs.Ac = np.asarray((C.conj().T @ (A @ C)).todense())
        cs.lu = sla.lu_factor(cs.Ac)
        self.coarse[lvl][p] = cs


def make_solver(cfg: dict, k_nodes, leaf_dtype=np.complex128, inner_iters=None) -> HierarchicalORAS:
    """Solver for a workload dict (dim, n_cells, m, overlap)."""
    return HierarchicalORAS(cfg["dim"], cfg["n_cells"], k_nodes, cfg["m"], cfg["overlap"],
                            inner_iters=inner_iters, leaf_dtype=leaf_dtype)

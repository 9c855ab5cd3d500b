"""Small helpers shared by the tests (input plumbing only, no solver arithmetic)."""

import numpy as np

import workloads as W


def omegas(S, lvl, rank, oversample, seed=0):
    """Gaussian test blocks for every box of level lvl, sized by the oracle's geometry."""
    out = []
    for i in range(len(S.H.levels[lvl])):
        m_in, _, s = S.sizes(lvl, i, rank, oversample)
        out.append(W.omega_block(seed, lvl, i, m_in, s))
    return out


def build_all(S, rank, oversample, seed=0):
    """build_coarse for every level, finest first."""
    for lvl in range(S.H.depth, 0, -1):
        S.build_coarse(lvl, rank, oversample, omegas(S, lvl, rank, oversample, seed))
    return S


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))

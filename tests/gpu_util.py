"""Helpers of the GPU parity tests: inputs for the library and the oracle from the same generators."""

import numpy as np
import torch

import workloads as W


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_omega(H, ctx, level, rank, oversample, seed=0):
    """The level's Gaussian blocks sized by the library's own geometry, concatenated.

    Block i is the generator's (s_i, m_in) array flattened row by row, i.e. the
    m_in x s_i column-major layout the library expects.
    """
    m_in, _, s = H.hh_level_info(ctx, level, rank, oversample)
    parts = [W.omega_block(seed, level, i, int(m_in[i]), int(s[i])).reshape(-1) for i in range(len(m_in))]
    flat = np.concatenate(parts) if parts else np.zeros(0, np.complex128)
    return (dev(flat) if flat.size else None), m_in, s


def oracle_omegas(S, level, rank, oversample, seed=0):
    out = []
    for i in range(len(S.H.levels[level])):
        m_in, _, s = S.sizes(level, i, rank, oversample)
        out.append(W.omega_block(seed, level, i, m_in, s))
    return out


def build_both(H, ctx, S, rank, oversample, seed=0):
    """build_coarse on every level, finest first, with the same Gaussian blocks on both sides."""
    for lvl in range(S.H.depth, 0, -1):
        om, m_in, s = gpu_omega(H, ctx, lvl, rank, oversample, seed)
        oms = oracle_omegas(S, lvl, rank, oversample, seed)
        assert [o.shape[1] for o in oms] == list(m_in), "interface sizes differ between library and oracle"
        assert [o.shape[0] for o in oms] == list(s), "sketch widths differ between library and oracle"
        H.hh_build_coarse(ctx, lvl, rank, oversample, om)
        S.build_coarse(lvl, rank, oversample, oms)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))

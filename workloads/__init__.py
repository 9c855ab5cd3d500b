"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and shapes them into the input fields of
the workloads (right-hand sides, wavenumber fields, the Gaussian test blocks of
the randomised SVD).  It holds none of the solver's arithmetic: no operator, no
decomposition rule, no solve.  Sizes that depend on the decomposition (the
interface dimension of a subdomain, its sketch width) are passed in by the
caller.

Every generator takes an explicit integer seed and uses NumPy's PCG64, so the
same call gives the same array on any machine.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "complex_gaussian",
    "box_filter5",
    "smoothed_gaussian_rhs",
    "white_rhs",
    "gaussian_random_field",
    "wavenumber_grf",
    "omega_block",
    "batch_problems",
    "WORKLOADS",
]


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(list(int(k) for k in key)))


def complex_gaussian(shape, seed: int, *stream: int) -> np.ndarray:
    """Standard complex Gaussian CN(0,1): real and imaginary parts i.i.d. N(0, 1/2)."""
    g = _rng(seed, *stream)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def box_filter5(w: np.ndarray) -> np.ndarray:
    """5x5 moving mean with zero padding, same output size, divided by 25."""
    n0, n1 = w.shape
    pad = np.zeros((n0 + 4, n1 + 4), dtype=w.dtype)
    pad[2:-2, 2:-2] = w
    out = np.zeros_like(w)
    for a in range(5):
        for b in range(5):
            out += pad[a:a + n0, b:b + n1]
    return out / 25.0


def white_rhs(n_nodes: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """nrhs i.i.d. CN(0,1) vectors of length n_nodes, shape (nrhs, n_nodes)."""
    return complex_gaussian((nrhs, n_nodes), seed, 1)


def smoothed_gaussian_rhs(n_cells: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """CN(0,1) on the (N+1)^2 node grid, smoothed by the 5x5 box filter.

    Returns shape (nrhs, (N+1)^2), node (p, q) at p*(N+1)+q.
    """
    n = n_cells + 1
    out = np.empty((nrhs, n * n), dtype=np.complex128)
    for j in range(nrhs):
        w = complex_gaussian((n, n), seed, 2, j)
        out[j] = box_filter5(w).reshape(-1)
    return out


def gaussian_random_field(n_cells: int, corr_len: float, seed: int) -> np.ndarray:
    """Zero-mean, unit-variance stationary field on the (N+1)^2 nodes.

    Covariance exp(-|x-y|^2 / (2 l^2)), sampled by circulant embedding on a
    periodic grid of 2(N+1) points per side (spectral square root of the
    embedded covariance, negative eigenvalues clipped to zero), then rescaled to
    unit sample variance.
    """
    n = n_cells + 1
    h = 1.0 / n_cells
    m = 2 * n
    d = np.minimum(np.arange(m), m - np.arange(m)) * h
    cov = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * corr_len ** 2))
    lam = np.fft.fft2(cov).real
    lam = np.maximum(lam, 0.0)
    g = _rng(seed, 3)
    z = g.standard_normal((m, m)) + 1j * g.standard_normal((m, m))
    field = np.fft.fft2(np.sqrt(lam / (m * m)) * z).real[:n, :n]
    field = field - field.mean()
    field = field / field.std()
    return field.reshape(-1)


def wavenumber_grf(n_cells: int, k0: float, amp: float, corr_len: float, seed: int) -> np.ndarray:
    """k(x) = k0 (1 + amp * clip(s(x), -1, 1)) on the nodes, s a unit Gaussian field."""
    s = gaussian_random_field(n_cells, corr_len, seed)
    return k0 * (1.0 + amp * np.clip(s, -1.0, 1.0))


def omega_block(seed: int, level: int, box: int, m_in: int, s: int) -> np.ndarray:
    """Gaussian test block of the randomised SVD for one subdomain.

    Shape (s, m_in): row t is the t-th sample vector on the subdomain's
    interface nodes (entries CN(0,1)).  Seeded per (seed, level, box).
    """
    return complex_gaussian((s, m_in), seed, 4, level, box)


# Workload definitions (sizes and seeds of the synthetic problems).
def batch_problems(count: int, seed: int):
    """The mixed batch of independent 2D problems: per problem a grid side drawn
    uniformly from {64, 96, 128, 192, 256}, k = side / 6.4 (about 40 points per
    wavelength) and an m x m split with m uniform in {2, 3, 4}.  Returns a list of
    (side, k, m)."""
    g = _rng(seed, 7)
    sides = g.choice(np.array([64, 96, 128, 192, 256]), size=count)
    ms = g.integers(2, 5, size=count)
    return [(int(s), float(s) / 6.4, int(m)) for s, m in zip(sides, ms)]


WORKLOADS = {
    # 1D, k = 20*pi, 2000 interior + 2 boundary nodes, two subdomains
    # overlapping by 20 cells, one interface mode per subdomain.
    "helm1d_n2001_k20pi": dict(dim=1, n_cells=2001, k=20.0 * np.pi, m=[(2, 1)],
                               overlap=[20], rank=1, oversample=10, rhs="white"),
    # 2D free space, 256 cells per side, k = 40, 4x4 subdomains, 4-cell overlap,
    # rank 8 per interface + 10 oversampling, smoothed Gaussian RHS.
    "helm2d_n256_k40_4x4": dict(dim=2, n_cells=256, k=40.0, m=[(4, 4)], overlap=[4],
                                rank=8, oversample=10, rhs="smooth"),
    # 2D hierarchical, 1024 cells per side, heterogeneous k, [2x2, 2x2, 2x2].
    "helm2d_n1024_grf_3lvl": dict(dim=2, n_cells=1024, k=160.0, k_amp=0.3, k_corr=0.1,
                                  m=[(2, 2), (2, 2), (2, 2)], overlap=[8, 8, 8],
                                  rank=16, oversample=10, rhs="smooth"),
    # 512 independent problems (batch_problems), 4-cell overlap, rank 8 per
    # interface + 10, white Gaussian RHS, complex64 local solves.
    "helm2d_batch512": dict(dim=2, count=512, overlap=[4], rank=8, oversample=10, rhs="white"),
}


# ---------------------------------------------------------------- counter-based Gaussian blocks
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC 2011) on arrays of counters.

    ctr: uint32 array (..., 4); key: two uint32 words.  Returns uint32 (..., 4).
    """
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(_PHILOX_M[0]) * c[0]
        p1 = np.uint64(_PHILOX_M[1]) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & mask, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & mask]
        k0 = (k0 + np.uint64(_PHILOX_W[0])) & mask
        k1 = (k1 + np.uint64(_PHILOX_W[1])) & mask
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def omega_philox(seed: int, level: int, box: int, m_in: int, s: int) -> np.ndarray:
    """Gaussian test block drawn from a seed with Philox4x32-10: shape (s, m_in), CN(0,1).

    Entry v = t*m_in + j uses counter (v, box, level, 0x4f4d4547) and key
    (seed low, seed high); two 53-bit uniforms in (0, 1) per entry and the
    Box-Muller transform give the real and imaginary parts (each / sqrt(2)).
    """
    n = m_in * s
    v = np.arange(n, dtype=np.uint64)
    ctr = np.stack([v & np.uint64(0xFFFFFFFF), np.full(n, box, np.uint64), np.full(n, level, np.uint64),
                    np.full(n, 0x4F4D4547, np.uint64)], axis=-1).astype(np.uint32)
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).astype(np.uint64)

    def unit(hi, lo):
        return (((hi << np.uint64(32)) | lo) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0) + \
            0.5 / 9007199254740992.0

    u1, u2 = unit(w[:, 0], w[:, 1]), unit(w[:, 2], w[:, 3])
    r = np.sqrt(-2.0 * np.log(u1)) / np.sqrt(2.0)
    out = r * np.cos(2.0 * np.pi * u2) + 1j * (r * np.sin(2.0 * np.pi * u2))
    return out.reshape(s, m_in)

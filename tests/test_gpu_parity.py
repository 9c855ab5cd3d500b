"""GPU parity: the HIP library through its C ABI against the FP64 oracle on the same inputs.

Tolerances: relative 1e-10 on solutions and preconditioner outputs of the FP64
path (the gate of the FP64 path); 1e-13 on single stencil applications; the
mixed path converges to a residual of 1e-8 and must then lie within 1e-7 of
the oracle's solution.
"""

import numpy as np
import pytest

import workloads as W
from oracle import krylov
from oracle import operator as op
from oracle.schwarz import HierarchicalORAS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_12538_amd as lib

    return lib


# ---------------------------------------------------------------- operator
@pytest.mark.parametrize("dim,N,nrhs", [(2, 37, 3), (1, 301, 2), (2, 256, 1)])
def test_stencil_matches_assembled_matrix(hh, dim, N, nrhs):
    from gpu_util import dev, host, rel

    n = (N + 1) ** dim
    k = np.random.default_rng(1).uniform(5, 25, n)
    ctx = hh.hh_setup(dim, N, k, hh.decomposition([(2, 2)], [4]))
    try:
        x = W.white_rhs(n, 2, nrhs)
        b = W.white_rhs(n, 3, nrhs)
        A = op.global_matrix(N, k, dim)
        y = dev(np.zeros_like(x))
        hh.hh_apply_operator(ctx, dev(x), y)
        ref = (A @ x.T).T
        assert rel(host(y), ref) < 1e-13
        hh.hh_apply_operator(ctx, dev(x), y, dev(b))
        assert rel(host(y), b - ref) < 1e-13
    finally:
        hh.hh_destroy(ctx)


# ---------------------------------------------------------------- local solves, no coarse space
@pytest.mark.parametrize("dim,N,m,ov", [
    (2, 48, [(3, 3)], [4]),
    (2, 70, [(3, 2)], [6]),
    (1, 400, [(4, 1)], [10]),
    (2, 64, [(2, 2), (2, 2)], [4, 4]),
])
def test_smoother_without_coarse_matches_oracle(hh, dim, N, m, ov):
    from gpu_util import build_both, dev, host, rel

    n = (N + 1) ** dim
    k = np.random.default_rng(4).uniform(8, 14, n)
    ctx = hh.hh_setup(dim, N, k, hh.decomposition(m, ov))
    S = HierarchicalORAS(dim, N, k, m, ov)
    try:
        build_both(hh, ctx, S, rank=0, oversample=0)
        r = W.white_rhs(n, 5, 2)
        z = dev(np.zeros_like(r))
        hh.hh_precondition(ctx, dev(r), z)
        ref = np.stack([S.precondition(r[i]) for i in range(2)])
        assert rel(host(z), ref) < 1e-11
    finally:
        hh.hh_destroy(ctx)


# ---------------------------------------------------------------- leaf sweep shapes
# Leaf widths b = ny in every shape bucket of the sweep kernel (<= 8, 16, 40,
# 72, 144, 256), boxes of two and three grid lines (the two-ended sweep with
# an empty bottom half), zero overlap, and batches whose column count leaves
# a ragged last chunk for every column-block width (1, 2 and 4 per group).
@pytest.mark.parametrize("dim,N,m,ov,nrhs", [
    (2, 8, [(8, 8)], [0], 3),      # 1-cell boxes: nx = ny = 2
    (2, 12, [(6, 6)], [0], 2),     # nx = ny = 3
    (2, 16, [(8, 8)], [2], 2),     # nx, ny in {4, 5}
    (2, 30, [(3, 3)], [2], 2),     # b <= 16
    (2, 60, [(2, 2)], [6], 2),     # b <= 40
    (2, 100, [(2, 1)], [4], 2),    # b = 101
    (2, 180, [(3, 1)], [4], 1),    # b = 181
    (2, 200, [(4, 4)], [4], 9),    # b <= 72, 32 half-box units: 2 columns per group, ragged
    (2, 200, [(4, 4)], [4], 33),   # 4 columns per group, ragged
])
def test_leaf_sweep_shapes_match_oracle(hh, dim, N, m, ov, nrhs):
    from gpu_util import build_both, dev, host, rel

    n = (N + 1) ** dim
    k = np.random.default_rng(7).uniform(6, 12, n)
    ctx = hh.hh_setup(dim, N, k, hh.decomposition(m, ov))
    S = HierarchicalORAS(dim, N, k, m, ov)
    try:
        build_both(hh, ctx, S, rank=0, oversample=0)
        r = W.white_rhs(n, 8, nrhs)
        z = dev(np.zeros_like(r))
        hh.hh_precondition(ctx, dev(r), z)
        ref = np.stack([S.precondition(r[i]) for i in range(nrhs)])
        assert rel(host(z), ref) < 1e-11
    finally:
        hh.hh_destroy(ctx)


# ---------------------------------------------------------------- 1D, two subdomains, exact basis
def test_1d_two_subdomains_one_step_exact(hh):
    from gpu_util import build_both, dev, host, rel

    N, k = 2001, 20 * np.pi
    ctx = hh.hh_setup(1, N, k, hh.decomposition([(2, 1)], [20]), outer=hh.HH_STATIONARY)
    S = HierarchicalORAS(1, N, np.full(N + 1, k), [(2, 1)], [20])
    try:
        build_both(hh, ctx, S, rank=1, oversample=10)
        f = W.white_rhs(N + 1, 11)
        u = dev(np.zeros_like(f))
        info = hh.hh_solve(ctx, dev(f), u, rtol=1e-8, maxit=5)
        us = op.direct_solve(S.A, f[0])
        assert info[0][0] == 1 and info[0][1]
        assert rel(host(u)[0], us) < 1e-10
    finally:
        hh.hh_destroy(ctx)


# ---------------------------------------------------------------- rSVD coarse space, one level
def _case_2d(hh, N, m, k, rank, p, outer=None, precision=None):
    n = (N + 1) ** 2
    kk = np.full(n, float(k)) if np.isscalar(k) else k
    kw = {}
    if outer is not None:
        kw["outer"] = outer
    if precision is not None:
        kw["precision"] = precision
    ctx = hh.hh_setup(2, N, kk, hh.decomposition(m, [4] * len(m)), **kw)
    S = HierarchicalORAS(2, N, kk, m, [4] * len(m), leaf_dtype=np.complex128)
    return ctx, S


def test_rsvd_singular_values_and_preconditioner_match(hh):
    from gpu_util import build_both, dev, host, rel

    ctx, S = _case_2d(hh, 48, [(3, 3)], 12.0, 4, 6)
    try:
        build_both(hh, ctx, S, rank=4, oversample=6)
        # singular values of the sketched B are invariant under the QR's phases
        cs = S.coarse[0][0]
        nsig = sum(sg.size for sg in cs.sigma)
        Ac, sig = hh.hh_get_coarse(ctx, 0, 0, nsig)
        ref = np.concatenate(cs.sigma)
        assert np.allclose(sig, ref, rtol=1e-9, atol=1e-12 * ref.max())
        assert Ac.shape == cs.Ac.shape
        # the coarse correction depends on span(C) only: compare B(r)
        r = W.white_rhs(S.A.shape[0], 12, 2)
        z = dev(np.zeros_like(r))
        hh.hh_precondition(ctx, dev(r), z)
        ref = np.stack([S.precondition(r[i]) for i in range(2)])
        assert rel(host(z), ref) < 1e-10
        # spectrum of A_c (invariant under C -> C W for unitary W)
        sv_gpu = np.linalg.svd(Ac, compute_uv=False)
        sv_orc = np.linalg.svd(cs.Ac, compute_uv=False)
        assert np.allclose(sv_gpu, sv_orc, rtol=1e-8)
    finally:
        hh.hh_destroy(ctx)


def test_full_size_2d_gmres_matches_oracle(hh):
    """N = 256, k = 40, 4x4 boxes, 4-cell overlap, rank 8 per interface + 10, smoothed RHS."""
    from gpu_util import build_both, dev, host, rel

    N = 256
    ctx, S = _case_2d(hh, N, [(4, 4)], 40.0, 8, 10, outer=hh.HH_GMRES)
    try:
        build_both(hh, ctx, S, rank=8, oversample=10)
        f = W.smoothed_gaussian_rhs(N, 1)
        uo, info_o = krylov.fgmres(lambda x: S.A @ x, S.precondition, f[0], tol=1e-8, maxit=200)
        assert info_o.converged
        # same iteration count on both sides: solutions within 1e-10
        u = dev(np.zeros_like(f))
        hh.hh_solve(ctx, dev(f), u, rtol=0.0, maxit=info_o.iters)
        assert rel(host(u)[0], uo) < 1e-10
        # the library's own stopping test
        info = hh.hh_solve(ctx, dev(f), u, rtol=1e-8, maxit=200)
        assert info[0][1] and info[0][2] < 1e-8
        assert abs(info[0][0] - info_o.iters) <= 1
        us = op.direct_solve(S.A, f[0])
        assert rel(host(u)[0], us) < 1e-7
    finally:
        hh.hh_destroy(ctx)


@pytest.mark.parametrize("full_reorth", [False, True])
def test_gram_schmidt_variants_match_oracle(hh, full_reorth):
    from gpu_util import build_both, dev, host, rel

    N = 96
    kk = np.full((N + 1) ** 2, 15.0)
    ctx = hh.hh_setup(2, N, kk, hh.decomposition([(4, 4)], [4]), full_reorth=full_reorth)
    S = HierarchicalORAS(2, N, kk, [(4, 4)], [4])
    try:
        build_both(hh, ctx, S, rank=4, oversample=6)
        f = W.smoothed_gaussian_rhs(N, 41, 2)
        u = dev(np.zeros_like(f))
        info = hh.hh_solve(ctx, dev(f), u, rtol=1e-10, maxit=200)
        assert all(i[1] for i in info)
        for b in range(2):
            uo, io = krylov.fgmres(lambda x: S.A @ x, S.precondition, f[b], tol=1e-10, maxit=200)
            assert abs(info[b][0] - io.iters) <= 1
            assert rel(host(u)[b], uo) < 1e-9
    finally:
        hh.hh_destroy(ctx)


def test_batch_invariance(hh):
    from gpu_util import build_both, dev, host

    ctx, S = _case_2d(hh, 48, [(3, 3)], 12.0, 4, 6)
    try:
        build_both(hh, ctx, S, rank=4, oversample=6)
        f = W.smoothed_gaussian_rhs(48, 21, 3)
        u3 = dev(np.zeros_like(f))
        info3 = hh.hh_solve(ctx, dev(f), u3, rtol=1e-8, maxit=100)
        alone = []
        for i in range(3):
            ui = dev(np.zeros_like(f[i:i + 1]))
            info1 = hh.hh_solve(ctx, dev(f[i:i + 1]), ui, rtol=1e-8, maxit=100)
            assert info1[0][0] == info3[i][0]
            alone.append(host(ui)[0])
        assert np.array_equal(host(u3), np.stack(alone))
    finally:
        hh.hh_destroy(ctx)


def test_columns_identical_across_coarse_kernel_paths(hh):
    """A column's bits do not depend on the batch width where the width picks
    another coarse restriction/prolongation kernel (vector FMA chains for up to
    four right-hand sides, matrix cores for more): 20 columns solved together,
    the first two alone and the first six alone."""
    from gpu_util import build_both, dev, host

    ctx, S = _case_2d(hh, 48, [(3, 3)], 12.0, 4, 6)
    try:
        build_both(hh, ctx, S, rank=4, oversample=6)
        f = W.smoothed_gaussian_rhs(48, 23, 20)
        u20 = dev(np.zeros_like(f))
        info20 = hh.hh_solve(ctx, dev(f), u20, rtol=1e-8, maxit=100)
        for w in (2, 6):
            uw = dev(np.zeros_like(f[:w]))
            infow = hh.hh_solve(ctx, dev(f[:w]), uw, rtol=1e-8, maxit=100)
            assert [i[0] for i in infow] == [i[0] for i in info20[:w]]
            assert np.array_equal(host(uw), host(u20)[:w])
    finally:
        hh.hh_destroy(ctx)


def test_hierarchy_two_levels_matches_oracle(hh):
    from gpu_util import build_both, dev, host, rel

    N = 64
    k = np.random.default_rng(6).uniform(10, 16, (N + 1) ** 2)
    ctx = hh.hh_setup(2, N, k, hh.decomposition([(2, 2), (2, 2)], [4, 4]))
    S = HierarchicalORAS(2, N, k, [(2, 2), (2, 2)], [4, 4])
    try:
        build_both(hh, ctx, S, rank=3, oversample=5)
        r = W.white_rhs((N + 1) ** 2, 13, 2)
        z = dev(np.zeros_like(r))
        hh.hh_precondition(ctx, dev(r), z)
        ref = np.stack([S.precondition(r[i]) for i in range(2)])
        assert rel(host(z), ref) < 1e-10
    finally:
        hh.hh_destroy(ctx)


def test_mixed_precision_converges_to_fp64_solution(hh):
    from gpu_util import build_both, dev, host, rel

    ctx, S = _case_2d(hh, 64, [(4, 4)], 10.0, 4, 6, precision=hh.HH_MIXED)
    try:
        build_both(hh, ctx, S, rank=4, oversample=6)
        f = W.smoothed_gaussian_rhs(64, 31)
        u = dev(np.zeros_like(f))
        info = hh.hh_solve(ctx, dev(f), u, rtol=1e-8, maxit=200)
        assert info[0][1]
        uo, io = krylov.fgmres(lambda x: S.A @ x, S.precondition, f[0], tol=1e-8, maxit=200)
        assert rel(host(u)[0], uo) < 1e-7
    finally:
        hh.hh_destroy(ctx)


# ---------------------------------------------------------------- API behaviour
def test_solve_before_build_is_a_state_error(hh):
    import torch

    ctx = hh.hh_setup(2, 32, 8.0, hh.decomposition([(2, 2)], [4]))
    try:
        f = torch.zeros((1, 33 * 33), dtype=torch.complex128, device="cuda")
        with pytest.raises(hh.HelmddError) as e:
            hh.hh_solve(ctx, f, torch.zeros_like(f), 1e-8, 10)
        assert e.value.status == 6
    finally:
        hh.hh_destroy(ctx)


def test_zero_rhs_returns_zero(hh):
    import torch

    ctx = hh.hh_setup(2, 32, 8.0, hh.decomposition([(2, 2)], [4]))
    try:
        hh.hh_build_coarse(ctx, 1, 0, 0, None)
        f = torch.zeros((2, 33 * 33), dtype=torch.complex128, device="cuda")
        u = torch.ones_like(f)
        info = hh.hh_solve(ctx, f, u, 1e-8, 10)
        assert all(i[0] == 0 and i[1] for i in info)
        assert torch.count_nonzero(u).item() == 0
    finally:
        hh.hh_destroy(ctx)


def test_invalid_arguments_rejected(hh):
    with pytest.raises(hh.HelmddError) as e:
        hh.hh_setup(2, 32, 8.0, hh.decomposition([(2, 2)], [3]))  # odd overlap
    assert e.value.status == 1
    with pytest.raises(hh.HelmddError):
        hh.hh_setup(2, 32, float("nan"), hh.decomposition([(2, 2)], [4]))


# ---------------------------------------------------------------- cached device memory
def test_recreated_context_reuses_cached_memory_with_identical_results(hh):
    """Contexts take their buffers from the library's device cache; a context
    built on recycled blocks (stale contents) must give the same bits."""
    from gpu_util import build_both, dev, host

    N, m, ov = 40, [(2, 2)], [4]
    k = np.full((N + 1) ** 2, 9.0)
    f = W.smoothed_gaussian_rhs(N, 31, 2)
    outs = []
    for _ in range(2):
        ctx = hh.hh_setup(2, N, k, hh.decomposition(m, ov))
        S = HierarchicalORAS(2, N, k, m, ov)
        try:
            build_both(hh, ctx, S, rank=3, oversample=4)
            u = dev(np.zeros_like(f))
            hh.hh_solve(ctx, dev(f), u, rtol=1e-9, maxit=80)
            outs.append(host(u))
        finally:
            hh.hh_destroy(ctx)
    assert np.array_equal(outs[0], outs[1])
    assert hh.hh_release_cached_memory() > 0
    assert hh.hh_release_cached_memory() == 0


# ---------------------------------------------------------------- limits and degenerate cases
def test_widest_supported_leaf_and_the_limit(hh):
    """Leaves 256 nodes wide (the largest sweep shape) match the oracle; 257 is refused."""
    from gpu_util import build_both, dev, host, rel

    N = 255
    n = (N + 1) ** 2
    k = np.random.default_rng(9).uniform(10, 14, n)
    ctx = hh.hh_setup(2, N, k, hh.decomposition([(2, 1)], [4]))
    S = HierarchicalORAS(2, N, k, [(2, 1)], [4])
    try:
        build_both(hh, ctx, S, rank=0, oversample=0)
        r = W.white_rhs(n, 14, 2)
        z = dev(np.zeros_like(r))
        hh.hh_precondition(ctx, dev(r), z)
        ref = np.stack([S.precondition(r[i]) for i in range(2)])
        assert rel(host(z), ref) < 1e-11
    finally:
        hh.hh_destroy(ctx)
    with pytest.raises(hh.HelmddError) as e:
        hh.hh_setup(2, 256, 12.0, hh.decomposition([(2, 1)], [4]))
    assert e.value.status == hh.HH_EUNSUPPORTED
    assert "wider than 256" in str(e.value)  # the set-up's message outlives its context


def test_full_interface_space_is_exact_in_one_step(hh):
    """Rank above the interface size: r_i = m_in, the coarse space spans every
    interface mode and one stationary step solves the problem (Sec. 2)."""
    from gpu_util import build_both, dev, host, rel

    N = 24
    n = (N + 1) ** 2
    k = np.full(n, 5.0)
    ctx = hh.hh_setup(2, N, k, hh.decomposition([(2, 2)], [2]), outer=hh.HH_STATIONARY)
    S = HierarchicalORAS(2, N, k, [(2, 2)], [2])
    try:
        m_in, r, s = hh.hh_level_info(ctx, 1, 1000, 10)
        assert list(r) == list(m_in) and list(s) == list(m_in)
        build_both(hh, ctx, S, rank=1000, oversample=10)
        # some modes extend to nothing on the owned nodes and are dropped on both sides
        assert S.coarse[0][0].size < int(np.sum(r))
        f = W.white_rhs(n, 15)
        z = dev(np.zeros_like(f))
        hh.hh_precondition(ctx, dev(f), z)
        assert rel(host(z)[0], S.precondition(f[0])) < 1e-9
        u = dev(np.zeros_like(f))
        info = hh.hh_solve(ctx, dev(f), u, rtol=0.0, maxit=1)
        assert info[0][0] == 1
        us = op.direct_solve(S.A, f[0])
        assert rel(host(u)[0], us) < 1e-9
    finally:
        hh.hh_destroy(ctx)

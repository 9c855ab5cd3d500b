"""Independent problems in one context (hh_setup_batch): every level of every
problem goes into the same launches; each problem's result must be the one it
gets alone (bit for bit: per-problem arithmetic does not depend on the batch)
and must match the FP64 oracle (1e-10 at equal iteration counts for the FP64
path; the mixed path converges to 1e-8 and lies within 1e-7 of the oracle).
"""

import numpy as np
import pytest

import workloads as W
from oracle import krylov
from oracle.schwarz import HierarchicalORAS

pytestmark = pytest.mark.gpu

# (N, k, splits, overlaps): uneven sizes and box counts, one level
ONE_LEVEL = [(40, 6.25, [(2, 2)], [4]), (48, 7.5, [(3, 3)], [4]), (64, 10.0, [(4, 4)], [4]),
             (57, 8.9, [(2, 3)], [4])]
# leaf widths in four sweep shape buckets (<= 16, 40, 72, 144)
BUCKETS = [(24, 5.0, [(2, 2)], [2]), (60, 9.0, [(2, 2)], [6]), (100, 12.0, [(2, 2)], [4]),
           (200, 20.0, [(2, 2)], [4])]
TWO_LEVEL = [(64, 10.0, [(2, 2), (2, 2)], [4, 4]), (48, 7.5, [(3, 3), (1, 2)], [4, 4])]
RANK, OVERS = 3, 4


@pytest.fixture(scope="module")
def hh():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_12538_amd as lib

    return lib


def _omega(hh, ctx, level, seeds, box_prob):
    """Gaussian blocks of a (batch) level: box i of problem p uses seed p and its index within p."""
    m_in, _, s = hh.hh_level_info(ctx, level, RANK, OVERS)
    local = {}
    parts = []
    for i in range(len(m_in)):
        p = box_prob[i]
        j = local.get(p, 0)
        local[p] = j + 1
        parts.append(W.omega_block(seeds[p], level, j, int(m_in[i]), int(s[i])).reshape(-1))
    from gpu_util import dev

    return dev(np.concatenate(parts))


def _box_prob(problems, level):
    out = []
    for p, (_, _, m, _) in enumerate(problems):
        nb = 1
        for l in range(level):
            nb *= m[l][0] * m[l][1]
        out += [p] * nb
    return out


def _setup(hh, problems, precision=None, build=True, seeds=None):
    kw = {} if precision is None else {"precision": precision}
    ctx = hh.hh_setup_batch(2, [(N, k, hh.decomposition(m, ov)) for N, k, m, ov in problems], **kw)
    seeds = seeds or list(range(len(problems)))
    if build:
        depth = len(problems[0][2])
        for lvl in range(depth, 0, -1):
            hh.hh_build_coarse(ctx, lvl, RANK, OVERS, _omega(hh, ctx, lvl, seeds, _box_prob(problems, lvl)))
    return ctx


def _rhs(problems, nrhs, seed0=100):
    return [W.white_rhs((N + 1) ** 2, seed0 + p, nrhs) for p, (N, _, _, _) in enumerate(problems)]


def _oracle(problems, p):
    N, k, m, ov = problems[p]
    S = HierarchicalORAS(2, N, np.full((N + 1) ** 2, k), m, ov)
    for lvl in range(len(m), 0, -1):
        oms = []
        for i in range(len(S.H.levels[lvl])):
            mi, _, s = S.sizes(lvl, i, RANK, OVERS)
            oms.append(W.omega_block(p, lvl, i, mi, s))
        S.build_coarse(lvl, RANK, OVERS, oms)
    return S


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_each_problem_alone(hh, precision):
    from gpu_util import dev, host

    prec = hh.HH_MIXED if precision == "mixed" else hh.HH_FP64
    probs = ONE_LEVEL
    fs = _rhs(probs, 2)
    ctx = _setup(hh, probs, prec)
    try:
        f = ctx.pack([dev(x) for x in fs])
        u = f.new_zeros(f.shape)
        info = hh.hh_solve(ctx, f, u, rtol=1e-8, maxit=300)
        ub = [host(x) for x in ctx.unpack(u, 2)]
    finally:
        hh.hh_destroy(ctx)
    assert all(i[1] for i in info)
    for p in range(len(probs)):
        solo = _setup(hh, [probs[p]], prec, seeds=[p])
        try:
            us = dev(np.zeros_like(fs[p]))
            inf1 = hh.hh_solve(solo, dev(fs[p]), us, rtol=1e-8, maxit=300)
            assert [i[0] for i in inf1] == [i[0] for i in info[2 * p: 2 * p + 2]]
            assert np.array_equal(host(us), ub[p])
        finally:
            hh.hh_destroy(solo)


def test_batch_matches_oracle_at_equal_iterations(hh):
    from gpu_util import dev, host, rel

    probs = ONE_LEVEL
    fs = _rhs(probs, 1, 200)
    M = 12
    ctx = _setup(hh, probs)
    try:
        f = ctx.pack([dev(x) for x in fs])
        u = f.new_zeros(f.shape)
        info = hh.hh_solve(ctx, f, u, rtol=0.0, maxit=M)
        ub = [host(x) for x in ctx.unpack(u, 1)]
    finally:
        hh.hh_destroy(ctx)
    assert all(i[0] == M for i in info)
    for p in range(len(probs)):
        S = _oracle(probs, p)
        uo, io = krylov.fgmres(lambda x: S.A @ x, S.precondition, fs[p][0], tol=0.0, maxit=M)
        assert io.iters == M
        assert rel(ub[p][0], uo) < 1e-10


def test_batch_mixed_precision_within_1e7_of_oracle(hh):
    from gpu_util import dev, host, rel

    probs = ONE_LEVEL[:3]
    fs = _rhs(probs, 1, 300)
    ctx = _setup(hh, probs, hh.HH_MIXED)
    try:
        f = ctx.pack([dev(x) for x in fs])
        u = f.new_zeros(f.shape)
        info = hh.hh_solve(ctx, f, u, rtol=1e-8, maxit=300)
        ub = [host(x) for x in ctx.unpack(u, 1)]
    finally:
        hh.hh_destroy(ctx)
    assert all(i[1] and i[2] < 1e-8 for i in info)
    for p in range(len(probs)):
        S = _oracle(probs, p)
        uo, io = krylov.fgmres(lambda x: S.A @ x, S.precondition, fs[p][0], tol=1e-8, maxit=300)
        assert io.converged
        assert rel(ub[p][0], uo) < 1e-7


@pytest.mark.parametrize("problems", [BUCKETS, TWO_LEVEL], ids=["buckets", "two_level"])
def test_batch_preconditioner_matches_oracle(hh, problems):
    from gpu_util import dev, host, rel

    rs = _rhs(problems, 2, 400)
    ctx = _setup(hh, problems)
    try:
        r = ctx.pack([dev(x) for x in rs])
        z = r.new_zeros(r.shape)
        hh.hh_precondition(ctx, r, z)
        zb = [host(x) for x in ctx.unpack(z, 2)]
    finally:
        hh.hh_destroy(ctx)
    for p in range(len(problems)):
        S = _oracle(problems, p)
        ref = np.stack([S.precondition(rs[p][i]) for i in range(2)])
        assert rel(zb[p], ref) < 1e-10


def test_batch_layout_and_errors(hh):
    probs = ONE_LEVEL[:2]
    ctx = _setup(hh, probs, build=False)
    try:
        assert ctx.nprob == 2 and ctx.n == sum((N + 1) ** 2 for N, _, _, _ in probs)
        with pytest.raises(hh.HelmddError):  # coarse spaces not built
            import torch

            f = torch.zeros((1, ctx.n), dtype=torch.complex128, device="cuda")
            hh.hh_solve(ctx, f, torch.zeros_like(f), rtol=1e-8, maxit=5)
    finally:
        hh.hh_destroy(ctx)
    with pytest.raises(hh.HelmddError):  # depths differ
        hh.hh_setup_batch(2, [(40, 6.0, hh.decomposition([(2, 2)], [4])),
                              (40, 6.0, hh.decomposition([(2, 2), (2, 2)], [4, 4]))])

"""Captured Arnoldi steps (HIP graphs) and the sweep autotuner: both must leave
every result bit-identical to the eager, untuned path.  Graph replays are
interleaved with other device work and host synchronisations, each replay is
checked, and a short restart makes the same step graphs replay several times
within one solve."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N, K, M, OV, RANK, OVERS = 56, 9.0, [(3, 3)], [4], 3, 4


@pytest.fixture(scope="module")
def hh():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_12538_amd as lib

    return lib


def _ctx(hh, stream, **kw):
    from gpu_util import gpu_omega

    ctx = hh.hh_setup(2, N, K, hh.decomposition(M, OV), stream=stream, **kw)
    om, _, _ = gpu_omega(hh, ctx, 1, RANK, OVERS)
    hh.hh_build_coarse(ctx, 1, RANK, OVERS, om)
    return ctx


def _solve(hh, ctx, f, restart_maxit=300):
    from gpu_util import dev, host

    u = dev(np.zeros_like(f))
    info = hh.hh_solve(ctx, dev(f), u, rtol=1e-9, maxit=restart_maxit)
    return host(u), [i[0] for i in info]


def test_autotuned_sweep_is_bit_identical(hh):
    import torch

    s = torch.cuda.Stream()
    f = W.white_rhs((N + 1) ** 2, 31, 9)
    plain = _ctx(hh, s)
    tuned = _ctx(hh, s, autotune=True)
    try:
        u0, i0 = _solve(hh, plain, f)
        u1, i1 = _solve(hh, tuned, f)
        assert i0 == i1 and np.array_equal(u0, u1)
        plan = hh.hh_sweep_plan(tuned)
        assert plan and all(p["tuned_for"] == 9 and p["qb"] in (1, 2, 4) for p in plan)
        assert sum(p["leaves"] for p in plan) == 9
    finally:
        hh.hh_destroy(plain)
        hh.hh_destroy(tuned)


@pytest.mark.parametrize("restart", [50, 6])
def test_graph_replays_match_eager_steps(hh, restart):
    import torch

    from gpu_util import dev

    s = torch.cuda.Stream()
    eager = hh.hh_setup(2, N, K, hh.decomposition(M, OV), stream=s, gmres_restart=restart)
    graph = hh.hh_setup(2, N, K, hh.decomposition(M, OV), stream=s, gmres_restart=restart, graphs=True)
    from gpu_util import gpu_omega

    try:
        for ctx in (eager, graph):
            om, _, _ = gpu_omega(hh, ctx, 1, RANK, OVERS)
            hh.hh_build_coarse(ctx, 1, RANK, OVERS, om)
        for rep, seed in enumerate([41, 42, 41, 43]):
            f = W.white_rhs((N + 1) ** 2, seed, 3)
            ue, ie = _solve(hh, eager, f)
            ug, ig = _solve(hh, graph, f)  # rep 0 eager, rep 1 captures, reps 2-3 replay
            assert ie == ig, rep
            assert np.array_equal(ue, ug), rep
            # unrelated eager work and a synchronisation between replays
            x = dev(W.white_rhs((N + 1) ** 2, 100 + rep, 2))
            y = torch.zeros_like(x)
            hh.hh_apply_operator(graph, x, y)
            torch.cuda.synchronize()
    finally:
        hh.hh_destroy(eager)
        hh.hh_destroy(graph)


def test_graphs_follow_a_rebuilt_coarse_space(hh):
    import torch

    from gpu_util import gpu_omega

    s = torch.cuda.Stream()
    eager = _ctx(hh, s)
    graph = _ctx(hh, s, graphs=True)
    try:
        f = W.white_rhs((N + 1) ** 2, 51, 2)
        for _ in range(2):
            _solve(hh, graph, f)
        # a different coarse space: the captured steps must not be reused
        for ctx in (eager, graph):
            om, _, _ = gpu_omega(hh, ctx, 1, RANK + 1, OVERS, seed=3)
            hh.hh_build_coarse(ctx, 1, RANK + 1, OVERS, om)
        for _ in range(3):
            ue, ie = _solve(hh, eager, f)
            ug, ig = _solve(hh, graph, f)
            assert ie == ig and np.array_equal(ue, ug)
    finally:
        hh.hh_destroy(eager)
        hh.hh_destroy(graph)


def test_concurrent_contexts_on_two_threads_match_sequential(hh):
    """Two host threads, each with its own stream, set up, build and solve
    concurrently (the benchmark's lanes): every result equals the one computed
    alone, bit for bit, and the cached device blocks pass between the streams
    safely."""
    import threading

    import torch

    f = W.white_rhs((N + 1) ** 2, 41, 4)

    def run(stream, out, k):
        with torch.cuda.stream(stream):
            for _ in range(3):
                ctx = _ctx(hh, stream)
                try:
                    out.append(_solve(hh, ctx, f))
                finally:
                    hh.hh_destroy(ctx)
        out.append(k)

    s0 = torch.cuda.Stream()
    alone = []
    run(s0, alone, "alone")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[], []]
    errors = []

    def guarded(i):
        try:
            run(streams[i], outs[i], i)
        except BaseException as e:  # noqa: BLE001 - re-raised below
            errors.append(e)

    threads = [threading.Thread(target=guarded, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    u_ref, it_ref = alone[0]
    for out in outs:
        assert len(out) == 4
        for u, it in out[:3]:
            assert it == it_ref and np.array_equal(u, u_ref)

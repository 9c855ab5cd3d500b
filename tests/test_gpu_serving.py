"""Serving loop (hh_server_*): continuous batching over operator ids on one GPU.

Checks that a result does not depend on what it was served with (alone, or
batched with other requests while other operators run), that a served result
equals a direct solve with the same Gaussian blocks, that the memory budget
evicts idle operators and refuses what cannot fit, and that invalid requests
are rejected at submission.
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

OPS = {
    # id: (N, k, m, overlap, ranks)
    11: (40, 9.0, [(2, 2)], [4], [3]),
    12: (48, 11.0, [(3, 3)], [4], [3]),
    13: (32, 7.0, [(2, 2), (2, 2)], [4, 4], [2, 2]),
}
# same shapes, different wavenumbers: equal footprints (the eviction test)
TWINS = {21: (40, 9.0, [(2, 2)], [4], [3]), 22: (40, 9.5, [(2, 2)], [4], [3])}
SPECS = {**OPS, **TWINS}
SEED = 77


@pytest.fixture(scope="module")
def hh():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_12538_amd as lib

    return lib


def _requests():
    """(operator id, nrhs, seed of f) in submission order."""
    rng = np.random.default_rng(5)
    out = []
    for t in range(14):
        oid = list(OPS)[t % 3] if t < 6 else int(rng.choice(list(OPS)))
        out.append((oid, int(rng.integers(1, 4)), 100 + t))
    return out


def _submit(hh, srv, oid, nrhs, fseed, rtol=1e-9):
    import torch

    N, k, m, ov, ranks = SPECS[oid]
    f = torch.from_numpy(W.white_rhs((N + 1) ** 2, fseed, nrhs)).to("cuda")
    u = torch.zeros_like(f)
    t = srv.submit(oid, 2, N, k, hh.decomposition(m, ov), ranks, 4, SEED, f, u, rtol=rtol, maxit=300)
    return t, u


def _serve(hh, reqs, workers, one_at_a_time, budget=8 << 30):
    import torch

    outs, results = [], []
    with hh.Server(budget, workers=workers, max_batch_rhs=8) as srv:
        if one_at_a_time:
            for oid, nrhs, fs in reqs:
                t, u = _submit(hh, srv, oid, nrhs, fs)
                results.append(srv.wait(t, 120.0))
                outs.append(u)
        else:
            pend = [_submit(hh, srv, *r) for r in reqs]
            for t, u in pend:
                results.append(srv.wait(t, 120.0))
                outs.append(u)
        torch.cuda.synchronize()
        stats = srv.stats()
        stats["last_error"] = srv.last_error()
    return [o.cpu().numpy() for o in outs], results, stats


def test_results_are_the_same_alone_and_in_the_mix(hh):
    reqs = _requests()
    alone, ra, _ = _serve(hh, reqs, workers=1, one_at_a_time=True)
    mixed, rm, stats = _serve(hh, reqs, workers=3, one_at_a_time=False)
    for r in ra + rm:
        assert r["status"] == hh.HH_OK and r["rel_residual"] < 1e-9
    assert max(r["batch_rhs"] for r in rm) > max(n for _, n, _ in reqs)  # requests were batched together
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)
    assert stats["served"] == len(reqs) and stats["misses"] == len(OPS)


def test_served_result_equals_direct_solve(hh):
    import torch

    oid = 12
    N, k, m, ov, ranks = OPS[oid]
    (u_srv,), (res,), _ = _serve(hh, [(oid, 2, 555)], workers=1, one_at_a_time=True)
    assert res["status"] == hh.HH_OK
    ctx = hh.hh_setup(2, N, k, hh.decomposition(m, ov))
    try:
        for level in range(len(m), 0, -1):
            m_in, _, s = hh.hh_level_info(ctx, level, ranks[level - 1], 4)
            om = np.concatenate([hh.hh_omega_philox(SEED, level, i, int(m_in[i]), int(s[i])).reshape(-1)
                                 for i in range(len(m_in))])
            hh.hh_build_coarse(ctx, level, ranks[level - 1], 4, torch.from_numpy(om).to("cuda"))
        f = torch.from_numpy(W.white_rhs((N + 1) ** 2, 555, 2)).to("cuda")
        u = torch.zeros_like(f)
        info = hh.hh_solve(ctx, f, u, rtol=1e-9, maxit=300)
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), u_srv)
        assert res["iters"] == max(i[0] for i in info)
    finally:
        hh.hh_destroy(ctx)


def test_budget_evicts_idle_operators_and_refuses_oversize(hh):
    reqs = [(21, 1, 900), (22, 1, 901), (21, 1, 902), (22, 1, 903)]
    ref, rr, _ = _serve(hh, reqs, workers=1, one_at_a_time=True)
    assert all(r["status"] == hh.HH_OK for r in rr)
    _, _, st1 = _serve(hh, reqs[:1], workers=1, one_at_a_time=True)
    resident = st1["reserved_bytes"]  # one prepared operator, no batch running
    N, k, m, ov, ranks = TWINS[21]
    need = hh.hh_estimate_device_bytes(2, N, hh.decomposition(m, ov), ranks, 4, 1)
    # one prepared operator plus a new one's admission does not fit; either alone does
    budget = resident + need - 1
    outs, res, stats = _serve(hh, reqs, workers=1, one_at_a_time=True, budget=budget)
    assert all(r["status"] == hh.HH_OK for r in res)
    assert stats["evictions"] >= 3 and stats["misses"] == 4
    for a, b in zip(ref, outs):
        assert np.array_equal(a, b)
    assert stats["last_error"] == ""
    _, res, stats = _serve(hh, [(21, 1, 904)], workers=1, one_at_a_time=True, budget=1 << 16)
    assert res[0]["status"] == hh.HH_ENOMEM
    assert stats["last_error"].startswith("HH_ENOMEM (operator 21, 1 rhs)")


def test_a_second_server_after_a_closed_one_serves_cleanly(hh):
    """Device blocks cached from a closed server's streams are reused by a new
    server without waiting on events of the destroyed streams."""
    reqs = _requests()
    first, r1, _ = _serve(hh, reqs, workers=3, one_at_a_time=False)
    second, r2, st2 = _serve(hh, reqs, workers=3, one_at_a_time=False)
    assert all(r["status"] == hh.HH_OK for r in r1 + r2) and st2["last_error"] == ""
    for a, b in zip(first, second):
        assert np.array_equal(a, b)


def test_invalid_requests_are_rejected(hh):
    import torch

    with hh.Server(1 << 30, workers=1, max_batch_rhs=2) as srv:
        N, k, m, ov, ranks = OPS[11]
        f = torch.zeros((3, (N + 1) ** 2), dtype=torch.complex128, device="cuda")
        with pytest.raises(hh.HelmddError):  # wider than a batch
            srv.submit(11, 2, N, k, hh.decomposition(m, ov), ranks, 4, SEED, f, torch.zeros_like(f))
        f1 = f[:1].contiguous()
        t = srv.submit(11, 2, N, k, hh.decomposition(m, ov), ranks, 4, SEED, f1, torch.zeros_like(f1))
        srv.wait(t, 60.0)
        with pytest.raises(hh.HelmddError):  # one id, one operator shape
            srv.submit(11, 2, N + 2, k, hh.decomposition(m, ov), ranks, 4, SEED,
                       torch.zeros((1, (N + 3) ** 2), dtype=torch.complex128, device="cuda"),
                       torch.zeros((1, (N + 3) ** 2), dtype=torch.complex128, device="cuda"))

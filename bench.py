"""Benchmark: Helmholtz solves/s at 1e-8 relative residual on one MI355X.

Workload (one step): the 2D impedance Helmholtz problem on the unit square,
N = 256 cells per side (66,049 nodes), k = 40 (about 40 points per
wavelength), 4x4 box subdomains with a 4-cell overlap, randomised-SVD coarse
space with rank 8 per interface and 10 oversampling samples, a batch of
seeded smoothed complex Gaussian right-hand sides.  A step runs the whole
path: hh_setup (leaf factorisations), hh_build_coarse (sketch, QR, adjoint,
small SVD, extension, Galerkin A_c and its inverse) and hh_solve (GMRES(50)
around the ORAS + coarse preconditioner) to a relative residual of 1e-8 for
every right-hand side.  Inputs (the RHS batch, the Gaussian blocks) are
resident in HBM before the timed region.

Prints one JSON line.  `--gpus N` with N > 1 exits: this path runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Helmholtz solves/s at 1e-8 rel. residual, mixed vs FP64 plain; p99 latency"
HBM_PEAK_GBS = 8000.0
# vector FP64 FMA rate, and FP32 without packed instructions (the build disables them):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
VALU_PEAK_TFS = 78.6
CFG = dict(N=256, k=40.0, m=[(4, 4)], overlap=[4], rank=8, oversample=10, rtol=1e-8, maxit=500, restart=50)
FAMILY = {0: "k_sweep (leaf block-tridiagonal solve, phase 1 + phase 2)", 1: "k_basis_update (Gram-Schmidt)",
          2: "k_dot_partial (Gram-Schmidt inner products)", 3: "k_apply_box (5-point stencil y = A z)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=2,
                    help="host threads (one stream and one context per step each) running steps concurrently")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="no live kernel events in the timed region")
    ap.add_argument("--cpu-rhs", type=int, default=2, help="right-hand sides in the CPU oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--serving-seconds", type=float, default=5.0,
                    help="length of the request stream of the serving measurement (0: skip)")
    ap.add_argument("--serving-rate", type=float, default=200.0, help="mean request arrivals per second (nominal)")
    ap.add_argument("--serving-rate-low", type=float, default=20.0,
                    help="a second, sustainable arrival rate (0: skip)")
    ap.add_argument("--serving-drain", type=float, default=20.0,
                    help="seconds to wait for queued requests after the stream ends")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="independent problems of the batched measurement (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed steps of the batched measurement")
    ap.add_argument("--no-steady", action="store_true", help="skip the steady-state (cached setup) solve measurement")
    ap.add_argument("--no-serial", action="store_true", help="skip the one-lane comparison run")
    return ap.parse_args()


def make_inputs(hh, torch, nrhs, seed=1):
    import workloads as W

    probe = hh.hh_setup(2, CFG["N"], CFG["k"], hh.decomposition(CFG["m"], CFG["overlap"]))
    m_in, _, s = hh.hh_level_info(probe, 1, CFG["rank"], CFG["oversample"])
    hh.hh_destroy(probe)
    f = W.smoothed_gaussian_rhs(CFG["N"], seed, nrhs)
    om = np.concatenate([W.omega_block(0, 1, i, int(m_in[i]), int(s[i])).reshape(-1) for i in range(len(m_in))])
    return torch.from_numpy(f).to("cuda"), torch.from_numpy(om).to("cuda"), f


def one_step(hh, fd, om, u, precision, phases=None, prof=None, stream=None):
    t0 = time.perf_counter()
    ctx = hh.hh_setup(2, CFG["N"], CFG["k"], hh.decomposition(CFG["m"], CFG["overlap"]), precision=precision,
                      outer=hh.HH_GMRES, gmres_restart=CFG["restart"], stream=stream)
    t1 = time.perf_counter()
    hh.hh_build_coarse(ctx, 1, CFG["rank"], CFG["oversample"], om)
    t2 = time.perf_counter()
    if prof is not None:
        hh.hh_profile(ctx, True)
    info = hh.hh_solve(ctx, fd, u, CFG["rtol"], CFG["maxit"], raise_on_notconv=True)
    t3 = time.perf_counter()
    if prof is not None:
        for fam in FAMILY:
            n, ms, by, fl = hh.hh_profile_read(ctx, fam)
            acc = prof.setdefault(fam, [0, 0.0, 0.0, 0.0])
            acc[0] += n
            acc[1] += ms
            acc[2] += by
            acc[3] += fl
    hh.hh_destroy(ctx)
    if phases is not None:
        phases["setup"].append(t1 - t0)
        phases["build_coarse"].append(t2 - t1)
        phases["solve"].append(t3 - t2)
    return info


def run_gpu(hh, torch, nrhs, precision, steps, warmup, profile, lanes=1):
    """Steps of the whole path on `lanes` host threads, each with its own stream and context per step, so that the
    set-up and coarse build of one step (latency-bound, few work-groups) overlap the solve of another (bandwidth-bound
    Krylov passes).  Warm-up and timed steps are dealt round-robin to the lanes."""
    import threading

    fd, om, f = make_inputs(hh, torch, nrhs)
    lanes = max(1, lanes)
    streams = [torch.cuda.Stream() for _ in range(lanes)]
    us = [torch.zeros_like(fd) for _ in range(lanes)]
    torch.cuda.synchronize()
    lock = threading.Lock()
    phases = {"setup": [], "build_coarse": [], "solve": []}
    prof = {} if profile else None
    lat = []
    iters = []
    errors = []

    def lane(k, count, record):
        try:
            with torch.cuda.stream(streams[k]):
                for _ in range(count):
                    ph = {"setup": [], "build_coarse": [], "solve": []} if record else None
                    pr = {} if (record and profile) else None
                    ts = time.perf_counter()
                    info = one_step(hh, fd, om, us[k], precision, ph, pr, streams[k])
                    dt = time.perf_counter() - ts
                    if not all(i[1] for i in info):
                        raise RuntimeError("a right-hand side did not converge")
                    if record:
                        with lock:
                            lat.append(dt)
                            iters[:] = [i[0] for i in info]
                            for key, v in ph.items():
                                phases[key].extend(v)
                            if pr is not None:
                                for fam, acc in pr.items():
                                    tot = prof.setdefault(fam, [0, 0.0, 0.0, 0.0])
                                    for j in range(4):
                                        tot[j] += acc[j]
        except BaseException as e:  # noqa: BLE001 - re-raised on the main thread
            errors.append(e)

    def run_lanes(total, record):
        counts = [total // lanes + (1 if k < total % lanes else 0) for k in range(lanes)]
        threads = [threading.Thread(target=lane, args=(k, counts[k], record)) for k in range(lanes) if counts[k] > 0]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]

    run_lanes(warmup, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_lanes(steps, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(wall=wall, phases=phases, lat=lat, iters=iters, u=us[0], f=f, prof=prof, lanes=lanes)


CSRC = os.path.join(ROOT, "paper_2512_12538_amd", "csrc")
# HBM traffic per launch of each kernel family, from the committed counter summaries, and the sources it depends on
TRAFFIC = {
    0: (os.path.join(ROOT, "profiles", "k_sweep_helm2d_n256_k40_4x4.md"),
        [os.path.join(CSRC, f) for f in ("k_sweep.hip", "common.h")]),
    1: (os.path.join(ROOT, "profiles", "k_basis_update_k_dot_partial_helm2d_n256_k40_4x4.md"),
        [os.path.join(CSRC, f) for f in ("k_krylov.hip", "common.h")]),
    2: (os.path.join(ROOT, "profiles", "k_basis_update_k_dot_partial_helm2d_n256_k40_4x4.md"),
        [os.path.join(CSRC, f) for f in ("k_krylov.hip", "common.h")]),
}


def measured_traffic(fam, nrhs, precision, lanes):
    """HBM bytes per launch of kernel family fam from the committed FETCH_SIZE / WRITE_SIZE passes, scaled by the
    copy calibration; None when there is no summary for it or the kernel source or the workload differs."""
    import hashlib

    if fam not in TRAFFIC:
        return None
    path, sources = TRAFFIC[fam]
    try:
        fig = {}
        for line in open(path):
            k, sep, v = line.strip().partition(": ")
            if sep:
                fig[k] = v
        h = hashlib.sha256()
        for f in sources:
            h.update(open(f, "rb").read())
    except OSError:
        return None
    if fig.get("kernel_source_sha256") != h.hexdigest():
        return None
    if fig.get("rhs_per_step") != str(nrhs) or fig.get("precision") != precision or fig.get("lanes") != str(lanes):
        return None
    try:
        fetch = float(fig[f"family_{fam}_fetch_kib_per_launch"]) * float(fig["fetch_scale"])
        write = float(fig[f"family_{fam}_write_kib_per_launch"]) * float(fig["write_scale"])
    except KeyError:
        return None
    return round((fetch + write) * 1024.0)


def roofline(prof, precision, nrhs, lanes):
    if not prof:
        return None
    fam = max(prof, key=lambda k: prof[k][1])
    n, ms, by, fl = prof[fam]
    if n == 0:
        return None
    avg_s = ms / n / 1000.0
    bytes_launch = by / n
    flops_launch = fl / n
    intensity = fl / by if by else 0.0
    ridge = VALU_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if fam == 0 and intensity >= ridge:
        achieved = flops_launch / avg_s / 1e12
        out = {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TFS, "unit": "TFLOP/s",
               "frac": round(achieved / VALU_PEAK_TFS, 4)}
    else:
        achieved = bytes_launch / avg_s / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4)}
    out.update({"traffic": measured_traffic(fam, nrhs, precision, lanes), "kernel": FAMILY[fam], "launches": int(n),
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": round(bytes_launch),
                "algorithmic_flops_per_launch": round(flops_launch), "intensity_flop_per_byte": round(intensity, 2),
                "other_families_ms": {FAMILY[k]: round(v[1], 2) for k, v in prof.items() if k != fam},
                "families": {FAMILY[k]: {"launches": int(v[0]), "total_ms": round(v[1], 2),
                                         "avg_launch_us": round(1000.0 * v[1] / v[0], 2) if v[0] else None,
                                         "algorithmic_bytes_per_launch": round(v[2] / v[0]) if v[0] else None,
                                         "hbm_frac": round(v[2] / (v[1] / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)
                                         if v[0] and v[1] > 0 else None,
                                         "traffic": measured_traffic(k, nrhs, precision, lanes)}
                             for k, v in prof.items()}})
    return out


def cpu_baseline(nrhs):
    """The FP64 oracle on a bounded sample: one full step (setup, coarse build, GMRES) for nrhs right-hand sides."""
    import workloads as W
    from oracle import krylov
    from oracle.schwarz import HierarchicalORAS

    try:
        from threadpoolctl import threadpool_info

        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    N = CFG["N"]
    kk = np.full((N + 1) ** 2, CFG["k"])
    f = W.smoothed_gaussian_rhs(N, 1, nrhs)
    t0 = time.perf_counter()
    S = HierarchicalORAS(2, N, kk, CFG["m"], CFG["overlap"])
    oms = []
    for i in range(len(S.H.levels[1])):
        m_in, _, s = S.sizes(1, i, CFG["rank"], CFG["oversample"])
        oms.append(W.omega_block(0, 1, i, m_in, s))
    S.build_coarse(1, CFG["rank"], CFG["oversample"], oms)
    its = []
    for j in range(nrhs):
        _, info = krylov.fgmres(lambda x: S.A @ x, S.precondition, f[j], tol=CFG["rtol"], maxit=CFG["maxit"],
                                restart=CFG["restart"])
        its.append(info.iters)
    dt = time.perf_counter() - t0
    return dict(value=round(nrhs / dt, 4), unit="solves/s", cores=int(cores), kind="oracle",
                sample=f"one full step (setup + coarse build + GMRES to 1e-8) of the same workload for {nrhs} "
                       f"right-hand sides, {dt:.1f} s, GMRES iterations {its}; BLAS threads = cores, SuperLU "
                       f"single-threaded")


# Request stream of the serving measurement: Poisson arrivals; grid side 128 / 256
# / 512 / 1024 with probabilities .4 / .3 / .2 / .1, k = side / 6.4, 1-4 right-
# hand sides; 70 % of the requests reuse an operator already seen for their
# side, the others bring a new one (k scaled by 1 + 0.05 u, u ~ U(-1, 1)), which
# forces a full set-up.  Decompositions: 128 -> [2x2] and 256 -> [4x4] (4-cell
# overlap, rank 8 per interface); 512 -> [2x2, 2x2] and 1024 -> [2x2, 2x2, 2x2]
# (8-cell overlap, rank 16); 10 oversampling samples; 200 GB device budget.
SERVING_SIDES = [(128, 0.4, [(2, 2)], [4], [8]), (256, 0.3, [(4, 4)], [4], [8]),
                 (512, 0.2, [(2, 2), (2, 2)], [8, 8], [16, 16]),
                 (1024, 0.1, [(2, 2), (2, 2), (2, 2)], [8, 8, 8], [16, 16, 16])]


def serving(hh, torch, precision, seconds, rate, drain=30.0, seed=11):
    """Drives hh_server_* with a seeded request stream for `seconds`, then waits at most `drain`
    seconds for the requests still queued or running.  Latency = arrival -> result in u (host);
    requests not finished by then count as unfinished (percentiles treat them as infinitely late)."""
    import threading

    rng = np.random.default_rng(seed)
    sched, seen, t, next_id = [], {}, 0.0, 1
    while t < seconds:
        t += rng.exponential(1.0 / rate)
        si = int(rng.choice(len(SERVING_SIDES), p=[x[1] for x in SERVING_SIDES]))
        side = SERVING_SIDES[si][0]
        if seen.get(side) and rng.random() < 0.7:
            oid, k = seen[side][int(rng.integers(len(seen[side])))]
        else:
            oid, k = next_id, side / 6.4 * (1.0 + 0.05 * rng.uniform(-1.0, 1.0))
            next_id += 1
            seen.setdefault(side, []).append((oid, k))
        sched.append((t, si, oid, k, int(rng.integers(1, 5))))
    # device right-hand sides per side (content is immaterial to the timing; CN(0,1))
    pool = {}
    for si, (side, _, _, _, _) in enumerate(SERVING_SIDES):
        n = (side + 1) ** 2
        g = torch.Generator(device="cuda").manual_seed(seed + si)
        pool[si] = torch.complex(torch.randn((4, n), device="cuda", dtype=torch.float64, generator=g),
                                 torch.randn((4, n), device="cuda", dtype=torch.float64, generator=g)) / np.sqrt(2.0)
    torch.cuda.synchronize()
    results = [None] * len(sched)
    srv = hh.Server(200 * 10 ** 9, workers=12, max_batch_rhs=32, precision=precision, gmres_restart=100)
    tickets = [None] * len(sched)
    t0 = time.perf_counter()
    deadline = t0 + seconds + drain

    def collect():
        pending = 0  # tickets below this index are all collected or not yet submitted
        while time.perf_counter() < deadline:
            done = True
            for i in range(pending, len(sched)):
                if tickets[i] is None:
                    done = False
                    break
                if results[i] is None:
                    results[i] = srv.poll(tickets[i])
                    done = done and results[i] is not None
            while pending < len(sched) and results[pending] is not None:
                pending += 1
            if done and pending == len(sched):
                return
            time.sleep(0.002)

    col = threading.Thread(target=collect)
    col.start()
    outs = []
    last = t0
    for i, (ta, si, oid, k, nr) in enumerate(sched):
        side, _, m, ov, ranks = SERVING_SIDES[si]
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        f = pool[si][:nr]
        u = torch.empty_like(f)
        outs.append(u)
        tickets[i] = srv.submit(oid, 2, side, k, hh.decomposition(m, ov), ranks, 10, 1000 + oid, f, u, rtol=1e-8,
                                maxit=1000)
        if time.perf_counter() - last > 2.0:
            last = time.perf_counter()
            print(f"serving: {i + 1}/{len(sched)} submitted, {sum(r is not None for r in results)} done",
                  file=sys.stderr, flush=True)
    while col.is_alive():
        col.join(2.0)
        print(f"serving: draining, {sum(r is not None for r in results)}/{len(sched)} done", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - t0
    stats = srv.stats()
    last_error = srv.last_error()
    srv.close()  # drops what is still queued; running batches end first
    fin = [(x, r) for x, r in zip(sched, results) if r is not None]
    lat = np.array([r["latency_s"] for _, r in fin] + [np.inf] * (len(sched) - len(fin))) * 1000.0
    ok = sum(1 for _, r in fin if r["status"] == hh.HH_OK)
    rhs_done = sum(x[4] for x, _ in fin)
    by_side = {}
    for x, r in fin:
        by_side.setdefault(SERVING_SIDES[x[1]][0], []).append(r["latency_s"] * 1000.0)

    def pct(v, p):
        q = float(np.percentile(v, p))
        return round(q, 1) if np.isfinite(q) else None

    return {
        "requests": len(sched), "finished": len(fin), "converged": ok, "rhs_finished": rhs_done,
        "stream_s": round(seconds, 2), "wall_s": round(wall, 2), "rhs_per_s": round(rhs_done / wall, 2),
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "latency_p50_ms_by_side": {str(k): round(float(np.percentile(v, 50)), 1) for k, v in sorted(by_side.items())},
        "mean_batch_rhs": round(float(np.mean([r["batch_rhs"] for _, r in fin])), 2) if fin else None,
        "cache_hit_rate": round(float(np.mean([r["cache_hit"] for _, r in fin])), 3) if fin else None,
        "operators_set_up": stats["misses"], "evictions": stats["evictions"],
        "status_by_side": _status_by_side(hh, fin),
        "last_batch_error": last_error or None,
    }


def _status_by_side(hh, fin):
    out = {}
    for x, r in fin:
        key = f"{SERVING_SIDES[x[1]][0]}:{hh._STATUS[r['status']]}"
        out[key] = out.get(key, 0) + 1
    return dict(sorted(out.items()))


def batched(hh, torch, precision, count, steps, warmup=1, seed=4):
    """The mixed batch of independent problems in one context: per step hh_setup_batch +
    hh_build_coarse + hh_solve (one RHS per problem, GMRES(50) to 1e-8)."""
    import workloads as W

    cfg = W.WORKLOADS["helm2d_batch512"]
    probs = W.batch_problems(count, seed)
    dec = {m: hh.decomposition([(m, m)], cfg["overlap"]) for m in (2, 3, 4)}
    problems = [(side, k, dec[m]) for side, k, m in probs]
    rank, over = cfg["rank"], cfg["oversample"]
    # inputs, resident on the device before the timed steps
    probe = hh.hh_setup_batch(2, problems, precision=precision)
    m_in, _, s = hh.hh_level_info(probe, 1, rank, over)
    hh.hh_destroy(probe)
    parts, box = [], 0
    for p, (_, _, m) in enumerate(probs):
        for i in range(m * m):
            parts.append(W.omega_block(1000 + p, 1, i, int(m_in[box]), int(s[box])).reshape(-1))
            box += 1
    om = torch.from_numpy(np.concatenate(parts)).to("cuda")
    del parts
    f = torch.cat([torch.from_numpy(W.white_rhs((side + 1) ** 2, 5000 + p).reshape(-1))
                   for p, (side, _, _) in enumerate(probs)]).to("cuda")
    u = torch.zeros_like(f)
    torch.cuda.synchronize()
    times, phases, iters = [], {"setup": [], "build_coarse": [], "solve": []}, []
    for it in range(warmup + steps):
        t0 = time.perf_counter()
        ctx = hh.hh_setup_batch(2, problems, precision=precision, outer=hh.HH_GMRES, gmres_restart=50)
        t1 = time.perf_counter()
        hh.hh_build_coarse(ctx, 1, rank, over, om)
        t2 = time.perf_counter()
        info = hh.hh_solve(ctx, f, u, 1e-8, 400, raise_on_notconv=True)
        t3 = time.perf_counter()
        hh.hh_destroy(ctx)
        print(f"batched {precision}: step {it} {t3 - t0:.3f} s", file=sys.stderr, flush=True)
        if it >= warmup:
            times.append(t3 - t0)
            phases["setup"].append(t1 - t0)
            phases["build_coarse"].append(t2 - t1)
            phases["solve"].append(t3 - t2)
            iters = [i[0] for i in info]
    wall = float(np.sum(times))
    by_side = {}
    for (side, _, _), it in zip(probs, iters):
        by_side.setdefault(side, []).append(it)
    return {
        "value": round(count * steps / wall, 3), "unit": "solves/s", "ms_per_step": round(1000 * wall / steps, 3),
        "phases_ms": {k: round(1000.0 * float(np.mean(v)), 3) for k, v in phases.items()},
        "solve_only_solves_per_s": round(count / float(np.mean(phases["solve"])), 3),
        "gmres_iterations": {"min": int(min(iters)), "max": int(max(iters)), "mean": round(float(np.mean(iters)), 2)},
        "iterations_mean_by_side": {str(k): round(float(np.mean(v)), 1) for k, v in sorted(by_side.items())},
        "nodes_total": int(f.numel()), "subdomains": int(box),
    }


def steady_state(hh, torch, precision, N, k, m, rank, nrhs, graphs, solves=6, seed=21):
    """Repeated solves on one prepared context (setup and coarse space cached): solves/s over the
    last solves-2 (the first runs eagerly and tunes the sweep, the second captures the step graphs)."""
    import workloads as W

    stream = torch.cuda.Stream()
    ctx = hh.hh_setup(2, N, k, hh.decomposition(m, [4]), precision=precision, outer=hh.HH_GMRES, gmres_restart=50,
                      stream=stream, autotune=True, graphs=graphs)
    m_in, _, s = hh.hh_level_info(ctx, 1, rank, 10)
    om = torch.from_numpy(np.concatenate([W.omega_block(0, 1, i, int(m_in[i]), int(s[i])).reshape(-1)
                                          for i in range(len(m_in))])).to("cuda")
    torch.cuda.synchronize()
    hh.hh_build_coarse(ctx, 1, rank, 10, om)
    f = torch.from_numpy(W.smoothed_gaussian_rhs(N, seed, nrhs)).to("cuda")
    u = torch.zeros_like(f)
    torch.cuda.synchronize()
    times = []
    for _ in range(solves):
        t0 = time.perf_counter()
        hh.hh_solve(ctx, f, u, 1e-8, 300, raise_on_notconv=True)
        times.append(time.perf_counter() - t0)
    plan = hh.hh_sweep_plan(ctx)
    hh.hh_destroy(ctx)
    t = float(np.mean(times[2:]))
    return {"solves_per_s": round(nrhs / t, 2), "ms_per_solve_call": round(1000 * t, 3),
            "sweep_qb": [p["qb"] for p in plan]}


def guarded(fn, *a, **kw):
    """Runs an optional measurement; a failure is recorded in the JSON line instead of ending the run."""
    try:
        return fn(*a, **kw)
    except Exception as e:  # noqa: BLE001 - any failure of a side measurement is reported, not raised
        print(f"bench: {getattr(fn, '__name__', fn)} failed: {e}", file=sys.stderr, flush=True)
        return {"error": f"{type(e).__name__}: {e}"}


def section_done(torch, name):
    """Progress line, and a device round trip so that an error left by a section is reported there."""
    try:
        torch.cuda.synchronize()
        torch.ones(1, device="cuda").add_(1)
        torch.cuda.synchronize()
        print(f"bench: {name} done", file=sys.stderr, flush=True)
    except Exception as e:  # noqa: BLE001 - reported; the next measurement records its own failure
        print(f"bench: device error after {name}: {e}", file=sys.stderr, flush=True)


def copy_calibration(torch):
    n = 1 << 26  # 1 GiB of complex128
    x = torch.ones(n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 16, "launches": 3}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2512_12538_amd as hh

    prec = hh.HH_MIXED if args.precision == "mixed" else hh.HH_FP64
    res = run_gpu(hh, torch, args.nrhs, prec, args.steps, args.warmup, not args.no_profile, args.lanes)
    wall = res["wall"]
    ms_per_step = 1000.0 * wall / args.steps
    value = args.nrhs * args.steps / wall
    lat = np.array(res["lat"]) * 1000.0
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "helm2d_n256_k40_4x4",
            "grid_cells": CFG["N"], "k": CFG["k"], "decomposition": "[4x4]", "overlap_cells": 4,
            "rank_per_interface": CFG["rank"], "oversample": CFG["oversample"], "rhs_per_step": args.nrhs,
            "outer": f"gmres({CFG['restart']})", "rtol": CFG["rtol"], "precision": args.precision,
            "step": "hh_setup + hh_build_coarse + hh_solve of the RHS batch",
            "lanes": res["lanes"],
            "lanes_note": "steps run on this many host threads, each with its own stream, so one step's set-up and "
                          "coarse build overlap another's solve; latency and phases are per step under that overlap",
        },
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)},
        "phases_ms": {k: round(1000.0 * float(np.mean(v)), 3) for k, v in res["phases"].items()},
        "gmres_iterations": {"min": int(min(res["iters"])), "max": int(max(res["iters"])),
                             "mean": round(float(np.mean(res["iters"])), 2)},
        "solve_only_solves_per_s": round(args.nrhs / float(np.mean(res["phases"]["solve"])), 3),
        "roofline": roofline(res["prof"], args.precision, args.nrhs, res["lanes"]),
    }
    section_done(torch, "main workload")
    if res["lanes"] > 1 and not args.no_serial:
        sres = run_gpu(hh, torch, args.nrhs, prec, max(2, args.steps // 2), 1, not args.no_profile, 1)
        slat = np.array(sres["lat"]) * 1000.0
        out["serial"] = {
            "note": "the same steps one after another on one stream",
            "value": round(args.nrhs * len(sres["lat"]) / sres["wall"], 3),
            "ms_per_step": round(1000.0 * sres["wall"] / len(sres["lat"]), 3),
            "latency_ms": {"p50": round(float(np.percentile(slat, 50)), 3),
                           "p99": round(float(np.percentile(slat, 99)), 3)},
            "phases_ms": {k: round(1000.0 * float(np.mean(v)), 3) for k, v in sres["phases"].items()},
            "solve_only_solves_per_s": round(args.nrhs / float(np.mean(sres["phases"]["solve"])), 3),
            "roofline": roofline(sres["prof"], args.precision, args.nrhs, 1),
        }
        section_done(torch, "serial steps")
    if not args.no_mixed and args.precision == "fp64":
        mres = run_gpu(hh, torch, args.nrhs, hh.HH_MIXED, max(2, args.steps // 2), res["lanes"], False, res["lanes"])
        mlat = np.array(mres["lat"]) * 1000.0
        out["mixed"] = {
            "value": round(args.nrhs * len(mres["lat"]) / mres["wall"], 3),
            "latency_ms": {"p50": round(float(np.percentile(mlat, 50)), 3),
                           "p99": round(float(np.percentile(mlat, 99)), 3)},
            "phases_ms": {k: round(1000.0 * float(np.mean(v)), 3) for k, v in mres["phases"].items()},
            "solve_only_solves_per_s": round(args.nrhs / float(np.mean(mres["phases"]["solve"])), 3),
            "gmres_iterations_mean": round(float(np.mean(mres["iters"])), 2),
        }
        section_done(torch, "mixed precision")
    if args.serving_seconds > 0:
        out["serving"] = {
            "stream": f"Poisson arrivals for {args.serving_seconds:g} s (then {args.serving_drain:g} s to drain); "
                      "sides 128/256/512/1024 (p .4/.3/.2/.1), k = side/6.4, 1-4 rhs, 70% operator reuse, 200 GB "
                      "budget, 12 workers, batches <= 32 rhs, GMRES(100) to 1e-8; latency = arrival to result on the "
                      "host, requests unfinished at the deadline count as infinitely late",
        }
        for rate in [args.serving_rate] + ([args.serving_rate_low] if args.serving_rate_low > 0 else []):
            res = {}
            for name, prec in (("fp64", hh.HH_FP64), ("mixed", hh.HH_MIXED)):
                section_done(torch, f"before serving {name} at {rate:g}/s")
                res[name] = guarded(serving, hh, torch, prec, args.serving_seconds, rate, args.serving_drain)
            out["serving"][f"rate_{rate:g}_per_s"] = res
        section_done(torch, "serving")
    if not args.no_steady:
        prec = hh.HH_MIXED if args.precision == "mixed" else hh.HH_FP64
        out["steady_state"] = {
            "note": "repeated hh_solve on one prepared context (setup + coarse space cached), autotuned sweep; "
                    "eager steps vs captured HIP-graph steps",
            "helm2d_n256_k40_4x4_64rhs": {g: guarded(steady_state, hh, torch, prec, CFG["N"], CFG["k"], CFG["m"],
                                                                  CFG["rank"], args.nrhs, g == "graphs")
                                          for g in ("eager", "graphs")},
            "helm2d_n128_k20_2x2_1rhs": {g: guarded(steady_state, hh, torch, prec, 128, 20.0, [(2, 2)], 8, 1,
                                                    g == "graphs")
                                         for g in ("eager", "graphs")},
        }
        section_done(torch, "steady state")
    if args.batch_count > 0:
        hh.hh_release_cached_memory()  # the serving runs leave the device cache full
        out["batched"] = {
            "workload": f"helm2d_batch{args.batch_count}: {args.batch_count} independent problems, side uniform in "
                        "{64,96,128,192,256}, k = side/6.4, m x m boxes with m uniform in {2,3,4}, 4-cell overlap, "
                        "rank 8 per interface + 10, one white Gaussian RHS each, GMRES(50) to 1e-8; one context, "
                        "every level of every problem in the same launches; step = setup + coarse build + solve",
            "mixed": guarded(batched, hh, torch, hh.HH_MIXED, args.batch_count, args.batch_steps),
            "fp64": guarded(batched, hh, torch, hh.HH_FP64, args.batch_count, args.batch_steps),
        }
    if not args.no_cpu:
        out["cpu_baseline"] = guarded(cpu_baseline, args.cpu_rhs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

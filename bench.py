#!/usr/bin/env python3
"""Benchmark of the Stokes kernel sums on one MI355X.

Headline workload (the benchmark spec's target is stated at 262k points): the
spindle geometry -- 4096 straight fibers x 64 CGL nodes = 262,144 points
radiating from two poles at (+-4, 0, 0), lengths U(1, 6), eps = 0.005 --
with the Stokeslet + doublet single-layer sum to every node (self-pairs
excluded), timed as K consecutive GMRES-iteration matvecs, each with its own
pre-generated seeded force vector N(0,1)/L.  One step = one matvec (source
preparation + pair sum + chunk reduction).  The mixed FP32/FP64 path is
`value`; the FP64 path is timed on the same inputs beside it.

Also reported: the roofline of the dominant kernel (counted algorithmic flops
per launch / kernel time from HIP events on the launch stream), a short
Poisson serving run (continuous batching of mobility solves) for p50/p99 solve
latency, and the CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps 40] [--warmup 3] [--no-serving] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

METRIC = "Gpair-interactions/s and %VALU peak (mixed vs FP64); p50/p99 solve latency"
FLOPS_PER_PAIR_SL = 34       # Stokeslet + doublet, counted (add/sub/mul 1, FMA 2, rsqrt 1)
FLOPS_PER_PAIR_DL = 33       # stresslet with the on-surface subtraction, counted the same way
PEAK_FP32 = 157.3            # TFLOP/s: published FP32 vector peak, 256 CU x 128 lanes x 2 x 2.4 GHz
PEAK_FP64 = 78.6             # TFLOP/s: published FP64 vector peak
NEAR_R = 0.0                 # mixed path: pairs closer than two fiber radii go FP64

# HBM traffic of one sl_mixed_kernel launch on this workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by the
# factors that make a 256 MiB elementwise copy in the same run read and write
# 256 MiB (FETCH x 1.99977, WRITE x 1.00000); see
# profiles/sl_mixed_spindle_262k_traffic.md.  Valid only for the kernel
# sources with this digest: after any change the field reports null.
TRAFFIC = {"digest": "fae4a9cbbb27fd32", "bytes": 542521081}
# VALU flops per pair from rocprofv3 instruction counters of the same kernel sources
# (64 x (2 FMA + MUL + ADD + TRANS) of the kernel's precision, per dispatch, over the
# pairs of one launch); see profiles/sl_spindle_262k_valu_counters.md.  Combined with
# the live kernel time they give the counter-based fraction of peak.
VALU_FLOPS_PER_PAIR = {"digest": "fae4a9cbbb27fd32", "mixed": 34.51, "fp64": 42.25}
KERNEL_SOURCES = ["paper_1602_05650_amd/csrc/sum_device.hpp",
                  "paper_1602_05650_amd/csrc/stokes_sums.hip",
                  "paper_1602_05650_amd/csrc/stokes_internal.hpp",
                  "paper_1602_05650_amd/csrc/host_logic.hpp",
                  "paper_1602_05650_amd/csrc/pair_math.hpp"]


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_fpp(mixed):
    """Counter-measured VALU flops per pair, or None once the kernel sources changed."""
    if kernel_digest() != VALU_FLOPS_PER_PAIR["digest"]:
        return None
    return VALU_FLOPS_PER_PAIR["mixed" if mixed else "fp64"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-other", action="store_true",
                    help="time the oracle on the headline workload only")
    ap.add_argument("--only", choices=["mixed", "fp64", "both", "none", "nonlocal", "particles",
                                       "treecode", "fiberstep", "serving_cpu", "far", "workloads"],
                    default="both",
                    help="none: serving run alone; nonlocal / particles / treecode / fiberstep: that "
                         "section alone")
    ap.add_argument("--extra", default="c0,c1,c4",
                    help="other workloads timed after the headline (c0,c1,c4 or none)")
    ap.add_argument("--step-pairs", type=float, default=0,
                    help="serving: single-layer pairs one request may take per step "
                         "(0: library default, < 0: whole matvec per step)")
    ap.add_argument("--serving-rate", type=float, default=0,
                    help="serving: fixed Poisson rate in requests/s (0: 0.7 x calibrated capacity)")
    ap.add_argument("--serving-fp64", action="store_true",
                    help="serving run with FP64 sums instead of mixed")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one elementwise copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_matvecs(S, torch, xyz, forces, fib, flen, eps, mixed, steps, warmup):
    """Run warmup + steps matvecs; returns (seconds, kernel_ms_total, launches, out of step 0)."""
    out = torch.empty_like(forces[0])
    kw = dict(src_fiber=fib, fiber_len=flen, eps=eps, mixed=mixed, near_r=NEAR_R, out=out)
    for w in range(warmup):
        S.sl_eval(xyz, forces[w % len(forces)], **kw)
    torch.cuda.synchronize()
    first = S.sl_eval(xyz, forces[0], **dict(kw, out=torch.empty_like(forces[0])))
    torch.cuda.synchronize()
    S.profile_read()                       # drop anything recorded so far
    S.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        S.sl_eval(xyz, forces[k % len(forces)], **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.profile_enable(False)
    ms, launches = S.profile_read()
    return t1 - t0, ms, launches, first


_CONFIGS = {}


def load_config(name):
    """Seeded workload by short name (generated once per process)."""
    from paper_1602_05650_amd import workloads as W
    if name not in _CONFIGS:
        _CONFIGS[name] = {"c0": W.config0, "c1": W.config1, "c4": W.config4}[name]()
    return _CONFIGS[name]


def config_run(S, torch, name, steps, warmup, log_fn):
    """Time the single layer (and, when the config has a sphere, the double layer) to all
    targets, for both precisions; report per sum the whole call (set-up, pair kernel,
    chunk reduction) and the pair kernel alone, in Gpair/s and as a fraction of the
    vector peak of the kernel's precision at the counted flops per pair, and the
    mixed-vs-FP64 error."""
    c = load_config(name)
    fs = c["fibers"]
    dev = torch.device("cuda:0")
    d = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, t)
    sph = c.get("sphere")
    X, F, FB, FL = d(fs.xyz), d(c["force"]), d(fs.fiber, torch.int32), d(fs.length)
    if sph is not None:
        trg = np.concatenate([fs.xyz, sph.xyz], axis=1)
        sl_self = np.concatenate([np.arange(fs.n), -np.ones(sph.n, dtype=np.int64)])
        dl_self = np.concatenate([-np.ones(fs.n, dtype=np.int64), np.arange(sph.n)])
        n_t = trg.shape[1]
        T, SS, DS = d(trg), d(sl_self, torch.int64), d(dl_self, torch.int64)
        sx, sn, sw, sq = d(sph.xyz), d(sph.normal), d(sph.weight), d(c["q"])
        pairs = {"sl": n_t * fs.n - fs.n, "dl": n_t * sph.n - sph.n}
    else:
        n_t = fs.n
        pairs = {"sl": fs.n * (fs.n - 1)}
    out = torch.empty((3, n_t), dtype=torch.float64, device=dev)

    def run_sum(which, mixed):
        if which == "sl" and sph is not None:
            S.sl_eval(X, F, src_fiber=FB, fiber_len=FL, eps=fs.eps, trg_xyz=T, trg_self=SS,
                      mixed=mixed, out=out)
        elif which == "sl":
            S.sl_eval(X, F, src_fiber=FB, fiber_len=FL, eps=fs.eps, mixed=mixed, out=out)
        else:
            S.dl_eval(sx, sn, sw, sq, trg_xyz=T, trg_self=DS, mixed=mixed, accumulate=True,
                      out=out)

    res = {"targets": n_t, "pairs": pairs}
    u = {}
    for mixed in (True, False):
        tag = "mixed" if mixed else "fp64"
        res[tag] = {}
        for which in pairs:
            # warm up for at least 0.25 s of this sum (the clock ramps up after the host
            # has generated the workload), then time `steps` calls
            tw = time.perf_counter()
            k = 0
            while k < warmup or time.perf_counter() - tw < 0.25:
                run_sum(which, mixed)
                k += 1
                if k % 8 == 0:
                    torch.cuda.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                run_sum(which, mixed)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            # the pair kernel alone (the library's HIP events around each launch), in a
            # second timed pass so that the events do not touch the whole-call time
            S.profile_enable(True)
            S.profile_read()
            for _ in range(steps):
                run_sum(which, mixed)
            torch.cuda.synchronize()
            kms, nk = S.profile_read()
            S.profile_enable(False)
            kt = kms / max(nk, 1) / 1e3
            fpp = FLOPS_PER_PAIR_SL if which == "sl" else FLOPS_PER_PAIR_DL
            peak = PEAK_FP32 if mixed else PEAK_FP64
            res[tag][which] = {"ms": round(dt * 1e3, 4),
                               "gpair_per_s": round(pairs[which] / dt / 1e9, 1),
                               "frac_of_peak": round(pairs[which] * fpp / dt / 1e12 / peak, 3),
                               "kernel_ms": round(kt * 1e3, 4),
                               "kernel_gpair_per_s": round(pairs[which] / kt / 1e9, 1),
                               "kernel_frac_of_peak": round(pairs[which] * fpp / kt / 1e12 / peak, 3)}
        run_sum("sl", mixed)
        if sph is not None:
            run_sum("dl", mixed)
        torch.cuda.synchronize()
        u[mixed] = out.cpu().numpy()       # SL (+ DL) of one step
    res["err_mixed_vs_fp64_relmax"] = float(
        f"{np.abs(u[True] - u[False]).max() / np.abs(u[False]).max():.3e}")
    log_fn(f"{name}: {res}")
    return res


def serving_run(S, n_req, log_fn, step_pairs=0, mixed=True, rate=0.0):
    """One Poisson stream of n_req mobility-solve requests through a session (64 slots,
    4 GiB), at `rate` requests/s or, when 0, at 0.7 x the capacity a calibration burst
    measures.  Latency is submit -> result, as the session's own clock records it."""
    from paper_1602_05650_amd import workloads as W
    reqs = [W.serving_request(3, rid) for rid in range(n_req)]
    pairs = sum(r["iters"] * r["fibers"].n * (r["fibers"].n - r["fibers"].nodes_per_fiber)
                for r in reqs)

    def submit(sess, r):
        fs = r["fibers"]
        return sess.submit(fs.xyz, fs.tangent, fs.length, r["rhs"], fs.nodes_per_fiber, fs.eps,
                           r["iters"], tag=r["rid"])

    with S.Session(hbm_budget_bytes=4 << 30, max_slots=64, mixed=mixed,
                   step_pairs=int(step_pairs)) as sess:
        # warm-up (arena, graph capture), then calibration: a burst of 48 requests drawn
        # like the stream (other ids) saturates the session; capacity = requests/s
        for t in [submit(sess, W.serving_request(3, 20000 + i, n_fib=32, iters=20))
                  for i in range(4)]:
            sess.wait(t)
        cal = [W.serving_request(3, 10000 + i) for i in range(48)]
        t0 = time.perf_counter()
        ts = [submit(sess, r) for r in cal]
        for t in ts:
            sess.wait(t)
        t_cal = time.perf_counter() - t0
        cap = len(cal) / t_cal
        cal_pairs = sum(r["iters"] * r["fibers"].n * (r["fibers"].n - r["fibers"].nodes_per_fiber) for r in cal)
        rate = rate if rate > 0 else 0.7 * cap
        arrivals = W.serving_stream(3, n_req, rate)
        log_fn(f"serving ({'mixed' if mixed else 'fp64'}): capacity {cap:.1f} req/s (calibration), "
               f"Poisson rate {rate:.1f} req/s, {n_req} requests")
        tickets = [None] * n_req

        def producer():
            start = time.perf_counter()
            for i, r in enumerate(reqs):
                dt = arrivals[i] - (time.perf_counter() - start)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = submit(sess, r)

        th = threading.Thread(target=producer)
        t_start = time.perf_counter()
        th.start()
        lat = []
        for i in range(n_req):
            while tickets[i] is None:
                time.sleep(0.0005)
            _, st = sess.wait(tickets[i])
            lat.append((st["t_finish_ns"] - st["t_submit_ns"]) * 1e-6)
            if (i + 1) % 500 == 0:
                log_fn(f"serving: {i + 1}/{n_req} requests done")
        th.join()
        wall = time.perf_counter() - t_start
    lat = np.array(lat)
    return {
        "requests": n_req, "rate_req_per_s": round(rate, 2), "capacity_req_per_s": round(cap, 2),
        "capacity_gpair_per_s": round(cal_pairs / t_cal / 1e9, 1),
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "mean_ms": round(float(lat.mean()), 2),
        "throughput_req_per_s": round(n_req / wall, 2),
        "gpair_per_s": round(pairs / wall / 1e9, 1),
        "precision": "mixed sums, FP64 GMRES" if mixed else "FP64 sums, FP64 GMRES",
        "hbm_budget_gib": 4, "max_slots": 64,
        "step_pairs": ("library default" if step_pairs == 0 else
                       "whole matvec" if step_pairs < 0 else int(step_pairs)),
        "workload": "Poisson stream; N_f log-uniform [32, 2048] fibers x {16,32,64} nodes; "
                    "20-60 GMRES iterations; same-fiber excluded, Clenshaw-Curtis weights",
    }


def serving_cpu(n_req, n_sample, log_fn):
    """The oracle on n_sample seeded requests of the serving stream: one GMRES iteration
    of each (operator application, Gram-Schmidt, Givens) timed on all host threads, and
    the time of the request's whole iteration budget extrapolated from it."""
    import oracle
    from paper_1602_05650_amd import workloads as W
    oracle.build(force=False)
    nthreads = max(1, min(16, os.cpu_count() or 1))
    ids = W.subsample(33, n_req, n_sample)
    t_meas, t_extrap, pairs = 0.0, 0.0, 0
    for rid in ids:
        r = W.serving_request(3, int(rid))
        fs = r["fibers"]
        t0 = time.perf_counter()
        oracle.mobility_solve(r["rhs"], fs.xyz, fs.tangent, fs.fiber, fs.length, fs.nodes_per_fiber,
                              fs.eps, 1, nthreads=nthreads)
        dt = time.perf_counter() - t0
        t_meas += dt
        t_extrap += dt * r["iters"]
        pairs += r["iters"] * fs.n * (fs.n - fs.nodes_per_fiber)
    out = {"kind": "oracle", "cores": nthreads, "requests": [int(i) for i in ids],
           "measured_s": round(t_meas, 2),
           "extrapolated_s_per_request": round(t_extrap / len(ids), 2),
           "extrapolated_gpair_per_s": round(pairs / t_extrap / 1e9, 4),
           "sample": f"{len(ids)} seeded requests of the stream, one GMRES iteration each "
                     "(measured); their whole iteration budgets extrapolated as iterations x "
                     "that time"}
    log_fn(f"serving cpu oracle: {out}")
    return out


FLOPS_PER_PAIR_NONLOCAL = 36   # K_delta node pair: 3 sub, |r|^2 5, a 3, r.f 5, b 2, 3 x (2 fma) 12, s-term 6


def nonlocal_run(S, torch, log_fn, n_fib=2048, nodes=64, iters=20, delta=0.01):
    """The nonlocal self term and the block-Jacobi preconditioner on the largest serving
    request shape: K_delta alone (node pairs/s), then one-shot solves with the local
    operator, with K_delta, and with K_delta and block-Jacobi preconditioning."""
    from paper_1602_05650_amd import workloads as W
    req = W.serving_request(3, 40000, n_fib=n_fib, nodes=nodes, iters=iters)
    fs = req["fibers"]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    X, T, L, V = d(fs.xyz), d(fs.tangent), d(fs.length), d(req["rhs"])
    out = torch.empty_like(V)
    n = fs.n
    pairs = n * (nodes - 1)
    for _ in range(3):
        S.nonlocal_sbt(X, T, L, V, nodes, delta, out=out)
    torch.cuda.synchronize()
    reps = 50
    t0 = time.perf_counter()
    for _ in range(reps):
        S.nonlocal_sbt(X, T, L, V, nodes, delta, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res = {"workload": f"{n_fib} fibers x {nodes} nodes ({n} points), delta={delta}",
           "k_delta": {"ms": round(dt * 1e3, 4), "node_pairs": pairs,
                       "gpair_per_s": round(pairs / dt / 1e9, 2),
                       "tflops_counted": round(pairs * FLOPS_PER_PAIR_NONLOCAL / dt / 1e12, 2)}}
    log_fn(f"K_delta: {dt * 1e3:.3f} ms for {pairs} node pairs")
    sl_pairs = iters * n * (n - nodes)
    for tag, dl, pre in (("local_operator", None, "local"), ("nonlocal_local_precond", delta, "local"),
                         ("nonlocal_block_precond", delta, "block")):
        S.mobility_solve(X, T, L, V, nodes, fs.eps, 2, mixed=True, delta=dl, precond=pre)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f, r, it = S.mobility_solve(X, T, L, V, nodes, fs.eps, iters, mixed=True, delta=dl,
                                    precond=pre)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        beta = float(torch.linalg.vector_norm(V))
        res[tag] = {"ms": round(dt * 1e3, 2), "iterations": it,
                    "relative_residual": float(f"{r / beta:.3e}"),
                    "sl_gpair_per_s": round(sl_pairs / dt / 1e9, 1)}
        log_fn(f"solve {tag}: {dt * 1e3:.1f} ms, {it} iterations, residual {r / beta:.2e}")
    return res


def particles_run(S, torch, log_fn, iters=30, reps=5):
    """Confined rigid spheres (second-kind boundary integrals): the concentric-sphere
    drag and torque against their closed forms, and a confined suspension of spheres
    timed per whole solve (set-up, iterations, solution; median of `reps` solves on
    device-resident inputs)."""
    import math
    from paper_1602_05650_amd import workloads as W
    mu = 1.0

    def sph(nt, nph, R, c=(0.0, 0.0, 0.0)):
        s = W.sphere_surface(nt, nph, R)
        return s.xyz + np.asarray(c, float)[:, None], s.normal, s.weight

    res = {}
    a, b = 1.0, 2.0
    lam = a / b
    per = sph(48, 96, b)
    part = (*sph(24, 48, a), np.zeros(3))
    U, Om, q, r, it = S.particle_solve([part], np.array([[0.0], [0.0], [1.0]]),
                                       np.array([[0.0], [0.0], [1.0]]), periphery=per, mu=mu,
                                       iters=iters)
    gam = 6 * math.pi * mu * a * 4 * (1 - lam ** 5) / (4 - 9 * lam + 10 * lam ** 3 - 9 * lam ** 5 + 4 * lam ** 6)
    res["concentric"] = {
        "points": f"periphery 48x96 = 4608 (R = 2), sphere 24x48 = 1152 (a = 1)",
        "drag_rel_error": float(f"{abs(float(U[2, 0]) * gam - 1.0):.3e}"),
        "torque_rel_error": float(f"{abs(float(Om[2, 0]) * 8 * math.pi * mu * a ** 3 / (1 - lam ** 3) - 1.0):.3e}"),
        "iterations": it}
    # a confined suspension: C1's periphery (64 x 96 on R = 5) and 16 spheres
    rng = np.random.default_rng(11)
    centres = []
    while len(centres) < 16:
        c = rng.uniform(-3.2, 3.2, 3)
        if np.linalg.norm(c) < 3.3 and all(np.linalg.norm(c - o) > 1.3 for o in centres):
            centres.append(c)
    parts = [(*sph(16, 32, 0.5, c), c) for c in centres]
    per = sph(64, 96, 5.0)
    F = rng.standard_normal((3, 16))
    L = rng.standard_normal((3, 16))
    ms = 6144 + 16 * 512
    pairs = ms * ms - ms          # double-layer pairs per operator application
    # the geometry, forces and torques resident on the device before the timed solves
    geom = S.ParticleGeometry(parts, per)
    Fd = torch.from_numpy(F).cuda()
    Ld = torch.from_numpy(L).cuda()
    for mixed in (False, True):
        S.particle_solve(geom, Fd, Ld, mu=mu, iters=2, mixed=mixed)
        torch.cuda.synchronize()
        dts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            U, Om, q, r, it = S.particle_solve(geom, Fd, Ld, mu=mu, iters=iters, mixed=mixed)
            torch.cuda.synchronize()
            dts.append(time.perf_counter() - t0)
        dt = float(np.median(dts))
        res["suspension_" + ("mixed" if mixed else "fp64")] = {
            "points": f"periphery 6144 (R = 5) + 16 spheres x 512 (a = 0.5) = {ms}",
            "ms": round(dt * 1e3, 2), "ms_min": round(min(dts) * 1e3, 2), "solves": reps,
            "iterations": it, "ms_per_iteration": round(dt * 1e3 / it, 3),
            "residual": float(f"{r:.3e}"),
            "dl_gpair_per_s": round(pairs * it / dt / 1e9, 1)}
        log_fn(f"particles {('mixed' if mixed else 'fp64')}: {dt * 1e3:.1f} ms (median of {reps}), "
               f"{it} iterations")
    return res


def fiberstep_run(S, torch, log_fn, reps=3, iters=60, tol=1e-5):
    """One implicit backward-Euler step of a sedimenting suspension of 2048 free bent
    fibers x 32 nodes (the paper's GMRES study: up to 2048 fibers of 31 points, GMRES
    tolerance 1e-5, dt = 1e-3 tau_E): time per step, GMRES iterations, and the share of
    the single-layer pair-sum kernels (the other fibers' flow, once per iteration and
    once for the right-hand side)."""
    from paper_1602_05650_amd import workloads as W
    c = W.config_step()
    fs = c["fibers"]
    n, N = fs.nodes_per_fiber, fs.n
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xyz, flen, fext = d(fs.xyz), d(fs.length), d(c["f_ext"])
    kw = dict(mu=c["mu"], iters=iters, tol=tol, near_r=NEAR_R)
    pairs = N * (N - n)                     # other-fiber pairs per operator application
    res = {"workload": f"{fs.n_fib} free bent fibers x {n} CGL nodes = {N} nodes in a ball of "
                       f"radius 5, L = 1, eps = {c['eps']}, E = {c['E']}, dt = {c['dt']:.4e} "
                       f"(1e-3 tau_E), sedimenting, GMRES tol {tol}"}
    for mixed in (False, True):
        S.fiber_step(xyz, flen, fext, n, c["eps"], c["E"], c["dt"], mixed=mixed, **dict(kw, iters=2))
        torch.cuda.synchronize()
        S.profile_read()
        S.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            X1, T1, r, it = S.fiber_step(xyz, flen, fext, n, c["eps"], c["E"], c["dt"], mixed=mixed, **kw)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        S.profile_enable(False)
        kms, launches = S.profile_read()
        tag = "mixed" if mixed else "fp64"
        res[tag] = {"ms_per_step": round(sec * 1e3, 2), "gmres_iterations": it,
                    "operator_applications": it + 1,
                    "pair_sum_ms": round(kms / reps, 2),
                    "pair_sum_share": round(kms / reps / (sec * 1e3), 3),
                    "pair_sum_gpair_per_s": round(pairs * (it + 1) / (kms / reps * 1e-3) / 1e9, 1),
                    "max_displacement": float(f"{float((X1 - xyz).abs().max()):.4e}"),
                    "max_tension": float(f"{float(T1.abs().max()):.4e}")}
        log_fn(f"fiber step {tag}: {sec * 1e3:.1f} ms, {it} iterations, pair sums "
               f"{kms / reps:.1f} ms")
    return res


def far_run(S, torch, log_fn, degree=6, theta=0.7, reps=3):
    """The solvers' u_bar sums through a treecode plan (one per call) against the direct
    sums: the 2048 x 32 implicit step (GMRES to 1e-5) and the largest serving request
    shape (2048 fibers x 64 nodes, 60 GMRES iterations) as a one-shot mobility solve;
    mixed sums; time, iterations and the result's difference from the direct one."""
    from paper_1602_05650_amd import workloads as W
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    far = (degree, theta)
    res = {"tree": {"degree": degree, "theta": theta}}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    c = W.config_step()
    fs = c["fibers"]
    n = fs.nodes_per_fiber
    a = (d(fs.xyz), d(fs.length), d(c["f_ext"]), n, c["eps"], c["E"], c["dt"])
    kw = dict(mu=c["mu"], iters=60, tol=1e-5, mixed=True)
    t_dir, (X0, _, _, i0) = timed(lambda: S.fiber_step(*a, **kw))
    t_far, (X1, _, _, i1) = timed(lambda: S.fiber_step(*a, far=far, **kw))
    dX0, dX1 = X0 - a[0], X1 - a[0]
    res["fiber_step_2048x32"] = {
        "direct_ms": round(t_dir * 1e3, 2), "tree_ms": round(t_far * 1e3, 2),
        "iterations": [i0, i1],
        "dX_rel_diff": float(f"{float((dX1 - dX0).abs().max() / dX0.abs().max()):.3e}")}
    log_fn(f"far field, fiber step: direct {t_dir * 1e3:.1f} ms, tree {t_far * 1e3:.1f} ms")
    req = W.serving_request(3, 40000, n_fib=2048, nodes=64, iters=60)
    fs = req["fibers"]
    b = (d(fs.xyz), d(fs.tangent), d(fs.length), d(req["rhs"]), fs.nodes_per_fiber, fs.eps, 60)
    t_dir, (f0, r0, j0) = timed(lambda: S.mobility_solve(*b, mixed=True))
    t_far, (f1, r1, j1) = timed(lambda: S.mobility_solve(*b, mixed=True, far=far))
    res["mobility_solve_2048x64_60it"] = {
        "direct_ms": round(t_dir * 1e3, 2), "tree_ms": round(t_far * 1e3, 2),
        "iterations": [j0, j1],
        "f_rel_diff": float(f"{float(torch.linalg.vector_norm(f1 - f0) / torch.linalg.vector_norm(f0)):.3e}")}
    log_fn(f"far field, mobility solve: direct {t_dir * 1e3:.1f} ms, tree {t_far * 1e3:.1f} ms")
    return res


def tree_run(S, torch, log_fn, degree=6, theta=0.7, leaf=128, reps=10):
    """Treecode single-layer sum on the spindle and the large confined fiber set: plan
    build time, evaluation time (mixed and FP64; mixed with same-fiber exclusion),
    interactions per second, and the error against the direct GPU sum on all targets;
    then the double layer on a sphere."""
    from paper_1602_05650_amd import workloads as W
    res = {"degree": degree, "theta": theta, "leaf_size": leaf}
    for name, gen in (("spindle_262k", W.config2), ("confined_524k_fibers", W.config4)):
        c = gen()
        fs = c["fibers"]
        d = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
        X, F, FB, FL = d(fs.xyz), d(c["force"]), d(fs.fiber, torch.int32), d(fs.length)
        n = fs.n
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T = S.Tree(X, degree=degree, theta=theta, leaf_size=leaf)
        t_plan = time.perf_counter() - t0
        info = T.info()
        out = torch.empty((3, n), dtype=torch.float64, device="cuda")
        ref = S.sl_eval(X, F, src_fiber=FB, fiber_len=FL, eps=fs.eps)       # direct FP64
        entry = {"points": n, "plan_s": round(t_plan, 3),
                 "pair_work_vs_direct": round((info["proxy_pairs"] + info["direct_pairs"]) / (n * (n - 1)), 4),
                 **info}
        for mixed in (True, False):
            T.sl_eval(F, src_fiber=FB, fiber_len=FL, eps=fs.eps, mixed=mixed, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                T.sl_eval(F, src_fiber=FB, fiber_len=FL, eps=fs.eps, mixed=mixed, out=out)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            err = float((out - ref).abs().max() / ref.abs().max())
            entry["mixed" if mixed else "fp64"] = {
                "ms": round(dt * 1e3, 3), "interactions_per_s_g": round(n * (n - 1) / dt / 1e9, 1),
                "err_vs_direct_relmax": float(f"{err:.3e}")}
            log_fn(f"tree {name} {'mixed' if mixed else 'fp64'}: {dt * 1e3:.2f} ms, err {err:.2e}")
        # same-fiber exclusion, mixed, against the direct FP64 sum with the same exclusion
        ref = S.sl_eval(X, F, src_fiber=FB, fiber_len=FL, eps=fs.eps, excl="fiber")
        kw = dict(src_fiber=FB, fiber_len=FL, eps=fs.eps, mixed=True, excl_fiber=True, out=out)
        T.sl_eval(F, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            T.sl_eval(F, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        err = float((out - ref).abs().max() / ref.abs().max())
        entry["mixed_excl_fiber"] = {"ms": round(dt * 1e3, 3), "err_vs_direct_relmax": float(f"{err:.3e}")}
        log_fn(f"tree {name} mixed, same-fiber exclusion: {dt * 1e3:.2f} ms, err {err:.2e}")
        T.close()
        res[name] = entry
    res["double_layer_sphere_393k"] = tree_dl_run(S, torch, log_fn)
    return res


def tree_dl_run(S, torch, log_fn, degree=8, theta=0.5, leaf=64, reps=5):
    """Treecode double-layer sum on a sphere of radius 5 with 512 x 768 quadrature points
    and random density, beside the direct sum: times (FP64 and mixed) and the errors
    against the direct FP64 sum."""
    from paper_1602_05650_amd import workloads as W
    sph = W.sphere_surface(512, 768, 5.0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64)
    X, N, Wt = d(sph.xyz), d(sph.normal), d(sph.weight)
    Q = d(np.random.default_rng(4).standard_normal((3, sph.n)))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    ref = S.dl_eval(X, N, Wt, Q)
    t_direct = timed(lambda: S.dl_eval(X, N, Wt, Q, out=ref))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = S.Tree(X, degree=degree, theta=theta, leaf_size=leaf)
    t_plan = time.perf_counter() - t0
    out = torch.empty_like(ref)
    t_tree = timed(lambda: T.dl_eval(N, Wt, Q, out=out))
    err = float((out - ref).abs().max() / ref.abs().max())
    t_tree_m = timed(lambda: T.dl_eval(N, Wt, Q, out=out, mixed=True, near_r=0.4))
    err_m = float((out - ref).abs().max() / ref.abs().max())
    out_d = torch.empty_like(ref)
    t_direct_m = timed(lambda: S.dl_eval(X, N, Wt, Q, mixed=True, near_r=0.4, out=out_d))
    err_dm = float((out_d - ref).abs().max() / ref.abs().max())
    entry = {"points": sph.n, "degree": degree, "theta": theta, "leaf_size": leaf, "plan_s": round(t_plan, 3),
             **T.info(), "tree_ms": round(t_tree * 1e3, 3), "direct_fp64_ms": round(t_direct * 1e3, 3),
             "err_vs_direct_relmax": float(f"{err:.3e}"), "tree_mixed_ms": round(t_tree_m * 1e3, 3),
             "direct_mixed_ms": round(t_direct_m * 1e3, 3), "mixed_near_r": 0.4,
             "mixed_err_vs_direct_relmax": float(f"{err_m:.3e}"),
             "direct_mixed_err_vs_direct_relmax": float(f"{err_dm:.3e}")}
    T.close()
    log_fn(f"tree double layer {sph.n}: {t_tree * 1e3:.2f} ms vs direct {t_direct * 1e3:.2f} ms, err {err:.2e}; "
           f"mixed {t_tree_m * 1e3:.2f} ms (err {err_m:.2e}) vs direct mixed {t_direct_m * 1e3:.2f} ms "
           f"(err {err_dm:.2e})")
    return entry


def cpu_baseline(c, seconds, log_fn, other=True):
    """The oracle (plain FP64 double loop, OpenMP over targets) on seeded samples of the
    headline workload: about 60% of `seconds` on all host threads, 25% on one thread;
    then, if `other`, the smaller workloads in full and a large one on a sample."""
    import oracle
    oracle.build(force=False)
    fs = c["fibers"]
    nthreads = max(1, min(16, os.cpu_count() or 1))
    from paper_1602_05650_amd import workloads as W
    idx = W.subsample(2, fs.n, 65536)
    kw = dict(src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps, excl=1)

    def timed(n_t, threads):
        t0 = time.perf_counter()
        oracle.sl(fs.xyz, c["force"], trg_xyz=fs.xyz[:, idx[:n_t]], trg_self=idx[:n_t],
                  nthreads=threads, **kw)
        return time.perf_counter() - t0

    def sized(threads, budget):
        n_t = 64 * threads
        dt = timed(n_t, threads)
        while dt < 0.5 and n_t < len(idx):       # calibrate on a run of at least 0.5 s
            n_t = min(len(idx), n_t * 4)
            dt = timed(n_t, threads)
        n_t = int(min(len(idx), max(n_t, n_t * budget / max(dt, 1e-6))))
        return n_t, timed(n_t, threads)

    n_t, dt = sized(nthreads, 0.6 * seconds)
    pairs = n_t * (fs.n - 1)
    log_fn(f"cpu oracle: {n_t} targets x {fs.n} sources in {dt:.2f} s on {nthreads} threads")
    n1, dt1 = sized(1, 0.25 * seconds)
    log_fn(f"cpu oracle: {n1} targets x {fs.n} sources in {dt1:.2f} s on 1 thread")
    out = {"value": round(pairs / dt / 1e9, 4), "unit": "Gpair/s", "cores": nthreads,
           "kind": "oracle",
           "sample": f"{n_t} seeded targets of the spindle workload x all {fs.n} sources, "
                     f"FP64 brute force, self-pairs excluded ({dt:.1f} s)",
           "single_thread": {"value": round(n1 * (fs.n - 1) / dt1 / 1e9, 4), "unit": "Gpair/s",
                             "cores": 1, "sample": f"{n1} seeded targets ({dt1:.1f} s)"}}
    if other:
        out["other_workloads"] = {}
        for name, label, n_sample in (("c0", "cloud_512", None), ("c1", "confined_32k", None),
                                      ("c4", "confined_524k", 4096)):
            out["other_workloads"][label] = cpu_config(load_config(name), n_sample, nthreads)
            log_fn(f"cpu oracle {label}: {out['other_workloads'][label]}")
    return out


def cpu_config(c, n_sample, nthreads):
    """Oracle Gpair/s of the single (and double) layer of one workload to all targets, or
    to n_sample seeded targets of each kind."""
    import oracle
    from paper_1602_05650_amd import workloads as W
    fs = c["fibers"]
    sph = c.get("sphere")
    fi = np.arange(fs.n) if n_sample is None else W.subsample(4, fs.n, n_sample)
    res = {"targets": "all" if n_sample is None else f"{len(fi)} fiber"}
    t0 = time.perf_counter()
    oracle.sl(fs.xyz, c["force"], src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps, excl=1,
              trg_xyz=fs.xyz[:, fi], trg_self=fi, nthreads=nthreads)
    t_sl = time.perf_counter() - t0
    pairs_sl = len(fi) * (fs.n - 1)
    if sph is not None:
        si = np.arange(sph.n) if n_sample is None else W.subsample(5, sph.n, n_sample)
        if n_sample is not None:
            res["targets"] += f" + {len(si)} sphere"
        t0 = time.perf_counter()
        oracle.sl(fs.xyz, c["force"], src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps,
                  excl=1, trg_xyz=sph.xyz[:, si], nthreads=nthreads)
        oracle.dl(sph.xyz, sph.normal, sph.weight, c["q"], trg_xyz=fs.xyz[:, fi],
                  subtract=False, nthreads=nthreads)
        oracle.dl(sph.xyz, sph.normal, sph.weight, c["q"], trg_xyz=sph.xyz[:, si], trg_self=si,
                  subtract=True, nthreads=nthreads)
        t_rest = time.perf_counter() - t0
        pairs_sl += len(si) * fs.n
        pairs_dl = (len(fi) + len(si)) * sph.n - len(si)
        res["sl_plus_dl_gpair_per_s"] = round((pairs_sl + pairs_dl) / (t_sl + t_rest) / 1e9, 4)
        res["seconds"] = round(t_sl + t_rest, 2)
    else:
        res["sl_gpair_per_s"] = round(pairs_sl / t_sl / 1e9, 4)
        res["seconds"] = round(t_sl, 3)
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a ROCm GPU")
    from paper_1602_05650_amd import stokes as S
    from paper_1602_05650_amd import workloads as W

    if args.only == "nonlocal":      # nonlocal-term section alone (for profiling it)
        print(json.dumps({"nonlocal": nonlocal_run(S, torch, log)}), flush=True)
        return
    if args.only == "treecode":      # treecode section alone (for profiling it)
        print(json.dumps({"treecode": tree_run(S, torch, log)}), flush=True)
        return
    if args.only == "fiberstep":     # implicit fiber time step alone (for profiling it)
        print(json.dumps({"fiber_step": fiberstep_run(S, torch, log)}), flush=True)
        return
    if args.only == "workloads":     # the --extra workloads alone (for profiling them)
        names = [e for e in args.extra.split(",") if e in ("c0", "c1", "c4")]
        print(json.dumps({"other_workloads": {e: config_run(S, torch, e, 200 if e == "c0" else 10, 3, log)
                                              for e in names}}), flush=True)
        return
    if args.only == "far":           # the solvers with the treecode far field
        print(json.dumps({"far_field_in_solvers": far_run(S, torch, log)}), flush=True)
        return
    if args.only == "particles":     # rigid-particle section alone (for profiling it)
        print(json.dumps({"particles": particles_run(S, torch, log)}), flush=True)
        return
    if args.only == "none":          # serving run alone (for profiling it)
        print(json.dumps({"serving": serving_run(S, args.serving_requests, log, args.step_pairs,
                                                 not args.serving_fp64, args.serving_rate)}), flush=True)
        return
    if args.only == "serving_cpu":   # the oracle's serving leg alone
        print(json.dumps({"serving_cpu": serving_cpu(args.serving_requests, 10, log)}), flush=True)
        return
    t_gen = time.perf_counter()
    c = W.config2()
    fs = c["fibers"]
    n = fs.n
    rng = np.random.Generator(np.random.PCG64([2, 40]))
    n_forces = max(1, min(args.steps, 40))
    forces_h = [rng.standard_normal((3, n)) / fs.length[fs.fiber][None, :] for _ in range(n_forces)]
    forces_h[0] = c["force"]
    dev = torch.device("cuda:0")
    xyz = torch.from_numpy(fs.xyz).to(dev)
    fib = torch.from_numpy(fs.fiber).to(dev)
    flen = torch.from_numpy(fs.length).to(dev)
    forces = [torch.from_numpy(f).to(dev) for f in forces_h]
    torch.cuda.synchronize()
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)          # reads and writes exactly MIB MiB each
        torch.cuda.synchronize()
        del src, dst
    log(f"spindle workload: {n} points, {fs.n_fib} fibers, generated in "
        f"{time.perf_counter() - t_gen:.1f} s")
    pairs = n * (n - 1)

    res = {}
    for mixed in ([True, False] if args.only == "both" else [args.only == "mixed"]):
        sec, kms, launches, first = time_matvecs(S, torch, xyz, forces, fib, flen, fs.eps, mixed,
                                                 args.steps, args.warmup)
        res[mixed] = dict(sec=sec, kms=kms, launches=launches, first=first)
        tag = "mixed" if mixed else "fp64"
        log(f"{tag}: {args.steps} matvecs in {sec * 1e3:.1f} ms -> "
            f"{args.steps * pairs / sec / 1e9:.1f} Gpair/s; kernel {kms / max(launches, 1):.3f} ms "
            f"x {launches}")
    head = True if True in res else False
    r = res[head]
    value = args.steps * pairs / r["sec"] / 1e9
    k_avg = r["kms"] / max(r["launches"], 1) * 1e-3
    achieved = pairs * FLOPS_PER_PAIR_SL / k_avg / 1e12
    peak = PEAK_FP32 if head else PEAK_FP64
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gpair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["sec"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head else "f64",
        "data": "synthetic",
        "config": {
            "workload": "spindle: 4096 fibers x 64 CGL nodes = 262144 points, poles (+-4,0,0), "
                        "L~U(1,6), eps=0.005, single layer (Stokeslet + doublet) to all nodes, "
                        "self-pairs excluded, one matvec per step with a fresh seeded force",
            "n_points": n, "pairs_per_step": pairs,
            "path": "mixed FP32+Kahan, FP64 near pairs" if head else "FP64",
            "near_r": NEAR_R,
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 2),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": (TRAFFIC["bytes"] if head and kernel_digest() == TRAFFIC["digest"]
                        else None),
            "kernel": "sl_mixed_kernel" if head else "sl_fp64_kernel",
            "flops_per_pair": FLOPS_PER_PAIR_SL,
            "kernel_ms": round(k_avg * 1e3, 4),
            "counter_flops_per_pair": counter_fpp(head),
            "counter_frac": (round(pairs * counter_fpp(head) / k_avg / 1e12 / peak, 4)
                             if counter_fpp(head) else None),
            "peak_basis": "published vector peak of the kernel's precision (FP32 for the mixed "
                          "kernel: 256 CUs x 128 FP32 lanes x 2 flops x 2.4 GHz)",
        },
    }
    if True in res and False in res:
        f64 = res[False]
        k64 = f64["kms"] / max(f64["launches"], 1) * 1e-3
        a64 = pairs * FLOPS_PER_PAIR_SL / k64 / 1e12
        u32 = res[True]["first"].cpu().numpy()
        u64 = f64["first"].cpu().numpy()
        out["fp64"] = {
            "value": round(args.steps * pairs / f64["sec"] / 1e9, 2), "unit": "Gpair/s",
            "ms_per_step": round(f64["sec"] / args.steps * 1e3, 3),
            "kernel_ms": round(k64 * 1e3, 4), "achieved_tflops": round(a64, 2),
            "frac_of_fp64_peak": round(a64 / PEAK_FP64, 4),
            "counter_flops_per_pair": counter_fpp(False),
            "counter_frac": (round(pairs * counter_fpp(False) / k64 / 1e12 / PEAK_FP64, 4)
                             if counter_fpp(False) else None),
        }
        out["mixed_over_fp64"] = round(f64["sec"] / res[True]["sec"], 3)
        out["err_mixed_vs_fp64_relmax"] = float(f"{np.abs(u32 - u64).max() / np.abs(u64).max():.3e}")
    extra = [e for e in args.extra.split(",") if e in ("c0", "c1", "c4")]
    if extra and args.only == "both":
        out["other_workloads"] = {
            {"c0": "cloud_512", "c1": "confined_32k", "c4": "confined_524k"}[e]:
            config_run(S, torch, e, 200 if e == "c0" else 10, 3, log) for e in extra}
    if extra and args.only == "both":
        out["nonlocal"] = nonlocal_run(S, torch, log)
        out["particles"] = particles_run(S, torch, log)
        out["treecode"] = tree_run(S, torch, log)
        out["fiber_step"] = fiberstep_run(S, torch, log)
        out["far_field_in_solvers"] = far_run(S, torch, log)
    if not args.no_serving:
        out["serving"] = {}
        for mixed in (True, False):
            tag = "mixed" if mixed else "fp64"
            try:
                out["serving"][tag] = serving_run(S, args.serving_requests, log, args.step_pairs,
                                                  mixed, args.serving_rate)
            except Exception as e:  # report, do not hide
                out["serving"][tag] = {"error": repr(e)}
                log(f"serving run ({tag}) failed:", repr(e))
        if not args.no_cpu:
            out["serving"]["cpu_oracle"] = serving_cpu(args.serving_requests, 10, log)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_seconds, log, not args.no_cpu_other)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

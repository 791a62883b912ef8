"""Benchmark: Landau-gauge overrelaxation on 32^4, mixed precision vs FP64.

Workload (one GPU): smooth SU(3) configurations U_mu(x) = h(x) exp(i 0.5
sum_a lambda_a xi_a) h(x+mu)^dag on a 32^4 lattice, seeds 2001-2004, fixed to
Landau gauge by overrelaxation (omega = 1.7) until theta < 1e-12, checked
every 20 sweeps (the check costs about half a sweep; a unit overshoots by at
most 19 sweeps, under 0.4% of a fix).

A step is one complete gauge fixing of one configuration (seeds in turn):
layout conversion of the device-resident natural-order FP64 input into the
FP32 12-real storage, the sweeps with their F/theta checks, and the final
FP64 reprojection and measurement.  The metric is OR site-updates per second
over the timed steps (sweeps x V / time); the line also carries the effective
HBM bandwidth, time-to-theta of the mixed and the plain FP64 (12-real) GPU
paths, the roofline of the half-sweep kernel (the launches of every 8th chunk
of sweeps timed with HIP events on the launch stream) and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (32, 32, 32, 32)
EPS = 0.5
SEEDS = (2001, 2002, 2003, 2004)
OMEGA = 1.7
TOL = 1e-12
CHECK = 20
REUNIT = 100
TAIL = 0.0           # FP64 update arithmetic below this theta (0: FP32 update throughout; Step 2 is FP64)
MAX_SWEEPS = 50000
TIME_EVERY = 8       # sampled kernel timing: the launches of every 8th chunk of CHECK sweeps
HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {"mixed": 768, "f64r12": 1536, "f64r18": 2304}  # 8 links loaded + stored


# Bytes per launch of the FP32-update half-sweep between L2 and the fabric
# (by launch shape "W/B/flags"), from rocprofv3 FETCH_SIZE and WRITE_SIZE
# passes over this workload, each scaled by what the counter reads for a
# plain 1 GiB device copy (profiles/k_sweep_landau_32x4_mixed_hbm_bytes.md).
# These counters count L2 misses sent to the memory side, Infinity-Cache
# hits included.  They hold for the kernel sources with the digest below;
# after any change of those sources the traffic is reported as null until
# the counters are taken again.
COUNTER_SOURCES = ("paper_1212_5221_amd/csrc/gf_sweep.hpp", "paper_1212_5221_amd/csrc/gf_device.hpp",
                   "paper_1212_5221_amd/csrc/gf_shared.hpp", "paper_1212_5221_amd/csrc/gf_variants.hpp",
                   "paper_1212_5221_amd/csrc/gf_sweep_table.hpp", "paper_1212_5221_amd/csrc/gf_sweep_inst.hip",
                   "paper_1212_5221_amd/build.py")
COUNTER_DIGEST = "079e1199447c65ec"
COUNTER_TRAFFIC = {"1/256/0": 402911937, "1/128/0": 402931194, "1/512/0": 402895355, "1/64/0": 403010040,
                   "2/256/0": 402935795}
# the same for the 48^4 lattice (non-temporal traffic, linear tile order;
# profiles/k_sweep_landau_48x4_mixed_beyond_cache.md)
COUNTER_TRAFFIC_48 = {"1/256/3": 2050320999, "1/128/3": 2052505301, "1/512/3": 2048528273, "1/64/3": 2057269007,
                      "2/128/3": 2057208470}


def kernel_digest():
    import hashlib
    d = hashlib.sha256()
    for f in COUNTER_SOURCES:
        d.update(f.encode())
        d.update(open(os.path.join(ROOT, f), "rb").read())
    return d.hexdigest()[:16]


def measured_traffic(shape_key, table=None):
    if COUNTER_DIGEST is None or kernel_digest() != COUNTER_DIGEST:
        return None
    return (COUNTER_TRAFFIC if table is None else table).get(shape_key)


def fp64_policy():
    upd = ("FP64 once theta < %g" % TAIL) if TAIL > 0 else "FP32 throughout"
    return ("F/theta reductions, applying G to the links, reprojection every %d sweeps; update arithmetic %s"
            % (REUNIT, upd))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_fixer(gf, storage):
    tail = TAIL if storage == "mixed" else 0.0
    fx = gf.GaugeFixer([DIMS], gauge="landau", storage=storage, reunit_every=REUNIT if storage == "mixed" else 0,
                       tail_theta=tail)
    fx.set_overrelax(OMEGA)
    return fx


def one_fix(fx, inp):
    """upload (device-resident natural layout) + fix; returns sweeps.  With
    FP32 storage and reprojection in use the sweeps end with the FP64
    reprojection of the links and a check of theta on the reprojected links
    (more sweeps if it no longer passes)."""
    fx.upload(0, inp)
    st, done = fx.sweep("or", max_sweeps=MAX_SWEEPS, tol=TOL, check_every=CHECK)
    return st, int(done[0])


def host_cpu():
    """CPU model, logical CPUs this process may run on, physical cores."""
    model, phys = None, set()
    try:
        cur = {}
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if "core id" in cur:
                    phys.add((cur.get("physical id"), cur["core id"]))
                cur = {}
                continue
            k, v = [x.strip() for x in line.split(":", 1)]
            cur[k] = v
            if k == "model name" and model is None:
                model = v
        if "core id" in cur:
            phys.add((cur.get("physical id"), cur["core id"]))
    except OSError:
        pass
    try:
        logical = len(os.sched_getaffinity(0))
    except AttributeError:
        logical = os.cpu_count()
    return {"model": model, "logical_cpus_available": logical, "physical_cores": len(phys) or None}


def cpu_baseline(budget_s=12.0, one_core_sweeps=20):
    """The oracle (FP64, OpenMP over the host cores) on a bounded sample: OR
    sweeps of the seed-2001 configuration until about budget_s seconds; then
    its rate on one core over a window of one_core_sweeps sweeps."""
    import ctypes

    import oracle as O
    from paper_1212_5221_amd import inputs as I
    U = I.smooth(DIMS, EPS, SEEDS[0])
    V = int(np.prod(DIMS))
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        gomp = None
    O.sweep(U, DIMS, "landau", "or", omega=OMEGA)  # warm-up (thread pool, pages)
    n = 0
    t0 = time.time()
    while True:
        O.sweep(U, DIMS, "landau", "or", omega=OMEGA)
        n += 1
        if time.time() - t0 > budget_s and n >= 2:
            break
    el = time.time() - t0
    # the OpenMP threads the oracle's parallel loops ran with
    threads = gomp.omp_get_max_threads() if gomp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": V * n / el, "unit": "site-updates/s", "cores": threads, "kind": "oracle",
           "sample": "%d Landau OR sweeps (omega 1.7) of the 32^4 seed-2001 configuration, FP64, %.1f s" % (n, el),
           "host": host_cpu()}
    # the same on one core (OpenMP limited to one thread for these sweeps)
    if gomp is not None:
        before = gomp.omp_get_max_threads()
        gomp.omp_set_num_threads(1)
        try:
            t0 = time.time()
            for _ in range(one_core_sweeps):
                O.sweep(U, DIMS, "landau", "or", omega=OMEGA)
            el1 = time.time() - t0
        finally:
            gomp.omp_set_num_threads(before)
        out["one_core"] = {"value": V * one_core_sweeps / el1, "cores": 1,
                           "sample": "%d sweeps, %.1f s" % (one_core_sweeps, el1)}
    return out


def warm_up(fx, upd, ms=30.0):
    """Untimed sweeps (update `upd`) for about `ms` milliseconds before a
    timed run: the first milliseconds of work after the GPU idled (a host
    copy, the autotuner's state save and restore) run at lower clocks."""
    n, spent = 1, 0.0
    while spent < ms * 1e-3:
        t0 = time.perf_counter()
        fx.sweep(upd, max_sweeps=n, tol=0.0, check_every=n)
        spent += time.perf_counter() - t0
        n = min(2 * n, 256)


def copy_ceiling(gf, torch, nbytes, reps=20):
    """The streaming kernels of the library (gf_stream: 16-byte loads and
    stores) over nbytes, the bytes one half-sweep reads and writes: a copy
    into a second buffer and an in-place pass (each 16 bytes read and written
    back, as the half-sweep updates its links in place), each cached and
    non-temporal, and a read-only pass.  Each kind: 3 untimed passes, then
    `reps` passes back to back between two events (as the half-sweeps of a
    chunk run); GB/s of bytes moved (read + written; read only for read)."""
    nbytes = nbytes // 16 * 16
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    sink = torch.empty(gf.stream_blocks(nbytes), dtype=torch.float32, device="cuda:0")
    out = {"bytes_read": nbytes, "kernel": "gf_stream (16-byte loads and stores)", "passes": reps}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for name, kind, dst, moved in (("copy", "copy", y, 2 * nbytes), ("copy_nt", "copy_nt", y, 2 * nbytes),
                                   ("inplace", "copy", x, 2 * nbytes), ("inplace_nt", "copy_nt", x, 2 * nbytes),
                                   ("read", "read", sink, nbytes)):
        for _ in range(3):
            gf.stream(kind, dst, x, nbytes)
        e0.record()
        for _ in range(reps):
            gf.stream(kind, dst, x, nbytes)
        e1.record()
        e1.synchronize()
        out[name + "_GBs"] = moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y, sink
    torch.cuda.empty_cache()
    return out


def beyond_cache(gf, torch, I, L=48, sweeps=40):
    """The same half-sweep on an L^4 lattice (L = 48: 1.02 GB of FP32-12
    links, four times the 256 MB Infinity Cache), smooth input (eps 0.5,
    seed 2001) generated and uploaded in slabs of 8 time-slices, autotuned:
    the mean launch time of the FP32-update half-sweep over `sweeps` OR
    sweeps (kernel events on the launch stream), against the 8 TB/s peak and
    the streaming kernels over the same bytes."""
    dims = (L, L, L, L)
    V = L ** 4
    fx = gf.GaugeFixer([dims], gauge="landau", storage="mixed", reunit_every=REUNIT)
    for t0 in range(0, L, 8):
        slab = torch.from_numpy(I.smooth(dims, EPS, SEEDS[0], t0=t0, nt=8).reshape(-1)).to("cuda:0")
        fx.upload(0, slab, t0=t0, nt=8)
        del slab
    fx.set_overrelax(OMEGA)
    fx.autotune(reps=8)  # the best shapes lie within 2% of each other here
    shape = fx.get_shape("fp32")
    key = "%d/%d/%d" % shape
    warm_up(fx, "or")
    fx.set_timing(True)
    fx.sweep("or", max_sweeps=sweeps, tol=0.0, check_every=CHECK)
    n, ms = fx.kernel_time("fp32")
    fx.set_timing(False)
    fx.close()
    bpl = BYTES_PER_SITE["mixed"] * V / 2
    achieved = bpl / (ms * 1e-3) / 1e9
    torch.cuda.empty_cache()
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(key, COUNTER_TRAFFIC_48) if L == 48 else None,
            "lattice": list(dims),
            "link_bytes": 48 * 4 * V, "kernel": "k_sweep (half-sweep)",
            "shape": {"waves_per_site_group": shape[0], "block": shape[1],
                      "nontemporal": bool(shape[2] & gf.SHAPE_NONTEMPORAL),
                      "xcd_tiles": not (shape[2] & gf.SHAPE_LINEAR_TILES)},
            "bytes_per_launch": bpl, "mean_launch_ms": ms, "launches": n,
            "copy_ceiling": copy_ceiling(gf, torch, int(bpl) // 2)}


def workloads(gf, I):
    """Wall time of further workloads, one JSON line each, inputs resident in
    HBM when the clock starts:
    * 32^4 MAG, eps 0.7, seed 4001: simulated annealing T 1.5 -> 0.01 over 3000
      steps (heatbath + 3 microcanonical sweeps each, Philox key 4002), then
      overrelaxation omega 1.7 to theta < 1e-12, FP32-12 storage;
    * 64^3 x 256 Coulomb: time per sweep (checks every 20 sweeps included)
      without and with Infinity-Cache groups;
    * MAG on a hot 16^4 configuration: annealing temperature scan, then
      overrelaxation;
    * precision study: 32^4 Landau seed 2001 in single, mixed and FP64-12;
    * 32 Gribov copies (8 random gauge copies each of 16^4, 24^4, 40x20^3,
      64x32^3, eps 0.5) fixed to Landau gauge in one batched launch,
      theta < 1e-12 per copy, FP32-12 storage;
    * gauge group SU(2): 32^4 (eps 0.5, seed 2001) Landau and MAG fixes in
      mixed and FP64 storage, and MAG annealing of a hot 32^4 field then
      overrelaxation."""
    import torch
    dims = (32, 32, 32, 32)
    inp = torch.from_numpy(I.smooth(dims, 0.7, 4001).reshape(-1)).to("cuda:0")
    fx = gf.GaugeFixer([dims], gauge="mag", storage="mixed", reunit_every=100, tail_theta=1e-9)
    fx.upload(0, inp)
    fx.set_overrelax(OMEGA)
    fx.autotune(reps=5)
    fx.upload(0, inp)
    fx.set_sweep_index(0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fx.set_anneal(1.5, 0.01, 3000, nmicro=3, seed=4002)
    fx.sweep("anneal")
    torch.cuda.synchronize()
    t_sa = time.perf_counter() - t0
    F_sa, th_sa = fx.measure(0)
    st, done = fx.sweep("or", max_sweeps=100000, tol=TOL, check_every=CHECK)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    F, th = fx.measure(0)
    print(json.dumps({"workload": "mag-32^4-eps0.7-anneal3000-T1.5to0.01-then-or", "anneal_s": round(t_sa, 3),
                      "anneal_sweeps": 12000, "F_after_anneal": F_sa, "or_sweeps": int(done[0]), "status": st,
                      "total_s": round(t_all, 3), "F": F, "theta": th}), flush=True)
    # the cooling pipeline of the annealing study: the same annealing, then
    # stochastic relaxation (p = 0.5) for at most 2000 sweeps until theta <
    # 1e-8, then overrelaxation to theta < 1e-12 (same random streams)
    fx.upload(0, inp)
    fx.set_sweep_index(0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fx.sweep("anneal")
    torch.cuda.synchronize()
    t_sa = time.perf_counter() - t0
    fx.set_stochastic(0.5)
    st_sr, d_sr = fx.sweep("sr", max_sweeps=2000, tol=1e-8, check_every=CHECK)
    torch.cuda.synchronize()
    t_sr = time.perf_counter() - t0
    F_sr, th_sr = fx.measure(0)
    st, done = fx.sweep("or", max_sweeps=100000, tol=TOL, check_every=CHECK)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    F, th = fx.measure(0)
    fx.close()
    print(json.dumps({"workload": "mag-32^4-eps0.7-anneal3000-then-sr-then-or", "anneal_s": round(t_sa, 3),
                      "F_after_anneal": F_sa, "theta_after_anneal": th_sa, "sr_sweeps": int(d_sr[0]),
                      "sr_status": st_sr, "sr_s": round(t_sr - t_sa, 3), "F_after_sr": F_sr,
                      "theta_after_sr": th_sr, "or_sweeps": int(done[0]), "status": st,
                      "total_s": round(t_all, 3), "F": F, "theta": th}), flush=True)

    # precision study (Sec. 4.5): the 32^4 Landau fix of seed 2001 in single
    # precision, mixed precision and FP64, against the oracle's F
    gold = golden_F().get(SEEDS[0])
    inp = torch.from_numpy(I.smooth(DIMS, EPS, SEEDS[0]).reshape(-1)).to("cuda:0")
    study = []
    for storage, R in (("single", REUNIT), ("mixed", REUNIT), ("f64r12", 0)):
        fx = gf.GaugeFixer([DIMS], gauge="landau", storage=storage, reunit_every=R, tail_theta=0.0)
        fx.upload(0, inp)
        fx.set_overrelax(OMEGA)
        fx.autotune(reps=3)
        fx.upload(0, inp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, done = fx.sweep("or", max_sweeps=MAX_SWEEPS, tol=TOL, check_every=CHECK)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        umean, umax = fx.unitarity(0)
        F, th = fx.measure(0)
        fx.close()
        study.append({"storage": storage, "reunit_every": R, "status": st, "sweeps": int(done[0]),
                      "s": round(el, 4), "F": F, "theta": th, "unitarity_max_at_stop": umax,
                      "F_rel_err_vs_oracle": abs(F - gold["F"]) / gold["F"] if gold else None})
    del inp
    print(json.dumps({"workload": "landau-32^4-seed2001-precision-study", "runs": study}), flush=True)

    # 64^3 x 256 Coulomb sweep throughput: 16 generated time-slices repeated
    # 16 times (the cost of a sweep does not depend on the link values), 40
    # sweeps without and with Infinity-Cache groups
    dims = (256, 64, 64, 64)
    vs = 64 ** 3
    slab = torch.from_numpy(I.smooth(dims, 0.5, 3001, t0=0, nt=16).reshape(-1)).to("cuda:0")
    fx = gf.GaugeFixer([dims], gauge="coulomb", storage="mixed", reunit_every=100, tail_theta=1e-9)
    for t0 in range(0, 256, 16):
        fx.upload(0, slab, t0=t0, nt=16)
    del slab
    fx.set_overrelax(OMEGA)
    fx.autotune(reps=2)
    out = {"workload": "coulomb-64^3x256-sweep-throughput"}
    for budget in (0, 224 << 20):
        fx.set_cache_budget(budget)
        fx.sweep("or", max_sweeps=CHECK, tol=0.0, check_every=CHECK)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx.sweep("or", max_sweeps=2 * CHECK, tol=0.0, check_every=CHECK)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / (2 * CHECK) * 1e3
        out["groups_%d" % fx.cache_groups()] = {"ms_per_sweep": round(ms, 3),
                                                 "GBs": round(672 * 256 * vs / (ms * 1e-3) / 1e9)}
    print(json.dumps(out), flush=True)
    coulomb_stop_distribution(fx, torch, I, dims)
    fx.close()

    # MAG on a hot (Haar-random) 16^4 configuration: annealing from several
    # starting temperatures to T = 0.01 (1000 steps, 3 microcanonical sweeps
    # each), then overrelaxation to theta < 1e-12 (at most 20000 sweeps)
    dims = (16, 16, 16, 16)
    hot = torch.from_numpy(I.hot(dims, 6001).reshape(-1)).to("cuda:0")
    scan = []
    for T0 in (0.5, 1.0, 1.5, 2.0):
        fx = gf.GaugeFixer([dims], gauge="mag", storage="mixed", reunit_every=100, tail_theta=1e-9)
        fx.upload(0, hot)
        fx.set_overrelax(OMEGA)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx.set_anneal(T0, 0.01, 1000, nmicro=3, seed=6002)
        fx.sweep("anneal")
        F_sa, _ = fx.measure(0)
        st, done = fx.sweep("or", max_sweeps=20000, tol=TOL, check_every=CHECK)
        torch.cuda.synchronize()
        F, th = fx.measure(0)
        scan.append({"T0": T0, "F_after_anneal": round(F_sa, 9), "or_sweeps": int(done[0]), "status": st,
                     "F": round(F, 12), "theta": th, "s": round(time.perf_counter() - t0, 3)})
        fx.close()
    print(json.dumps({"workload": "mag-16^4-hot-anneal-temperature-scan", "scan": scan}), flush=True)

    shapes = [(16, 16, 16, 16), (24, 24, 24, 24), (40, 20, 20, 20), (64, 32, 32, 32)]
    ncopy = 8
    dl = [d for d in shapes for _ in range(ncopy)]
    fx = gf.GaugeFixer(dl, gauge="landau", storage="mixed", reunit_every=100, tail_theta=1e-9)
    ins = []
    for li, d in enumerate(shapes):
        base = I.smooth(d, 0.5, 5001 + li)
        for c in range(ncopy):
            U = base.copy()
            I.gauge_copy(U, d, 5100 + 8 * li + c)
            ins.append(torch.from_numpy(U.reshape(-1)).to("cuda:0"))
    for k, x in enumerate(ins):
        fx.upload(k, x)
    fx.set_overrelax(OMEGA)
    fx.autotune(reps=3)
    for k, x in enumerate(ins):
        fx.upload(k, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, done = fx.sweep("or", max_sweeps=100000, tol=TOL, check_every=CHECK)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    Fs = [fx.measure(k)[0] for k in range(len(dl))]
    groups = fx.cache_groups()
    fx.close()
    su = sum(int(np.prod(d)) * int(n) for d, n in zip(dl, done))
    best = {"x".join(map(str, d)): round(max(Fs[i * ncopy:(i + 1) * ncopy]), 12) for i, d in enumerate(shapes)}
    print(json.dumps({"workload": "landau-gribov-batch-32-copies", "status": st, "total_s": round(t_all, 3),
                      "site_updates_per_s": su / t_all, "sweeps": done.tolist(), "cache_groups": groups,
                      "best_F": best}), flush=True)
    gribov_annealing(gf, torch, shapes, ncopy, dl, ins)
    del ins
    landau_temperature_scan(gf, torch, I)

    # gauge group SU(2): 32^4 Landau and MAG fixes (overrelaxation to
    # theta < 1e-12) in mixed and FP64 storage; the second of two runs is timed
    d2 = (32, 32, 32, 32)
    V = int(np.prod(d2))
    u2 = torch.from_numpy(I.su2_smooth(d2, 0.5, 2001).reshape(-1)).to("cuda:0")
    runs = []
    for gauge in ("landau", "mag"):
        for storage in ("mixed", "f64r18"):
            fx = gf.GaugeFixer([d2], gauge=gauge, storage=storage, reunit_every=100, group=2)
            fx.set_overrelax(OMEGA)
            for _ in range(2):
                fx.upload(0, u2)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, done = fx.sweep("or", max_sweeps=20000, tol=TOL, check_every=CHECK)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
            F, th = fx.measure(0)
            fx.close()
            runs.append({"gauge": gauge, "storage": storage, "status": st, "sweeps": int(done[0]),
                         "s": round(t, 4), "site_updates_per_s": V * int(done[0]) / t, "F": F, "theta": th})
    print(json.dumps({"workload": "su2-32^4-eps0.5-seed2001-or-fix", "runs": runs}), flush=True)
    # SU(2) MAG on a hot 32^4 field: annealing T 1.5 -> 0.01 over 1000 steps
    # (heatbath + 3 microcanonical sweeps each), then overrelaxation to
    # theta < 1e-12, mixed storage
    hot = torch.from_numpy(I.su2_hot(d2, 4011).reshape(-1)).to("cuda:0")
    fx = gf.GaugeFixer([d2], gauge="mag", storage="mixed", reunit_every=100, group=2)
    fx.set_overrelax(OMEGA)
    fx.upload(0, hot)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fx.set_anneal(1.5, 0.01, 1000, nmicro=3, seed=4012)
    fx.sweep("anneal")
    torch.cuda.synchronize()
    t_sa = time.perf_counter() - t0
    F_sa, _ = fx.measure(0)
    st, done = fx.sweep("or", max_sweeps=100000, tol=TOL, check_every=CHECK)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    F, th = fx.measure(0)
    m, x = fx.unitarity(0)
    fx.close()
    print(json.dumps({"workload": "su2-mag-32^4-hot-anneal1000-T1.5to0.01-then-or", "anneal_s": round(t_sa, 4),
                      "F_after_anneal": F_sa, "or_status": st, "or_sweeps": int(done[0]),
                      "total_s": round(t_all, 4), "F": F, "theta": th, "unitarity_max": x}), flush=True)


def coulomb_stop_distribution(fx, torch, I, dims, max_sweeps=10000, slab=16):
    """The 64^3 x 256 Coulomb input (eps 0.5, seed 3001, generated and
    uploaded in slabs of 16 time-slices) fixed by overrelaxation with
    per-time-slice stopping at theta_t < 1e-12, bounded at max_sweeps
    sweeps: how many time-slices stopped, the distribution of their sweep
    counts, and theta_t of those still running."""
    for t0 in range(0, dims[0], slab):
        x = torch.from_numpy(I.smooth(dims, 0.5, 3001, t0=t0, nt=slab).reshape(-1)).to("cuda:0")
        fx.upload(0, x, t0=t0, nt=slab)
        del x
    fx.set_cache_budget(224 << 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, done = fx.sweep("or", max_sweeps=max_sweeps, tol=TOL, check_every=CHECK)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    F_t, th_t = fx.measure_timeslices(0)
    stopped = done < max_sweeps
    q = np.percentile(done[stopped], [0, 25, 50, 75, 100]).tolist() if stopped.any() else []
    print(json.dumps({"workload": "coulomb-64^3x256-stop-distribution", "max_sweeps": max_sweeps, "status": st,
                      "s": round(el, 2), "stopped": int(stopped.sum()), "of": int(dims[0]),
                      "stop_sweeps_quartiles": q,
                      "theta_t_max_running": float(th_t[~stopped].max()) if (~stopped).any() else None,
                      "theta_t_max_stopped": float(th_t[stopped].max()) if stopped.any() else None,
                      "F_t_min": float(F_t.min()), "F_t_max": float(F_t.max())}), flush=True)


def gribov_annealing(gf, torch, shapes, ncopy, dl, ins, nsteps=3000, T0=4.0, T1=1e-4, tol=1e-10):
    """Global-maximum search over Gribov copies (Landau gauge): the 32 copies
    of the batch fixed by overrelaxation alone (0 annealing steps) and after
    simulated annealing (nsteps steps, T linear from T0 to T1, heatbath + 3
    microcanonical sweeps each, Philox key 7001), both to theta < tol, in one
    batched launch each.  Per copy F_rel = (F_max - F) / F_max with F_max the
    largest F found for its lattice by either run."""
    res = {}
    for steps in (0, nsteps):
        fx = gf.GaugeFixer(dl, gauge="landau", storage="mixed", reunit_every=100, tail_theta=1e-9)
        for k, x in enumerate(ins):
            fx.upload(k, x)
        fx.set_overrelax(OMEGA)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if steps:
            fx.set_anneal(T0, T1, steps, nmicro=3, seed=7001)
            fx.sweep("anneal")
        torch.cuda.synchronize()
        t_sa = time.perf_counter() - t0
        st, done = fx.sweep("or", max_sweeps=100000, tol=tol, check_every=CHECK)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        Fs = [fx.measure(k)[0] for k in range(len(dl))]
        fx.close()
        res[steps] = {"F": Fs, "or_sweeps": done.tolist(), "status": st, "anneal_s": round(t_sa, 3),
                      "total_s": round(t_all, 3)}
    out = {"workload": "landau-gribov-batch-32-copies-annealing-search", "anneal_steps": nsteps,
           "T0": T0, "T1": T1, "tol": tol, "lattices": {}}
    for i, d in enumerate(shapes):
        sl = slice(i * ncopy, (i + 1) * ncopy)
        Fmax = max(max(res[s]["F"][sl]) for s in res)
        out["lattices"]["x".join(map(str, d))] = {
            "F_max": Fmax,
            **{"steps_%d" % s: {"best_F": max(res[s]["F"][sl]),
                                 "F_rel": [float("%.3e" % ((Fmax - f) / Fmax)) for f in res[s]["F"][sl]],
                                 "or_sweeps": res[s]["or_sweeps"][sl]} for s in res}}
    for s in res:
        out["steps_%d" % s] = {k: res[s][k] for k in ("status", "anneal_s", "total_s")}
    print(json.dumps(out), flush=True)


def landau_temperature_scan(gf, torch, I, nsteps=3000, T0=4.0, T1=1e-4, nseg=10):
    """Landau gauge on a hot (Haar-random) 32^4 field: simulated annealing
    over nsteps steps (T linear from T0 to T1, heatbath + 3 microcanonical
    sweeps each), run as nseg consecutive pieces of the same schedule with F
    and theta measured after each, then overrelaxation to theta < 1e-12."""
    dims = (32, 32, 32, 32)
    hot = torch.from_numpy(I.hot(dims, 6101).reshape(-1)).to("cuda:0")
    fx = gf.GaugeFixer([dims], gauge="landau", storage="mixed", reunit_every=100, tail_theta=1e-9)
    fx.upload(0, hot)
    fx.set_overrelax(OMEGA)
    Ts = [T0 + (T1 - T0) * k / (nsteps - 1) for k in range(nsteps)]
    F, th = fx.measure(0)
    scan = [{"step": 0, "T": T0, "F": F, "theta": th}]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges = [round(nsteps * j / nseg) for j in range(nseg + 1)]
    for a, b in zip(edges[:-1], edges[1:]):
        fx.set_anneal(Ts[a], Ts[b - 1], b - a, nmicro=3, seed=6102)
        fx.sweep("anneal")
        F, th = fx.measure(0)
        scan.append({"step": b, "T": Ts[b - 1], "F": F, "theta": th})
    torch.cuda.synchronize()
    t_sa = time.perf_counter() - t0
    st, done = fx.sweep("or", max_sweeps=100000, tol=TOL, check_every=CHECK)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    F, th = fx.measure(0)
    fx.close()
    print(json.dumps({"workload": "landau-32^4-hot-anneal-temperature-scan", "scan": scan, "anneal_s": round(t_sa, 3),
                      "or_sweeps": int(done[0]), "status": st, "F": F, "theta": th,
                      "total_s": round(t_all, 3)}), flush=True)


def lattice_scan(gf, torch, I, nsweeps=20):
    """Half-sweep time against the lattice size (the paper's performance-vs-
    volume study): Landau OR on L^4 for L = 16 ... 56, FP32-12 mixed and
    FP64-12, smooth input (eps 0.5, seed 2001) uploaded in slabs of 8
    time-slices, autotuned, then nsweeps sweeps timed with kernel events; one
    JSON line per lattice and storage."""
    link = {"mixed": 48, "f64r12": 96}
    for L in (16, 24, 32, 40, 48, 56):
        dims = (L, L, L, L)
        V = L ** 4
        for storage in ("mixed", "f64r12"):
            fx = gf.GaugeFixer([dims], gauge="landau", storage=storage, reunit_every=0)
            for t0 in range(0, L, 8):
                fx.upload(0, I.smooth(dims, EPS, SEEDS[0], t0=t0, nt=min(8, L - t0)), t0=t0, nt=min(8, L - t0))
            fx.set_overrelax(OMEGA)
            fx.autotune(reps=3)
            table = "fp32" if storage == "mixed" else "fp64"
            shape = fx.get_shape(table)
            warm_up(fx, "or")
            fx.set_timing(True)
            fx.sweep("or", max_sweeps=nsweeps, tol=0.0, check_every=nsweeps)
            n, ms = fx.kernel_time(table)
            fx.set_timing(False)
            fx.close()
            bps = 16 * link[storage]
            gbs = bps * V / 2 / (ms * 1e-3) / 1e9
            print(json.dumps({"lattice": list(dims), "storage": storage, "link_MB": round(4 * V * link[storage] / 1e6, 1),
                              "shape": "%d/%d/%d" % shape, "mean_launch_ms": round(ms, 5),
                              "site_updates_per_s": V / 2 / (ms * 1e-3), "GBs": round(gbs, 1),
                              "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}), flush=True)
            torch.cuda.empty_cache()


def kernel_table(gf, torch, I, nsweeps=20):
    """Half-sweep launch time and effective bandwidth of every gauge x
    storage x update on a 32^4 lattice (Coulomb: 32 time-slices of 32^3),
    autotuned (the heatbath table too), about 30 ms of untimed sweeps, the
    input uploaded again from device memory, then nsweeps sweeps with kernel
    timing; one JSON line each; then the same for the gauge group SU(2) (one
    wavefront per site group)."""
    V = int(np.prod(DIMS))
    U = torch.from_numpy(I.smooth(DIMS, EPS, SEEDS[0]).reshape(-1)).to("cuda:0")
    link = {"mixed": 48, "single": 48, "f64r12": 96, "f64r18": 144}
    for gauge in ("landau", "coulomb", "mag"):
        nl = 6 if gauge == "coulomb" else 8
        for storage in ("mixed", "single", "f64r12", "f64r18"):
            # algorithmic bytes per site update: links loaded and stored (+ G for Coulomb)
            bps = 2 * nl * link[storage] + (2 * link[storage] if gauge == "coulomb" else 0)
            for upd in (("or",) if storage == "single" else ("or", "heatbath")):
                fx = gf.GaugeFixer([DIMS], gauge=gauge, storage=storage, reunit_every=0, tail_theta=0.0)
                fx.set_cache_budget(0)  # one launch per half-sweep over all time-slices
                fx.upload(0, U)
                fx.set_overrelax(OMEGA)
                fx.set_temperature(0.5)
                fx.set_seed(7)
                fx.autotune(reps=5)
                if upd == "heatbath":
                    fx.autotune_heatbath(reps=3)
                warm_up(fx, upd)
                fx.upload(0, U)  # device to device: the clocks stay up
                fx.set_timing(True)
                fx.sweep(upd, max_sweeps=nsweeps, tol=0.0, check_every=nsweeps)
                n, ms = fx.kernel_time("all")
                fx.set_timing(False)
                shape = fx.get_shape("heatbath" if upd == "heatbath" else
                                     ("fp32" if storage in ("mixed", "single") else "fp64"))
                fx.close()
                gbs = bps * V / 2 / (ms * 1e-3) / 1e9
                print(json.dumps({"group": "su3", "gauge": gauge, "storage": storage, "update": upd,
                                  "shape": "%d/%d/%d" % shape, "launches": n, "mean_launch_ms": round(ms, 5),
                                  "bytes_per_site_update": bps, "GBs": round(gbs, 1),
                                  "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}), flush=True)
    # gauge group SU(2): 4 reals per link (16 bytes FP32, 32 bytes FP64)
    U2 = torch.from_numpy(I.su2_smooth(DIMS, EPS, SEEDS[0]).reshape(-1)).to("cuda:0")
    link2 = {"mixed": 16, "single": 16, "f64r18": 32}
    for gauge in ("landau", "coulomb", "mag"):
        nl = 6 if gauge == "coulomb" else 8
        for storage in ("mixed", "single", "f64r18"):
            bps = 2 * nl * link2[storage] + (2 * link2[storage] if gauge == "coulomb" else 0)
            for upd in (("or",) if storage == "single" else ("or", "heatbath")):
                fx = gf.GaugeFixer([DIMS], gauge=gauge, storage=storage, reunit_every=0, tail_theta=0.0, group=2)
                fx.set_cache_budget(0)
                fx.upload(0, U2)
                fx.set_overrelax(OMEGA)
                fx.set_temperature(0.5)
                fx.set_seed(7)
                fx.autotune(reps=5)
                if upd == "heatbath":
                    fx.autotune_heatbath(reps=3)
                warm_up(fx, upd)
                fx.upload(0, U2)
                fx.set_timing(True)
                fx.sweep(upd, max_sweeps=nsweeps, tol=0.0, check_every=nsweeps)
                n, ms = fx.kernel_time("all")
                fx.set_timing(False)
                shape = fx.get_shape("heatbath" if upd == "heatbath" else
                                     ("fp32" if storage in ("mixed", "single") else "fp64"))
                fx.close()
                gbs = bps * V / 2 / (ms * 1e-3) / 1e9
                print(json.dumps({"group": "su2", "gauge": gauge, "storage": storage, "update": upd,
                                  "shape": "%d/%d/%d" % shape, "launches": n, "mean_launch_ms": round(ms, 5),
                                  "bytes_per_site_update": bps, "GBs": round(gbs, 1),
                                  "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}), flush=True)


def golden_F():
    p = os.path.join(ROOT, "tests", "golden", "c2_landau_oracle.json")
    if not os.path.exists(p):
        return {}
    d = json.load(open(p))
    return {int(k): v for k, v in d.items()}


def main():
    global TAIL
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison runs")
    ap.add_argument("--fp64-tail", type=float, default=None,
                    help="compute the update in FP64 once a unit's theta is below this (default %g)" % TAIL)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (scale for rocprof byte counters)")
    ap.add_argument("--workloads", action="store_true",
                    help="only time the annealing (32^4 MAG) and Gribov-copy batch workloads end to end")
    ap.add_argument("--kernel-table", action="store_true",
                    help="only time the half-sweep of every gauge, storage and update on 32^4 (one JSON line each)")
    ap.add_argument("--profile-sweeps", type=int, default=0,
                    help="only run this many OR sweeps of the workload (for profiler counter runs)")
    ap.add_argument("--lattice-scan", action="store_true",
                    help="only time the Landau OR half-sweep on L^4, L = 16 ... 56, mixed and FP64-12 (one JSON "
                         "line each)")
    ap.add_argument("--stream-sizes", action="store_true",
                    help="only time the streaming kernels (copy, non-temporal copy, read) over buffer sizes "
                         "16 MiB .. 2 GiB (one JSON line each)")
    ap.add_argument("--profile-lattice", type=int, default=32,
                    help="lattice extent L (L^4) of --profile-sweeps (default 32)")
    ap.add_argument("--profile-shapes", default="1/256/0",
                    help="launch shapes W/B/flags of --profile-sweeps, comma-separated (default 1/256/0)")
    ap.add_argument("--profile-heatbath", type=int, default=0,
                    help="only run this many heatbath sweeps (T = 0.5) of the 32^4 workload in Landau and MAG gauge, "
                         "mixed storage (for profiler counter runs)")
    ap.add_argument("--profile-coulomb", type=int, default=0,
                    help="only run this many OR sweeps of the 64^3 x 256 Coulomb configuration (mixed storage, "
                         "Infinity-Cache groups, after autotuning and a warm-up; for profiler runs)")
    ap.add_argument("--profile-su2", type=int, default=0,
                    help="only run this many OR sweeps of the 32^4 SU(2) Landau field, mixed storage "
                         "(for profiler counter runs)")
    args = ap.parse_args()
    if args.fp64_tail is not None:
        TAIL = args.fp64_tail
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the gauge-fixing path is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1212_5221_amd import gf, inputs as I

    if args.calibrate_copy:
        n = 1 << 30
        x = torch.empty(n // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}))
        return
    if args.lattice_scan:
        lattice_scan(gf, torch, I)
        return
    if args.stream_sizes:
        for mb in (16, 32, 64, 128, 160, 200, 256, 320, 512, 1024, 2048):
            c = copy_ceiling(gf, torch, mb << 20)
            print(json.dumps({"MiB_read": mb, **{k: (round(v, 1) if isinstance(v, float) else v)
                                                 for k, v in c.items()}}), flush=True)
        return
    if args.kernel_table:
        kernel_table(gf, torch, I)
        return
    if args.workloads:
        workloads(gf, I)
        return
    if args.profile_heatbath:
        # heatbath half-sweeps of seed 2001 at a fixed temperature, default
        # launch shapes, after about 30 ms of untimed heatbath sweeps; kernel
        # time from events on the launch stream
        U = torch.from_numpy(I.smooth(DIMS, EPS, SEEDS[0]).reshape(-1)).to("cuda:0")
        out = {"profile_heatbath_sweeps": args.profile_heatbath, "T": 0.5}
        for gauge in ("landau", "mag"):
            fx = gf.GaugeFixer([DIMS], gauge=gauge, storage="mixed", reunit_every=0)
            fx.upload(0, U)
            fx.set_temperature(0.5)
            fx.set_seed(7)
            warm_up(fx, "heatbath")
            fx.upload(0, U)
            fx.set_timing(True)
            fx.sweep("heatbath", max_sweeps=args.profile_heatbath, tol=0.0, check_every=args.profile_heatbath)
            n, ms = fx.kernel_time("all")
            out[gauge] = {"launches": n, "mean_launch_ms": ms, "shape": fx.get_shape("heatbath")}
            fx.close()
        print(json.dumps(out), flush=True)
        return
    if args.profile_coulomb:
        # 64^3 x 256 Coulomb, 16 generated time-slices repeated 16 times (as in
        # the workload's throughput line), default cache budget: the sweeps run
        # group by group; tol 0, so every time-slice runs every sweep
        dims = (256, 64, 64, 64)
        slab = torch.from_numpy(I.smooth(dims, 0.5, 3001, t0=0, nt=16).reshape(-1)).to("cuda:0")
        fx = gf.GaugeFixer([dims], gauge="coulomb", storage="mixed", reunit_every=100, tail_theta=1e-9)
        for t0 in range(0, 256, 16):
            fx.upload(0, slab, t0=t0, nt=16)
        del slab
        fx.set_overrelax(OMEGA)
        fx.autotune(reps=2)
        warm_up(fx, "or")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fx.sweep("or", max_sweeps=args.profile_coulomb, tol=0.0, check_every=CHECK)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        groups = fx.cache_groups()
        shape = fx.get_shape("fp32")
        fx.close()
        print(json.dumps({"profile_coulomb_sweeps": args.profile_coulomb, "lattice": list(dims), "cache_groups": groups,
                          "shape": "%d/%d/%d" % shape, "ms_per_sweep": el / args.profile_coulomb * 1e3,
                          "bytes_per_site_update": 672}), flush=True)
        return
    if args.profile_su2:
        # 32^4 SU(2), eps 0.5, seed 2001: one upload, then the sweeps in one
        # chunk; a half-sweep moves 256 B per site update over V/2 sites
        u2 = I.su2_smooth(DIMS, EPS, SEEDS[0])
        fx = gf.GaugeFixer([DIMS], gauge="landau", storage="mixed", reunit_every=0, group=2)
        fx.upload(0, u2)
        fx.set_overrelax(OMEGA)
        fx.sweep("or", max_sweeps=args.profile_su2, tol=0.0, check_every=args.profile_su2)
        fx.close()
        print(json.dumps({"profile_su2_sweeps": args.profile_su2, "bytes_per_launch": 256 * int(np.prod(DIMS)) // 2}),
              flush=True)
        return
    if args.profile_sweeps:
        # a fixed number of OR sweeps of the seed-2001 configuration on an
        # L^4 lattice (uploaded in slabs of 8 time-slices) with the FP32-update
        # half-sweep in each given launch shape "W/B/flags" in turn (for
        # profiler counter runs; the kernel names carry the shape)
        L = args.profile_lattice
        dims = (L, L, L, L)
        fx = gf.GaugeFixer([dims], gauge="landau", storage="mixed", reunit_every=REUNIT)
        fx.set_overrelax(OMEGA)
        bpl = BYTES_PER_SITE["mixed"] * L ** 4 / 2
        out = {"profile_sweeps": args.profile_sweeps, "lattice": list(dims), "kernel_digest": kernel_digest(),
               "bytes_per_launch": bpl}
        for key in args.profile_shapes.split(","):
            w, b, f = (int(x) for x in key.split("/"))
            fx.set_shape("fp32", w, b, f)
            for t0 in range(0, L, 8):
                fx.upload(0, I.smooth(dims, EPS, SEEDS[0], t0=t0, nt=min(8, L - t0)), t0=t0, nt=min(8, L - t0))
            fx.set_timing(True)
            fx.sweep("or", max_sweeps=args.profile_sweeps, tol=0.0, check_every=args.profile_sweeps)
            n, ms = fx.kernel_time("fp32")
            fx.set_timing(False)
            out[key] = {"launches": n, "mean_launch_ms": ms,
                        "achieved_GBs": bpl / (ms * 1e-3) / 1e9 if ms > 0 else None}
        fx.close()
        print(json.dumps(out))
        return

    dev = torch.device("cuda:0")
    V = int(np.prod(DIMS))
    log("generating inputs", DIMS, "seeds", SEEDS)
    inputs = [torch.from_numpy(I.smooth(DIMS, EPS, s).reshape(-1)).to(dev) for s in SEEDS]
    torch.cuda.synchronize()

    fx = make_fixer(gf, "mixed")
    fx.upload(0, inputs[0])  # autotune on the workload's data (it runs real sweeps)
    lanes, _ = fx.autotune(reps=10)
    shape = fx.get_shape("fp32")
    shape_key = "%d/%d/%d" % shape
    log("autotune: waves per site group, block, flags", shape)
    for w in range(args.warmup):
        one_fix(fx, inputs[w % len(SEEDS)])
    torch.cuda.synchronize()

    # ---- timed region: K complete fixes; the half-sweep launches of every
    # TIME_EVERY-th chunk are bracketed by HIP events recorded by the launch
    # itself on its stream, the other chunks replay HIP graphs
    fx.set_timing(True, every=TIME_EVERY)
    sweeps = []
    status = []
    per_step = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st, n = one_fix(fx, inputs[k % len(SEEDS)])
        per_step.append(time.perf_counter() - ts)
        sweeps.append(n)
        status.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, mean_ms = fx.kernel_time("fp32")    # the dominant kernel: FP32 update
    launches64, mean_ms64 = fx.kernel_time("fp64")  # FP64 tail
    fx.set_timing(False)

    gold = golden_F()
    F_err = {}
    for i, s in enumerate(SEEDS):
        if i < args.steps and s in gold:
            one_fix(fx, inputs[i])
            F, th = fx.measure(0)
            F_err[str(s)] = {"F": F, "theta": th, "F_oracle": gold[s]["F"],
                             "rel_err": abs(F - gold[s]["F"]) / gold[s]["F"]}
    fx.close()

    site_updates = V * float(sum(sweeps))
    value = site_updates / elapsed
    bytes_per_launch = BYTES_PER_SITE["mixed"] * V / 2
    achieved = bytes_per_launch / (mean_ms * 1e-3) / 1e9 if mean_ms > 0 else 0.0
    eff_gbs = site_updates * BYTES_PER_SITE["mixed"] / elapsed / 1e9

    # ---- plain FP64 GPU path: time to theta < 1e-12 per seed
    ttt = {"mixed_s": [round(t, 4) for t in per_step[:len(SEEDS)]], "mixed_sweeps": sweeps[:len(SEEDS)]}
    if not args.no_fp64:
        f64 = make_fixer(gf, "f64r12")
        f64.upload(0, inputs[0])
        f64.autotune(reps=5)
        one_fix(f64, inputs[0])
        tt, sw = [], []
        for i in range(min(args.steps, len(SEEDS))):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            st, n = one_fix(f64, inputs[i])
            torch.cuda.synchronize()
            tt.append(round(time.perf_counter() - ts, 4))
            sw.append(n)
        f64.close()
        ttt["fp64_s"] = tt
        ttt["fp64_sweeps"] = sw
        ttt["speedup_mixed_vs_fp64"] = round(sum(tt) / sum(per_step[:len(tt)]), 3)

    ceiling = copy_ceiling(gf, torch, int(bytes_per_launch) // 2)
    big = beyond_cache(gf, torch, I)
    # the same input handed over from host memory (pageable numpy array):
    # the PCIe-inclusive cost of a fix, reported beside the HBM-resident value
    host_in = I.smooth(DIMS, EPS, SEEDS[0])
    fx2 = make_fixer(gf, "mixed")
    fx2.upload(0, host_in)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    fx2.upload(0, host_in)
    torch.cuda.synchronize()
    host_upload_ms = (time.perf_counter() - ts) * 1e3
    fx2.close()
    del host_in
    cpu = None if args.no_cpu else cpu_baseline()

    line = {
        "metric": "OR site-updates/s (Landau, mixed FP32-12 storage, to theta<1e-12)",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "landau-32^4-eps0.5-seeds2001-2004-omega1.7-theta1e-12", "lattice": list(DIMS),
                   "gauge": "landau", "storage": "fp32-12real", "fp64": fp64_policy(), "check_every": CHECK,
                   "launch_shape": {"waves_per_site_group": shape[0], "block": shape[1],
                                    "nontemporal": bool(shape[2] & gf.SHAPE_NONTEMPORAL),
                                    "xcd_tiles": not (shape[2] & gf.SHAPE_LINEAR_TILES)},
                   "status": status, "sweeps": sweeps},
        "hbm_gbs_effective": eff_gbs,
        "time_to_theta": ttt,
        "host_upload_ms": host_upload_ms,
        "F_vs_oracle": F_err,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(shape_key),
                     "kernel": "k_sweep (half-sweep)", "bytes_per_launch": bytes_per_launch,
                     "mean_launch_ms": mean_ms, "launches": launches, "timed_chunks_every": TIME_EVERY,
                     "fp64_tail_launches": launches64, "fp64_tail_mean_ms": mean_ms64,
                     "copy_ceiling": ceiling,
                     "note": "the 201 MB of links stay partly in the 256 MB Infinity Cache between half-sweeps "
                             "(compare copy_ceiling.inplace_GBs, an in-place streaming pass over the same bytes); "
                             "traffic counts L2-to-fabric bytes (FETCH_SIZE, WRITE_SIZE), cache hits included"},
        "roofline_beyond_cache": big,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

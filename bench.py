#!/usr/bin/env python3
"""Benchmark: real collisions/s of the electron-swarm hot path on one MI355X.

Workload (the argon-like E/N sweep): 32 swarm instances of a synthetic argon-like gas at
E/N log-spaced over 1-1000 Td, B = 0, 100,000 electrons x 20,000 real collisions each,
seed 0, dummy ionisation (6.4e10 real collisions per step).

A step is one batched launch of all 32 instances in FP32-mixed precision: one persistent
kernel (the default launch shape; --autotune runs the autotuner first) plus the tally
reductions, replayed from a hipGraph.  `value` = real collisions per second over the timed steps.  Also measured once:
the same workload as 32 plain FP64 single-instance runs, the FP32-vs-FP64 tally agreement,
a short serving run (p50/p99 request latency), and the FP64 CPU oracle on a bounded sample
on the host cores.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]   (--help lists the other legs)
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU work per unit, in lane-instruction slots of the FP32-mixed path with
# B = 0 (full-rate VALU instruction = 1 slot; transcendentals log/sqrt/rsqrt/sin/cos = 2, as
# measured on gfx950; 32x32->64 integer multiply-add = 1, also measured full rate; a
# three-input xor = 1, gfx950 has it as one instruction).
# Trial (38): half a Philox4x32-10 call (20 multiply-adds + 20 three-input xors per call),
# the flight time from the 24-bit uniform (shift, convert, 1 - u by one FMA, log, FMA: 4 +
# log), x = R nu' (3), |v(T)|^2 m/2e (2 FMA), octave-grid position from the bits (clamp of
# the energy by one median-of-three, shift, address, and the weight as the masked low
# mantissa bits converted: 5), interpolated rate and compare (2).  (Until the kernel found the
# median-of-three clamp and the integer weight, the grid position counted 7 and the trial 40.)
# Real collision (113): one Philox call for the scattering block (40), channel search over the running sums
# (12), onset compare in FP64 (8), isotropic direction (16), cos(theta) (6), energy transfer
# (3), FP64 energy sums, position and time (16), new velocity (6), next-flight constants (4).
OPS_PER_TRIAL = 38
OPS_PER_REAL = 113
# The FP64 path, counted the same way (FP64 FMA issues at the full lane rate on gfx950, so the
# same lane-slot peak applies).  Trial (82): a full Philox call for the HI and one for the LO
# words per block (40 per trial), 1 - u exactly from the 53-bit uniform (5), the table-driven
# logarithm and the flight-time update (20: exponent and mantissa 2, table index and address 3,
# reduction 1, series to r^9 9, exponent and table terms 4, scaled add 1), x = R nu' (4), energy
# (3), grid position (7), interpolation and compare (3).  Real collision (184): the HI and LO
# scattering calls (80), channel search (12), onset compare (1), isotropic direction with
# binary64 sqrt and sincospi (42), cos(theta) with its square root and division (21), energy
# transfer (3), energy sums, position and time (8), new speed and velocity (13), next-flight
# constants (4).
OPS_PER_TRIAL_FP64 = 82
OPS_PER_REAL_FP64 = 184
PEAK_LANE_OPS = 256 * 64 * 2.4e9      # 256 CUs x 64 FP32 lanes/clock x 2.4 GHz = 3.93e13 /s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--electrons", type=int, default=100_000)
    ap.add_argument("--collisions", type=int, default=20_000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variable", action="store_true",
                    help="skip the leg with the variable trial frequency")
    ap.add_argument("--no-binned", action="store_true",
                    help="skip the leg with the binned trial frequency")
    ap.add_argument("--no-thermal", action="store_true",
                    help="skip the leg with moving targets")
    ap.add_argument("--no-relativistic", action="store_true",
                    help="skip the FP64 leg with the relativistic mover")
    ap.add_argument("--no-anisotropic", action="store_true",
                    help="skip the leg with screened-Coulomb scattering")
    ap.add_argument("--no-real", action="store_true",
                    help="skip the real-secondaries leg (mixture, 1e6 primaries)")
    ap.add_argument("--real-only", action="store_true",
                    help="only run the real-secondaries leg (used for its kernel trace)")
    ap.add_argument("--no-batch256", action="store_true",
                    help="skip the 256-instance batch leg")
    ap.add_argument("--serve-rate", type=float, default=50.0,
                    help="requests per second of the serving leg (the random-mixture request stream is stated at 50/s)")
    ap.add_argument("--serve-seconds", type=float, default=40.0,
                    help="arrival window of the serving leg; measured at its end")
    ap.add_argument("--serve-schedule", type=int, default=1,
                    help="serving schedule: 0 every admitted request each epoch, 1 shortest remaining work first")
    ap.add_argument("--serve-drain", action="store_true",
                    help="after the window, wait for every request instead of cancelling the unfinished ones")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg (one JSON line), e.g. for a sweep of --serve-rate")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shape with the autotuner first (default: the library default)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device a few times (counter calibration)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def committed_traffic():
    """HBM bytes per launch of the swarm kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None if the kernel source
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "swarm_dummy_f32_argon_sweep_traffic.json")
    src = os.path.join(ROOT, "paper_1901_08140_amd", "csrc", "swarm_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def agreement(a, b, keys):
    ok = 0
    for k in keys:
        va, sa, _ = a[k]
        vb, sb, _ = b[k]
        if math.isfinite(va) and math.isfinite(vb) and abs(va - vb) <= 3 * math.hypot(sa, sb) + 0.005 * abs(vb):
            ok += 1
    return ok


def _per_electron(rec):
    """Per-electron contributions to the mean-type tallies (dummy mode: equal collision counts)."""
    import numpy as np
    rec = rec[(rec["flags"] & 1) != 0]
    r, t = rec["r"], rec["t"]
    k = (rec["k_end"].astype(np.int64) - rec["k_start"]).astype(float)
    wz = np.mean(r[:, 2] / t)
    dz = r[:, 2] - t * wz
    dp2 = r[:, 0] ** 2 + r[:, 1] ** 2
    return rec["id"], {"W": -r[:, 2] / t, "mean_energy": rec["sum_eps"] / k, "mean_energy_after": rec["sum_epsp"] / k,
                       "D": (dz ** 2 + dp2) / t, "DL": dz ** 2 / (2 * t), "DT": dp2 / (4 * t),
                       "alpha": rec["G"] / -r[:, 2]}


def fp32_bias(cfgs, h32, h64):
    """Bias of the FP32-mixed tallies against FP64 on the same electrons and random streams: per
    E/N point and tally, the difference of the two runs' means and its standard error from the
    per-electron paired differences.  The two precisions share streams, so the paired error is
    far below that of independent estimates (at high E/N most electrons keep the same event
    sequence in both).  Reported relative to the FP64 value."""
    import numpy as np
    keys = ["W", "mean_energy", "mean_energy_after", "D", "DL", "DT", "alpha"]
    points = {k: [] for k in keys}
    for c, a, b in zip(cfgs, h32, h64):
        ra, rb = a.records(), b.records()
        ia, qa = _per_electron(ra[np.argsort(ra["id"], kind="stable")])
        ib, qb = _per_electron(rb[np.argsort(rb["id"], kind="stable")])
        if not np.array_equal(ia, ib):
            return {"error": f"{c.label}: the precisions finished different electrons"}
        for k in keys:
            d = qa[k] - qb[k]
            ref = float(np.mean(qb[k]))
            bias = float(np.mean(d))
            sig = float(np.std(d, ddof=1) / math.sqrt(len(d)))
            points[k].append([round(c.extra["td"], 4), bias / ref if ref else 0.0, sig / abs(ref) if ref else 0.0])
    summary = {}
    for k in keys:
        z = [abs(b) / s for _, b, s in points[k] if s > 0]
        summary[k] = {"max_abs_bias_rel": max(abs(b) for _, b, _ in points[k]),
                      "max_abs_z": max(z) if z else 0.0,
                      "within_3_paired_sigma": f"{sum(1 for _, b, s in points[k] if abs(b) <= 3 * s)}/{len(points[k])}",
                      "median_paired_sigma_rel": float(np.median([s for _, _, s in points[k]]))}
    return {"summary": summary, "points_td_bias_rel_sigma_rel": points}


def _oracle_counts(records):
    k = (records["k_end"].astype("i8") - records["k_start"]).sum()
    trials = k + records["n_null"].sum() + records["n_forbidden"].sum() + records["n_fail"].sum()
    return int(k), int(trials)


def cpu_baseline(sw, args):
    """The oracle as it stands, on the host cores (one thread per core of the process's
    affinity), on three bounded samples of the workloads, each beside the GPU's FP64 and
    FP32-mixed single runs of the same electrons:
      the Maxwell gas in full: 1000 electrons x 10,000 collisions, 10 Td;
      an argon-sweep subset: electrons 0..999 at E/N indices 0, 10, 21, 31 of the sweep
        (1, 9.3, 108, 1000 Td), 20,000 collisions each;
      a mixture subset: primaries 0..999 of the argon:CO2 mixture (100 Td, 1 T at 45 deg) with
        real secondaries, lineage-complete at a 2000-collision budget.
    `value` is the argon-sweep subset (the bench workload's gas)."""
    import oracle
    import synth
    import torch
    threads = max(1, len(os.sched_getaffinity(0)))
    sweep = synth.cfg2_argon_sweep()
    samples = [
        ("Maxwell gas in full: 1000 e x 10000 collisions, 10 Td, dummy",
         [synth.cfg1_maxwell()], 1000, 10_000),
        ("argon-sweep subset: ids 0..999 x 20000 collisions at 1, 9.3, 108, 1000 Td, dummy",
         [sweep[i] for i in (0, 10, 21, 31)], 1000, 20_000),
        ("mixture subset: primaries 0..999 of the argon:CO2 mixture, 100 Td, 1 T at 45 deg, real "
         "secondaries, lineage-complete at 2000 collisions",
         [synth.cfg3_mixture_real(n_electrons=1000, n_collisions=2000)], 1000, 2000),
    ]
    entries = []
    for name, cfgs, n_e, n_c in samples:
        real = trials = 0
        t0 = time.perf_counter()
        for c in cfgs:
            r = oracle.OracleModel.from_config(c).run(n_e, n_c, c.seed, n_threads=threads)
            k, tr = _oracle_counts(r.records)
            real += k
            trials += tr
        dt = time.perf_counter() - t0
        ent = {"sample": name, "oracle_real_per_s": real / dt, "oracle_trials_per_s": trials / dt,
               "oracle_seconds": dt, "real_collisions": real}
        for prec, key in ((sw.SWARM_FP64, "gpu_fp64"), (sw.SWARM_FP32_MIXED, "gpu_fp32")):
            hs = [sw.Swarm.from_config(c, prec) for c in cfgs]
            hs[0].run(min(n_e, 64), min(n_c, 100), 1)      # warm-up
            torch.cuda.synchronize()
            g_real = 0
            t1 = time.perf_counter()
            for h, c in zip(hs, cfgs):
                h.run(n_e, n_c, c.seed)
                g_real += h.tallies()["n_real"]
            torch.cuda.synchronize()
            ent[key + "_real_per_s"] = g_real / (time.perf_counter() - t1)
            for h in hs:
                h.close()
        entries.append(ent)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    main = entries[1]
    return {"value": main["oracle_real_per_s"], "unit": "real collisions/s", "cores": threads, "kind": "oracle",
            "sample": main["sample"], "trials_per_s": main["oracle_trials_per_s"], "cpu_model": model,
            "entries": entries,
            "note": "GPU numbers of these small samples (1000 electrons) leave most of the device idle; "
                    "they are the same electrons, not the device's throughput"}


def serve(sw, args):
    """The random-mixture request stream (random mixtures of 1-6 components, E/N 1-1000 Td, |B| 0-2 T,
    1e3-1e6 electrons x 1e3-1e5 collisions) arriving as a Poisson process at --serve-rate over an
    arrival window of --serve-seconds into the continuous-batching server (HBM budget 200 GB,
    FP32-mixed).  Measured at the end of the window: the requests completed in it and their
    arrival-to-result latency (p50/p99), the real collisions served in the window against those
    offered, and the backlog (requests waiting and admitted, collisions still owed) sampled every
    second.  Requests still unfinished are then cancelled (unless --serve-drain)."""
    import numpy as np
    import synth
    rng = np.random.default_rng(5)
    arrivals = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / args.serve_rate)
        if t >= args.serve_seconds:
            break
        arrivals.append(t)
    reqs = [synth.cfg5_request(i) for i in range(len(arrivals))]
    srv = sw.swarm_server_create(200 << 30, sw.SWARM_FP32_MIXED, schedule=args.serve_schedule)
    try:
        t0 = sw.swarm_server_now(srv)
        tickets, backlog = [], []
        next_sample = 0.0

        def tick():
            nonlocal next_sample
            if sw.swarm_server_now(srv) - t0 >= next_sample:
                st = sw.swarm_server_stats(srv)
                backlog.append({"t_s": round(st["time_s"] - t0, 2), "waiting": st["n_pending"],
                                "admitted": st["n_active"], "finished": st["n_finished"],
                                "collisions_owed": st["work_left"], "collisions_served": st["work_done"]})
                next_sample += 1.0

        for a, c in zip(arrivals, reqs):
            while sw.swarm_server_now(srv) - t0 < a:
                tick()
                time.sleep(0.001)
            tickets.append(sw.swarm_server_submit(srv, c.components, sw.params_from_config(c, 1),
                                                  c.n_electrons, c.n_collisions, c.seed))
        while sw.swarm_server_now(srv) - t0 < args.serve_seconds:
            tick()
            time.sleep(0.001)
        if args.serve_drain:
            sw.swarm_server_drain(srv)
        t_end = sw.swarm_server_now(srv)
        st_end = sw.swarm_server_stats(srv)
        lat, real, trials, served_in_requests = [], 0, 0, 0
        for tk in tickets:
            done, tal, info = sw.swarm_server_poll(srv, tk)
            served_in_requests += info["progress"]
            if done:
                lat.append(info["done_s"] - info["submit_s"])
                real += tal["n_real"]
                trials += tal["n_real"] + tal["n_null"] + tal["n_forbidden"] + tal["n_fail"]
        lat = np.array(lat)
        window = t_end - t0
        offered = sum(c.n_electrons * c.n_collisions for c in reqs)
        return {"requests": len(tickets), "rate_per_s": args.serve_rate, "arrival_window_s": args.serve_seconds,
                "measured_window_s": window,
                "completed": int(len(lat)), "completed_fraction": len(lat) / max(1, len(tickets)),
                "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "latency_of": "requests completed in the window (arrival to result)",
                "served_real_per_s": st_end["work_done"] / window,
                "offered_real_per_s": offered / args.serve_seconds,
                "collisions_owed_at_end": st_end["work_left"],
                "completed_real": real, "completed_efficiency": real / trials if trials else None,
                "schedule": "shortest remaining work first" if args.serve_schedule == 1 else "every admitted request",
                "backlog": backlog}
    finally:
        sw.swarm_server_destroy(srv)


def adaptive_leg(sw, args, cfgs, jobs, opts, tall_const, ms_const, strategy):
    """The same batched FP32 step with one of the paper's adaptive trial frequencies
    (variable: per-electron nu' = (1 + zeta) nu(eps); binned: the nu' of the energy's bin;
    both renewed every `grace` trials and after fails): throughput, efficiency, fails, and
    how far its tallies move from the exact constant-frequency run."""
    hv = [sw.Swarm.from_config(c.scaled(**strategy), sw.SWARM_FP32_MIXED) for c in cfgs]
    b = sw.swarm_batch_create([h.h for h in hv], jobs, opts)
    try:
        sw.swarm_batch_launch(b)
        sw.swarm_batch_wait(b)
        ms = []
        for _ in range(max(1, args.steps)):
            sw.swarm_batch_launch(b)
            ms.append(sw.swarm_batch_wait(b))
        tv = [sw.swarm_batch_tallies(b, i) for i in range(len(cfgs))]
    finally:
        sw.swarm_batch_destroy(b)
    avg = sum(ms) / len(ms)
    real = sum(t["n_real"] for t in tv)
    trials = sum(t["n_real"] + t["n_null"] + t["n_forbidden"] + t["n_fail"] for t in tv)
    keys = ["W", "mean_energy", "mean_energy_after", "D", "DL", "DT", "alpha"]
    agree = sum(agreement(a, c, keys) for a, c in zip(tv, tall_const))
    shift = {}
    for k in keys:
        rel = [(a[k][0] - c[k][0]) / abs(c[k][0]) for a, c in zip(tv, tall_const)
               if c[k][0] != 0 and math.isfinite(a[k][0]) and math.isfinite(c[k][0])]
        shift[k] = {"min": min(rel), "max": max(rel)} if rel else None
    out = {"value": real / (avg * 1e-3), "unit": "real collisions/s", "device_ms_per_step": avg}
    out.update({k: v for k, v in strategy.items() if k != "trial_strategy"})
    out.update({"efficiency": real / trials, "fails_per_real": sum(t["n_fail"] for t in tv) / real,
                "speedup_vs_constant": ms_const / avg,
                "within_tolerance_of_constant": f"{agree}/{len(keys) * len(cfgs)}",
                "rel_shift_vs_constant": shift})
    out["exact"] = bool(all(t["exact"] for t in tv))      # the library's flag: False for these strategies
    if strategy["trial_strategy"] == 2:
        # electrons whose retry failed again (flag 16: where the paper throws), from the tallies
        n16 = sum(t["n_retry_failed"] for t in tv)
        out["n_retry_failed"] = n16
        out["retry_failed_electron_fraction"] = n16 / sum(j[0] for j in jobs)
    return out


def batched_run(sw, args, cfgs, jobs, opts, precision, steps=None):
    """One warm-up and `steps` (default args.steps) timed batched launches of the configs;
    (avg ms, tallies)."""
    hs = [sw.Swarm.from_config(c, precision) for c in cfgs]
    b = sw.swarm_batch_create([h.h for h in hs], jobs, opts)
    try:
        sw.swarm_batch_launch(b)
        sw.swarm_batch_wait(b)
        ms = []
        for _ in range(max(1, args.steps if steps is None else steps)):
            sw.swarm_batch_launch(b)
            ms.append(sw.swarm_batch_wait(b))
        tl = [sw.swarm_batch_tallies(b, i) for i in range(len(cfgs))]
    finally:
        sw.swarm_batch_destroy(b)
    return sum(ms) / len(ms), tl


def ratio_range(ta, tb, keys):
    out = {}
    for k in keys:
        r = [a[k][0] / b[k][0] for a, b in zip(ta, tb) if b[k][0] != 0 and math.isfinite(a[k][0])]
        out[k] = {"min": min(r), "max": max(r)} if r else None
    return out


def thermal_leg(sw, args, cfgs, jobs, opts, tall_const, ms_const, T_K=293.0):
    """The batched FP32 step with moving targets (Maxwell-Boltzmann at T_K): throughput, time
    relative to targets at rest, and how the drift velocity and mean energy move (little at
    these E/N, 1-1000 Td)."""
    avg, tt = batched_run(sw, args, [c.scaled(thermal_targets=1, T_K=T_K) for c in cfgs], jobs, opts,
                          sw.SWARM_FP32_MIXED)
    real = sum(t["n_real"] for t in tt)
    return {"value": real / (avg * 1e-3), "unit": "real collisions/s", "device_ms_per_step": avg, "T_K": T_K,
            "time_vs_at_rest": avg / ms_const,
            "ratio_to_at_rest": ratio_range(tt, tall_const, ("W", "mean_energy"))}


def relativistic_leg(sw, args, cfgs, jobs, opts):
    """The batched FP64 step with the relativistic mover against the classical one: throughput,
    time ratio and the tally ratios (relativistic corrections are O(eps / m c^2) here)."""
    o = {k: v for k, v in opts.items() if k != "use_graph"}
    o["use_graph"] = 1
    # (FP64 launches of this workload take seconds: one timed launch each)
    ms_c, tc = batched_run(sw, args, cfgs, jobs, o, sw.SWARM_FP64, steps=1)
    ms_r, tr = batched_run(sw, args, [c.scaled(relativistic=1) for c in cfgs], jobs, o, sw.SWARM_FP64, steps=1)
    real = sum(t["n_real"] for t in tr)
    return {"value": real / (ms_r * 1e-3), "unit": "real collisions/s", "device_ms_per_step": ms_r,
            "classical_device_ms_per_step": ms_c, "time_vs_classical": ms_r / ms_c,
            "ratio_to_classical": ratio_range(tr, tc, ("W", "mean_energy"))}


def anisotropic_leg(sw, args, cfgs, jobs, opts, tall_const, ms_const):
    """The same batched FP32 step with screened-Coulomb (anisotropic) scattering of the
    argon-like atom: throughput, and how the drift velocity and mean energy move."""
    ca = [c.scaled(components=[k.with_scattering(1) for k in c.components]) for c in cfgs]
    ha = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in ca]
    b = sw.swarm_batch_create([h.h for h in ha], jobs, opts)
    try:
        sw.swarm_batch_launch(b)
        sw.swarm_batch_wait(b)
        ms = []
        for _ in range(max(1, args.steps)):
            sw.swarm_batch_launch(b)
            ms.append(sw.swarm_batch_wait(b))
        ta = [sw.swarm_batch_tallies(b, i) for i in range(len(cfgs))]
    finally:
        sw.swarm_batch_destroy(b)
    avg = sum(ms) / len(ms)
    real = sum(t["n_real"] for t in ta)
    trials = sum(t["n_real"] + t["n_null"] + t["n_forbidden"] + t["n_fail"] for t in ta)
    ratio = {k: [a[k][0] / c[k][0] for a, c in zip(ta, tall_const) if c[k][0] != 0]
             for k in ("W", "mean_energy")}
    return {"value": real / (avg * 1e-3), "unit": "real collisions/s", "device_ms_per_step": avg,
            "efficiency": real / trials, "time_vs_isotropic": avg / ms_const,
            "ratio_to_isotropic": {k: {"min": min(v), "max": max(v)} for k, v in ratio.items()}}


def real_secondaries_leg(sw, args, n_electrons=1_000_000, n_collisions=2000):
    """The real-secondaries kernel on the 90:10 argon-like:CO2-like mixture at 100 Td, B = 1 T at
    45 degrees: 1e6 primaries, with the largest collision budget whose lineage growth fits the
    default capacity.  FP32-mixed and FP64 single runs (a launch per generation, with the
    stragglers parked for the next, after a small warm-up run): throughput, launches and
    electrons parked, electrons created and attached, and how the FP32 tallies agree with the
    FP64 ones."""
    import torch
    import synth
    cfg = synth.cfg3_mixture_real(n_electrons=n_electrons, n_collisions=n_collisions)
    out = {"workload": f"90:10 argon-like:CO2-like, 100 Td, B = 1 T at 45 deg, real secondaries, "
                       f"{n_electrons} primaries x {n_collisions} real collisions, seed 0"}
    tall = {}
    for name, prec in (("fp32", sw.SWARM_FP32_MIXED), ("fp64", sw.SWARM_FP64)):
        s = sw.Swarm.from_config(cfg, prec)
        s.run(n_electrons // 100, n_collisions, 1)        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(n_electrons, n_collisions, 0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_ms, total_ms = s.timing()
        launches, parked = s.launches()
        t = s.tallies()
        tall[name] = t
        out[name] = {"value": t["n_real"] / wall, "unit": "real collisions/s", "seconds": wall,
                     "kernel_ms": kernel_ms, "device_ms": total_ms, "n_real": t["n_real"],
                     "efficiency": t["efficiency"], "n_electrons": t["n_electrons"],
                     "n_created": t["n_created"], "n_attached": t["n_attached"], "n_dropped": t["n_dropped"],
                     "launches": launches, "parked": parked}
        s.close()
    keys = ["W", "Wx", "Wy", "mean_energy", "D_vec", "alpha"]
    out["fp32_vs_fp64_within_tolerance"] = f"{agreement(tall['fp32'], tall['fp64'], keys)}/{len(keys)}"
    out["fp32_speedup"] = out["fp32"]["value"] / out["fp64"]["value"]
    return out


def batch256_leg(sw, args):
    """The 256-instance sweep (4 mixtures x 64 E/N over 1-1000 Td, B = 0 or 1 T at random
    angles, electron counts 1e3-1e6 and collision budgets 1e3-1e5 log-uniform) in one
    persistent FP32 launch: about 8e11 real collisions, timed once."""
    import synth
    cfgs = synth.cfg4_batch()
    jobs = [(c.n_electrons, c.n_collisions, c.seed) for c in cfgs]
    hs = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    b = sw.swarm_batch_create([h.h for h in hs], jobs, {"use_graph": 1})
    try:
        # (one launch of about 30 s: the kernels are warm from the other legs)
        sw.swarm_batch_launch(b)
        ms = sw.swarm_batch_wait(b)
        tl = [sw.swarm_batch_tallies(b, i) for i in range(len(cfgs))]
    finally:
        sw.swarm_batch_destroy(b)
    real = sum(t["n_real"] for t in tl)
    trials = sum(t["n_real"] + t["n_null"] + t["n_forbidden"] + t["n_fail"] for t in tl)
    return {"value": real / (ms * 1e-3), "unit": "real collisions/s", "device_ms": ms, "instances": len(cfgs),
            "n_real": real, "efficiency": real / trials,
            "workload": "4 mixtures x 64 E/N (1-1000 Td), B 0 or 1 T, uneven sizes, FP32-mixed, one launch"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.serve_only:
        import paper_1901_08140_amd as sw
        print(json.dumps({"serving": serve(sw, args)}), flush=True)
        return
    if args.real_only:
        import paper_1901_08140_amd as sw
        print(json.dumps({"real_secondaries": real_secondaries_leg(sw, args)}), flush=True)
        return
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)
        return
    import paper_1901_08140_amd as sw
    import synth
    cfgs = synth.cfg2_argon_sweep(n_electrons=args.electrons, n_collisions=args.collisions)
    jobs = [(c.n_electrons, c.n_collisions, c.seed) for c in cfgs]
    h32 = [sw.Swarm.from_config(c, sw.SWARM_FP32_MIXED) for c in cfgs]
    handles = [h.h for h in h32]
    opts = {"use_graph": 1}
    if args.autotune:
        # probe budgets of a fifth of the run's: short probes misjudge the end of the launch
        # (the tail of the last work items), which the work-item size is about
        best = sw.swarm_autotune(handles, jobs, max(300, args.collisions // 5))
        opts.update(best)
        opts["use_graph"] = 1
        log(args, "autotuned launch options", opts)
    batch = sw.swarm_batch_create(handles, jobs, opts)
    for _ in range(args.warmup):
        sw.swarm_batch_launch(batch)
        sw.swarm_batch_wait(batch)
    torch.cuda.synchronize()
    dev_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sw.swarm_batch_launch(batch)
        dev_ms.append(sw.swarm_batch_wait(batch))
        log(args, f"step {len(dev_ms)}: {dev_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tall32 = [sw.swarm_batch_tallies(batch, i) for i in range(len(cfgs))]
    sw.swarm_batch_destroy(batch)
    real_per_step = sum(t["n_real"] for t in tall32)
    trials_per_step = sum(t["n_real"] + t["n_null"] + t["n_forbidden"] + t["n_fail"] for t in tall32)
    value = real_per_step * args.steps / wall
    avg_ms = sum(dev_ms) / len(dev_ms)
    ops = trials_per_step * OPS_PER_TRIAL + real_per_step * OPS_PER_REAL
    achieved = ops / (avg_ms * 1e-3)
    out = {
        "metric": "real collisions/s on 1 MI355X (FP32 batched vs FP64 plain); p50/p99 solve latency",
        "value": value, "unit": "real collisions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (f64 positions, times, sums, onset compare)", "data": "synthetic",
        "config": {"workload": f"argon-like E/N sweep: 32 x 1-1000 Td, B=0, {args.electrons} electrons x "
                               f"{args.collisions} real collisions each, dummy ionisation, seed 0",
                   "instances": len(cfgs), "electrons": args.electrons, "collisions": args.collisions,
                   "launch": opts},
        "trials_per_s": trials_per_step * args.steps / wall,
        "efficiency": real_per_step / trials_per_step,
        "device_ms_per_step": avg_ms,
        "device_ms_median": sorted(dev_ms)[len(dev_ms) // 2] if len(dev_ms) % 2 else
                            0.5 * (sorted(dev_ms)[len(dev_ms) // 2 - 1] + sorted(dev_ms)[len(dev_ms) // 2]),
        "device_ms_steps": dev_ms,
        "roofline": {"bound": "alu", "achieved": achieved / 1e9, "peak": PEAK_LANE_OPS / 1e9, "unit": "Gop/s",
                     "frac": achieved / PEAK_LANE_OPS, "traffic": committed_traffic(),
                     "kernel": "k_swarm_dummy<float,false,false,0>",
                     "ops_per_trial": OPS_PER_TRIAL, "ops_per_real": OPS_PER_REAL},
    }
    if not args.no_variable:
        out["fp32_batched_variable"] = adaptive_leg(sw, args, cfgs, jobs, opts, tall32, avg_ms,
                                                    dict(trial_strategy=1, trial_zeta=0.25, trial_grace=5000))
        log(args, "variable trial frequency", out["fp32_batched_variable"])
    if not args.no_binned:
        out["fp32_batched_binned"] = adaptive_leg(sw, args, cfgs, jobs, opts, tall32, avg_ms,
                                                  dict(trial_strategy=2, trial_bins=10, trial_grace=5000))
        log(args, "binned trial frequency", out["fp32_batched_binned"])
    if not args.no_anisotropic:
        out["fp32_batched_screened_coulomb"] = anisotropic_leg(sw, args, cfgs, jobs, opts, tall32, avg_ms)
        log(args, "screened-Coulomb scattering", out["fp32_batched_screened_coulomb"])
    if not args.no_thermal:
        out["fp32_batched_moving_targets"] = thermal_leg(sw, args, cfgs, jobs, opts, tall32, avg_ms)
        log(args, "moving targets", out["fp32_batched_moving_targets"])
    if not args.no_relativistic:
        out["fp64_batched_relativistic"] = relativistic_leg(sw, args, cfgs, jobs, opts)
        log(args, "relativistic", out["fp64_batched_relativistic"])
    if not args.no_real:
        out["real_secondaries"] = real_secondaries_leg(sw, args)
        log(args, "real secondaries", out["real_secondaries"])
    if not args.no_batch256:
        out["fp32_batch_256_instances"] = batch256_leg(sw, args)
        log(args, "256-instance batch", out["fp32_batch_256_instances"])
    if not args.no_fp64:
        # the plain FP64 form: one swarm per launch, default launch shape
        h64 = [sw.Swarm.from_config(c, sw.SWARM_FP64) for c in cfgs]
        h64[0].run(*jobs[0])       # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for h, (ne, nc, seed) in zip(h64, jobs):
            h.run(ne, nc, seed)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t1
        tall64 = [h.tallies() for h in h64]
        real64 = sum(t["n_real"] for t in tall64)
        keys = ["W", "mean_energy", "mean_energy_after", "D", "DL", "DT", "alpha"]
        agree = sum(agreement(a, b, keys) for a, b in zip(tall32, tall64))
        out["fp64_plain"] = {"value": real64 / dt64, "unit": "real collisions/s", "seconds": dt64,
                             "speedup_fp32_batched": value / (real64 / dt64)}
        out["fp32_vs_fp64_within_tolerance"] = f"{agree}/{len(keys) * len(cfgs)}"
        worst = {}
        for k in keys:
            rel = [abs(a[k][0] - b[k][0]) / abs(b[k][0]) for a, b in zip(tall32, tall64)
                   if b[k][0] != 0 and math.isfinite(a[k][0]) and math.isfinite(b[k][0])]
            worst[k] = max(rel) if rel else None
        out["fp32_vs_fp64_max_rel_diff"] = worst
        out["fp32_bias"] = fp32_bias(cfgs, h32, h64)
        log(args, "fp32 bias against fp64 (paired)", out["fp32_bias"].get("summary"))
        log(args, f"fp64 plain {real64 / dt64:.3e}/s; fp32 within tolerance {agree}/{len(keys) * len(cfgs)}")
        # the same FP64 work batched (separates the precision gain from the batching gain)
        b64 = sw.swarm_batch_create([h.h for h in h64], jobs, {"use_graph": 1, **{k: v for k, v in opts.items()
                                                                                 if k != "use_graph"}})
        sw.swarm_batch_launch(b64)
        ms64 = sw.swarm_batch_wait(b64)
        sw.swarm_batch_destroy(b64)
        trials64 = sum(t["n_real"] + t["n_null"] + t["n_forbidden"] + t["n_fail"] for t in tall64)
        ach64 = (trials64 * OPS_PER_TRIAL_FP64 + real64 * OPS_PER_REAL_FP64) / (ms64 * 1e-3)
        out["fp64_batched"] = {"value": real64 / (ms64 * 1e-3), "unit": "real collisions/s",
                               "device_ms": ms64,
                               "roofline": {"bound": "alu", "achieved": ach64 / 1e9, "peak": PEAK_LANE_OPS / 1e9,
                                            "unit": "Gop/s", "frac": ach64 / PEAK_LANE_OPS,
                                            "kernel": "k_swarm_dummy<double,false,false,0>",
                                            "ops_per_trial": OPS_PER_TRIAL_FP64, "ops_per_real": OPS_PER_REAL_FP64}}
        del h64

    if args.serve_seconds > 0 and args.serve_rate > 0:
        out["serving"] = serve(sw, args)
        out["p50_latency_s"] = out["serving"]["p50_latency_s"]
        out["p99_latency_s"] = out["serving"]["p99_latency_s"]
        log(args, "serving", out["serving"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sw, args)
        log(args, "cpu baseline", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

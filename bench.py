"""Throughput benchmark of the quasi-greedy many-clone dynamics on one MI355X.

Workload (default, "steady"): 16 planted instances with N = 1024 spins (3-regular 3-uniform
hypergraph, M = N, planted J), 2^20 clones each in uint64 words, run together as one batch (one
sweep-chunk launch over all tiles of all instances), 10^4 sweeps per step. One step = one full
pass of the path over the batch: start configurations drawn on the device, sweeps in chunks of
100, ground-state capture, stop checks, end-of-run energies, TTS and winner reduction, the
winner's configuration. `--workload batched` runs the 64 x N = 256 x 65,536-clone batch to its
first ground state (or a per-step budget) instead.

Prints one JSON line: clone-spin updates per ns for the whole job, the sweep kernel's roofline
record (LDS bound: 1 byte of LDS traffic per update, from HIP-event timing of every sweep-chunk
launch on the stream it runs on), TTS p50/p99 of the small single-instance workload run one at a
time, batched and served, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic LDS traffic per update: the 7 state bits an update reads (own spin and the two
# partners in each of its three triplets) and the 1 bit it writes = 1 byte.
ALGO_LDS_BYTES_PER_UPDATE = 1.0
# LDS peak for 16-byte reads: a conflict-free ds_read_b128 keeps the LDS busy 4 clocks per wave
# (1 KB), so 256 CUs x 256 B/clk x 2.4 GHz = 157.3 TB/s (a streaming microbenchmark with 16
# waves per CU reached 136 TB/s at 94 % LDS busy).
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12
# Secondary figure: VALU issue. 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s of
# full-rate 32-bit VALU work. Algorithmic VALU instructions per clone-spin update: the rule takes
# 7 three-input operations per 32-clone word; one Philox4x32-10 call (10 rounds of 2 wide
# products and 2 three-input XORs) plus 8 threshold compares serve 8 groups = 256 clones:
# 7/32 + 48/256 = 0.406. The fraction below counts every one of them as a full-rate operation
# (the rate of the 32x32->64 product is not measured here), so it is an upper bound on VALU use.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
ALGO_OPS_PER_UPDATE = 7 / 32 + (10 * (2 + 2) + 8) / 256
# With w0 > 0 the rule takes 9 operations per word and every draw is compared with both
# thresholds.
ALGO_OPS_PER_UPDATE_W0 = 9 / 32 + (10 * (2 + 2) + 16) / 256

# Headline workloads: (instances, N, clones, default sweeps per step, stop at first ground
# state, instance-seed config number, default sweeps per chunk). Each chunk boundary stages
# the tiles out and in, so chunks are long: a budget run checks nothing between chunks, and a
# run to the first ground state sees a hit at the end of its chunk (first hits, TTS and the
# solved configuration stay exact; at most one chunk of sweeps follows the hit, against a TTS
# near 4e7 sweeps at N = 256 with 65,536 clones).
HEADLINES = {
    "steady": dict(count=16, n=1024, clones=1 << 20, budget=10000, stop=False, config=3,
                   chunk=1000),
    "batched": dict(count=64, n=256, clones=65536, budget=50000, stop=True, config=2, chunk=500),
}
# HBM counter records per headline workload (FETCH_SIZE / WRITE_SIZE of the sweep kernel).
TRAFFIC_RECORDS = {"steady": "qg_queue_run_n1024x16_hbm_counters.json",
                   "batched": "qg_queue_run_n256x64_hbm_counters.json"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=None,
                    help="headline workloads: instances (default: the workload's)")
    ap.add_argument("--n", type=int, default=None, help="headline workloads: spins")
    ap.add_argument("--clones", type=int, default=None, help="headline workloads: clones")
    ap.add_argument("--place-rows", action="store_true",
                    help="batched: build the LDS row placement whatever the run length "
                         "(tiles under eight blocks, large N; speed only)")
    ap.add_argument("--budget", type=int, default=None,
                    help="sweep budget per instance and step (default: 10^4 for steady, uneven "
                         "and serve; 5*10^4 for batched, whose first ground states at N=256 take "
                         "far longer, so most instances end at the budget)")
    ap.add_argument("--chunk", type=int, default=None,
                    help="sweeps per chunk (default: 1000 for the steady workload, 500 for the "
                         "batched one, else 100)")
    ap.add_argument("--per-chunk", action="store_true",
                    help="launch every chunk separately (XS_PER_CHUNK) instead of the persistent "
                         "work-queue launch (speed only)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM counters)")
    ap.add_argument("--tts-runs", type=int, default=200,
                    help="headline: runs of the small single-instance workload for the TTS "
                         "block (0 = skip)")
    ap.add_argument("--workload", default="steady",
                    choices=["steady", "batched", "uneven", "serve", "tts", "w1scan", "paper",
                             "paper256", "single"],
                    help="steady: the default line, 16 x N=1024 x 2^20 clones, 10^4 sweeps; "
                         "batched: 64 x N=256 x 65536 clones to the first ground state or a "
                         "budget; uneven: 512 instances of uneven N and clone count, batched vs "
                         "served vs one at a time; serve: Poisson stream through the server vs "
                         "one run at a time; tts: the exponential TTS law on many runs of one "
                         "small instance, tau x N_cl scaling and the short-timeout estimate; "
                         "w1scan: mean TTS against w1 on one small instance, and the same w1 "
                         "with w0 = w1^3; paper: TTS_99 in seconds at the paper's clone count "
                         "(327,680) on planted N = 128 instances, one run at a time, and a "
                         "short-timeout estimate at N = 256; paper256: per-instance TTS_99 at "
                         "N = 256 by the short-timeout protocol; single: the N = 64, 1,024-clone "
                         "instance run to its first ground state with many seeds, one run at a "
                         "time vs all runs batched, and the oracle on the same runs")
    ap.add_argument("--accept-thr0", type=int, default=0,
                    help="batched: w0 threshold (w0 = thr0 / 65536); > 0 runs the w0 rule for "
                         "the full budget (a ground state is not absorbing, so no early stop)")
    ap.add_argument("--scan-n", type=int, default=100, help="w1scan: spins of the instance")
    ap.add_argument("--scan-w1", type=str, default="",
                    help="w1scan: comma-separated w1 values (default: 13 values, 0.03..0.20)")
    ap.add_argument("--cap", type=int, default=32,
                    help="largest colour class of the partition (the paper's 32); it fixes the "
                         "update order, so it changes trajectories, not the dynamics")
    ap.add_argument("--paper-instances", type=int, default=100, help="paper: N = 128 instances")
    ap.add_argument("--paper-runs", type=int, default=16, help="paper: runs per N = 128 instance")
    ap.add_argument("--paper-clones", type=int, default=327680,
                    help="paper: clones per run (the paper's 327,680 by default)")
    ap.add_argument("--paper-timeout-instances", type=int, default=32,
                    help="paper: N = 256 instances, one capped run each")
    ap.add_argument("--paper-timeout-sweeps", type=int, default=2000000,
                    help="paper: sweep cap of the N = 256 runs")
    ap.add_argument("--p256-first", type=int, default=0, help="paper256: first instance")
    ap.add_argument("--p256-instances", type=int, default=4, help="paper256: instances")
    ap.add_argument("--p256-runs", type=int, default=32, help="paper256: runs per instance")
    ap.add_argument("--p256-cap", type=int, default=1000000,
                    help="paper256: sweep cap of every run")
    ap.add_argument("--parts", default="batched,served,single",
                    help="uneven: which of batched, served, single (one run at a time) to run")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: arrival window (s)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="serve: device memory the server may hold for resident requests")
    return ap.parse_args()


def kernel_source_sha256():
    """Hash of the kernel sources: counter records name the source they were taken on."""
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.hip", "xs_internal.h"):
        with open(os.path.join(ROOT, "paper_2102_09510_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(args, wl, dims, updates_per_launch, kernel):
    """HBM bytes per sweep launch: the committed FETCH_SIZE/WRITE_SIZE record of the headline
    workload (HBM bytes per clone-spin update, from the scaled counters of whole launches)
    times this launch's updates, if the record was taken on the current kernel source, the
    same kernel and this workload's default configuration; otherwise None."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_RECORDS[wl])
    H = HEADLINES[wl]
    if (not os.path.exists(path) or dims != (H["count"], H["n"], H["clones"]) or
            (args.chunk or H["chunk"]) != H["chunk"] or args.accept_thr0 or args.cap != 32):
        return None
    rec = json.load(open(path))
    if kernel_source_sha256() != rec.get("kernel_source_sha256") or rec.get("kernel") != kernel:
        return None
    return rec["hbm_bytes_per_update"] * updates_per_launch


def cpu_baseline(insts, args, target_s):
    """The oracle on a bounded sample: every instance, one 256-clone block, S sweeps."""
    import oracle

    threads = os.cpu_count() or 1
    perms = [oracle.colour(i.tri, args.cap)[0] for i in insts]
    # calibrate on one instance
    t0 = time.perf_counter()
    oracle.run(insts[0].tri, insts[0].J, perms[0], seed=1, instance_id=0, thr=3604,
               thr0=args.accept_thr0, n_sweeps=200, clone_count=256, threads=threads)
    per_sweep = max((time.perf_counter() - t0) / 200, 1e-6)
    sweeps = int(max(10, min(5000, target_s / (per_sweep * len(insts)))))
    t0 = time.perf_counter()
    updates = 0
    for k, inst in enumerate(insts):
        oracle.run(inst.tri, inst.J, perms[k], seed=k, instance_id=k, thr=3604,
                   thr0=args.accept_thr0, n_sweeps=sweeps, clone_count=256, threads=threads)
        updates += 256 * inst.n * sweeps
    dt = time.perf_counter() - t0
    # one core: the first instance, 256 clones, a tenth of the sweeps
    s1 = max(10, sweeps // 10)
    t1 = time.perf_counter()
    oracle.run(insts[0].tri, insts[0].J, perms[0], seed=0, instance_id=0, thr=3604,
               thr0=args.accept_thr0, n_sweeps=s1, clone_count=256, threads=1)
    one = 256 * insts[0].n * s1 / (time.perf_counter() - t1) / 1e9
    return {"value": updates / dt / 1e9, "unit": "clone-spin updates/ns", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(insts)} instances x 256 clones x {sweeps} sweeps (N={insts[0].n}), "
                      f"{updates:.3e} updates in {dt:.1f} s; the rate on this sample is taken "
                      f"as the whole workload's (extrapolated)",
            "single_core_value": one,
            "single_core_sample": f"1 instance x 256 clones x {s1} sweeps, 1 thread"}


def pct(v, q):
    return float(np.percentile(v, q)) if len(v) else None


def workload_uneven(args, xorsat, torch):
    """512 planted instances of uneven N and clone count, each to its first ground state or
    10^4 sweeps: one batched run (a first call, which also builds the schedules, then a warm
    one), the server with every request queued at once, and one run per instance in sequence.
    Results are bit-identical across the three (checked). --parts picks which run."""
    from paper_2102_09510_amd.instances import (THR_PAPER, gen_seed, planted_instance, run_seed,
                                                uneven_sizes)

    parts = set(args.parts.split(","))
    sizes = uneven_sizes(512)
    insts = [planted_instance(n, gen_seed(4, k)) for k, (n, _) in enumerate(sizes)]
    hs = [xorsat.Instance(i.tri, i.J, colour_cap=args.cap) for i in insts]
    budget = args.budget if args.budget is not None else 10000

    def cfg(k):
        return xorsat.make_config(n_clones=sizes[k][1], seed=run_seed(4, k), instance_id=k,
                                  accept_thr=THR_PAPER, max_sweeps=budget, stop_on_first=True,
                                  chunk_sweeps=args.chunk or 100, per_chunk=args.per_chunk)

    print(f"# uneven: {len(sizes)} instances, budget {budget}, parts {sorted(parts)}",
          file=sys.stderr, flush=True)
    results = {}
    out = {"metric": "clone-spin updates/ns and completion latency, uneven batch",
           "config": {"workload": "512 planted instances, N uniform on {32..1024}, clones "
                                  "uniform on {4096..65536}, to first ground state or "
                                  f"{budget} sweeps"}}
    upd = None
    if "batched" in parts:
        times = []
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            batch = xorsat.run_batch(hs, [cfg(k) for k in range(len(hs))], want_energy=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            print(f"# batched run {rep} done in {times[-1]:.2f} s", file=sys.stderr, flush=True)
        upd = sum(o.clone_spin_updates for o in batch)
        results["batched"] = batch
        out["batched"] = {"seconds": round(times[1], 3),
                          "updates_per_ns": round(upd / times[1] / 1e9, 1),
                          "first_call_seconds": round(times[0], 3),
                          "launch": "persistent work queue" if batch[0].persistent
                          else "one per chunk",
                          "completion_s_p50": round(times[1], 3),
                          "completion_s_p99": round(times[1], 3)}
    if "served" in parts:
        srv = xorsat.Server(hbm_budget_bytes=int(args.serve_budget_gib * (1 << 30)))
        t0 = time.perf_counter()
        tickets = {srv.submit(hs[k], cfg(k), want_first_hit=False, want_energy=False): k
                   for k in range(len(hs))}
        served = {}
        while True:
            active = srv.step()
            for c in srv.poll():
                served[tickets[c.ticket]] = c
            if active == 0:
                break
        for c in srv.poll():
            served[tickets[c.ticket]] = c
        t_serve = time.perf_counter() - t0
        srv.close()
        print(f"# served run done in {t_serve:.2f} s", file=sys.stderr, flush=True)
        results["served"] = [served[k] for k in range(len(hs))]
        upd_s = sum(c.clone_spin_updates for c in results["served"])
        lat = [served[k].latency_s for k in range(len(hs))]
        out["served"] = {"seconds": round(t_serve, 3),
                         "updates_per_ns": round(upd_s / t_serve / 1e9, 1),
                         "completion_s_p50": pct(lat, 50), "completion_s_p99": pct(lat, 99)}
    if "single" in parts:
        single_done, single = [], []
        t0 = time.perf_counter()
        for k in range(len(hs)):
            single.append(xorsat.run(hs[k], cfg(k), want_energy=False))
            torch.cuda.synchronize()
            single_done.append(time.perf_counter() - t0)
        t_single = single_done[-1]
        print(f"# one-at-a-time done in {t_single:.2f} s", file=sys.stderr, flush=True)
        results["single"] = single
        upd_1 = sum(o.clone_spin_updates for o in single)
        out["one_at_a_time"] = {"seconds": round(t_single, 3),
                                "updates_per_ns": round(upd_1 / t_single / 1e9, 1),
                                "completion_s_p50": pct(single_done, 50),
                                "completion_s_p99": pct(single_done, 99)}
    keys = {name: [(o.tts_sweeps, o.winner_clone, o.end_sweep) for o in res]
            for name, res in results.items()}
    assert len({tuple(v) for v in keys.values()}) <= 1, "results differ between parts"
    first = next(iter(results.values()))
    tts = [o.tts_sweeps for o in first if o.tts_sweeps >= 0]
    out["tts_sweeps"] = {"solved": len(tts), "censored": len(hs) - len(tts),
                         "p50": pct(tts, 50), "p99": pct(tts, 99)}
    out["identical_results"] = True if len(results) > 1 else None  # None: one part, nothing to compare
    return out


def workload_serve(args, xorsat, torch):
    """Poisson arrivals of planted instances (N log-uniform in [64, 2048], 16384 clones, first
    ground state or 10^4 sweeps) through the server, then the first requests of the same stream
    served one run at a time in arrival order (FIFO) for comparison."""
    from paper_2102_09510_amd.instances import (THR_PAPER, gen_seed, planted_instance,
                                                poisson_stream, run_seed)

    arrivals = poisson_stream(args.rate, args.duration)
    budget = args.budget if args.budget is not None else 10000
    print(f"# serve: {len(arrivals)} requests over {args.duration} s, preparing instances",
          file=sys.stderr, flush=True)
    hs = []
    for k, (_, n) in enumerate(arrivals):
        inst = planted_instance(n, gen_seed(5, k))
        hs.append(xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap))

    def cfg(k):
        return xorsat.make_config(n_clones=16384, seed=run_seed(5, k), instance_id=k,
                                  accept_thr=THR_PAPER, max_sweeps=budget, stop_on_first=True,
                                  chunk_sweeps=args.chunk or 100)

    srv = xorsat.Server(hbm_budget_bytes=int(args.serve_budget_gib * (1 << 30)))
    tickets = {}
    done = {}
    nxt = 0
    max_resident = 0
    print("# serving", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    last_report = t0
    while nxt < len(arrivals) or len(done) < len(arrivals):
        now = time.perf_counter() - t0
        while nxt < len(arrivals) and arrivals[nxt][0] <= now:
            tickets[srv.submit(hs[nxt], cfg(nxt), want_first_hit=False, want_energy=False)] = nxt
            nxt += 1
        active = srv.step()
        for c in srv.poll():
            done[tickets[c.ticket]] = c
        max_resident = max(max_resident, srv.stats()["resident"])
        if time.perf_counter() - last_report > 10:
            last_report = time.perf_counter()
            print(f"# t={last_report - t0:.0f}s submitted {nxt} done {len(done)} "
                  f"resident {srv.stats()['resident']}", file=sys.stderr, flush=True)
        if active == 0 and nxt < len(arrivals):
            time.sleep(max(0.0, min(0.002, arrivals[nxt][0] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = [done[k].latency_s for k in range(len(arrivals))]
    solved = [k for k in range(len(arrivals)) if done[k].tts_sweeps >= 0]
    tts = [done[k].tts_sweeps for k in solved]
    # One run at a time, FIFO in arrival order, on the first requests of the same stream.
    m = min(len(arrivals), 400)
    finish = 0.0
    single_lat = []
    service = []
    print(f"# one-at-a-time on the first {m} requests", file=sys.stderr, flush=True)
    for k in range(m):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o = xorsat.run(hs[k], cfg(k), want_energy=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        assert (o.tts_sweeps, o.end_sweep) == (done[k].tts_sweeps, done[k].end_sweep), k
        service.append(dt)
        start = max(arrivals[k][0], finish)
        finish = start + dt
        single_lat.append(finish - arrivals[k][0])
    offered = sum(service) / max(arrivals[m - 1][0], 1e-9)
    return {"metric": "served TTS latency p50/p99 and sustained clone-spin updates/ns",
            "config": {"workload": f"Poisson stream, {args.rate}/s for {args.duration} s "
                                   f"({len(arrivals)} requests), N log-uniform in [64, 2048], "
                                   f"16384 clones, first ground state or {budget} sweeps",
                       "hbm_budget_gib": args.serve_budget_gib},
            "served": {"wall_s": round(wall, 2),
                       "sustained_updates_per_ns": round(st["clone_spin_updates"] / wall / 1e9, 1),
                       "latency_s_p50": pct(lat, 50), "latency_s_p99": pct(lat, 99),
                       "solved": len(solved), "censored": len(arrivals) - len(solved),
                       "solved_latency_s_p50": pct([lat[k] for k in solved], 50),
                       "solved_latency_s_p99": pct([lat[k] for k in solved], 99),
                       "tts_sweeps_p50": pct(tts, 50), "tts_sweeps_p99": pct(tts, 99),
                       "max_resident": max_resident, "steps": st["steps"]},
            "one_at_a_time_first_requests": {
                "requests": m, "latency_s_p50": pct(single_lat, 50),
                "latency_s_p99": pct(single_lat, 99),
                "service_s_mean": float(np.mean(service)),
                "offered_load": round(offered, 2),
                "same_requests_served_latency_s_p50": pct(lat[:m], 50),
                "same_requests_served_latency_s_p99": pct(lat[:m], 99)},
            "identical_results_checked": m}


def workload_tts(args, xorsat, torch):
    """Many independent runs (different seeds) of one planted N = 80 instance at two clone
    counts: the fastest-clone TTS law (Eq. 2), tau estimators, tau x N_cl (SM), and tau from
    runs capped at a short timeout (inverse-gamma posterior)."""
    from paper_2102_09510_amd import tts_stats as ts
    from paper_2102_09510_amd.instances import THR_PAPER, gen_seed, planted_instance

    n, runs = 80, 512
    inst = planted_instance(n, gen_seed(6, 0))
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap)
    out = {"metric": "TTS distribution of many-clone runs (sweeps)",
           "config": {"workload": f"1 planted instance, N={n}, {runs} runs per clone count, "
                                  "to first ground state"}}
    taus = {}
    for ncl in (1024, 4096):
        cfgs = [xorsat.make_config(n_clones=ncl, seed=0xC0FFEE + 7919 * r, instance_id=r,
                                   accept_thr=THR_PAPER, max_sweeps=10**6, stop_on_first=True,
                                   chunk_sweeps=20) for r in range(runs)]
        t0 = time.perf_counter()
        res = xorsat.run_batch([h] * runs, cfgs, want_energy=False)
        dt = time.perf_counter() - t0
        tts = np.array([r.tts_sweeps for r in res])
        assert (tts >= 0).all()
        s = ts.summarize(tts, n_clones=ncl)
        s["seconds"] = round(dt, 2)
        taus[ncl] = s["tau"]
        # short timeout: cap every run at tau/10 and estimate tau from the successes alone
        cap = max(1, int(s["tau"] / 10))
        n_succ = int((tts < cap).sum())
        post = ts.TimeoutPosterior(n_succ, runs, cap)
        s["timeout"] = {"t_max": cap, "successes": n_succ,
                        "tau_posterior_mean": post.mean() if n_succ > 1 else None,
                        "tau_posterior_median": post.quantile(0.5) if n_succ > 0 else None}
        out[f"clones_{ncl}"] = s
        print(f"# {ncl} clones: tau {s['tau']:.1f} sweeps, KS p {s['ks_pvalue']:.3f}", file=sys.stderr, flush=True)
    out["tau_ratio_1024_over_4096"] = taus[1024] / taus[4096]
    out["shifted_scale_ratio_1024_over_4096"] = (out["clones_1024"]["shifted_scale"] /
                                                 out["clones_4096"]["shifted_scale"])
    out["tail_tau_ratio_1024_over_4096"] = (out["clones_1024"]["tail_tau"] /
                                            out["clones_4096"]["tail_tau"])
    return out


def workload_w1scan(args, xorsat, torch):
    """Mean TTS against w1 (Section "Numerical results": w1 was chosen at the minimum of a
    quadratic fit of the mean TTS) on one planted instance, many runs per value; then the same
    pseudo-temperatures with w0 = w1^3 (detailed balance), scored by the share of runs whose end
    configuration holds a ground state after as many sweeps as the quasi-greedy median TTS."""
    from paper_2102_09510_amd import tts_stats as ts
    from paper_2102_09510_amd.instances import gen_seed, planted_instance

    n, runs, ncl, cap = args.scan_n, 512, 1024, 400000
    w1s = ([float(v) for v in args.scan_w1.split(",")] if args.scan_w1 else
           [0.03, 0.04, 0.05, 0.055, 0.06, 0.07, 0.08, 0.09, 0.10, 0.12, 0.14, 0.17, 0.20])
    inst = planted_instance(n, gen_seed(7, 0))
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap)
    rows, times_of = [], {}
    for w1 in w1s:
        thr = round(w1 * 65536)
        cfgs = [xorsat.make_config(n_clones=ncl, seed=0xBEEF + 104729 * r, instance_id=r,
                                   accept_thr=thr, max_sweeps=cap, stop_on_first=True,
                                   chunk_sweeps=20) for r in range(runs)]
        t0 = time.perf_counter()
        res = xorsat.run_batch([h] * runs, cfgs, want_energy=False)
        dt = time.perf_counter() - t0
        tts = np.array([r.tts_sweeps for r in res])
        solved = tts >= 0
        times = np.where(solved, tts, cap)
        times_of[w1] = times
        tau = ts.tau_censored_mle(times, solved)
        rows.append({"w1": w1, "accept_thr": thr, "mean_tts": float(times.mean()),
                     "tau": tau, "p50": float(np.percentile(times, 50)),
                     "censored": int((~solved).sum()), "seconds": round(dt, 2)})
        print(f"# w1 {w1}: mean TTS {times.mean():.0f} sweeps, {dt:.1f} s", file=sys.stderr,
              flush=True)
    w = np.array([r["w1"] for r in rows])
    m = np.array([r["mean_tts"] for r in rows])
    k = int(np.argmin(m))
    lo, hi = max(0, k - 2), min(len(w), k + 3)
    w_opt = None
    if hi - lo >= 3:
        c2, c1, _ = np.polyfit(w[lo:hi], m[lo:hi], 2)
        w_opt = float(-c1 / (2 * c2)) if c2 > 0 else None
    # w0 = w1^3 at the same pseudo-temperatures, fixed budget
    budget = int(next((r["p50"] for r in rows if r["w1"] == 0.055), rows[0]["p50"]))
    met = []
    for w1 in w1s:
        thr, thr0 = round(w1 * 65536), max(1, round(w1 ** 3 * 65536))
        cfgs = [xorsat.make_config(n_clones=ncl, seed=0xBEEF + 104729 * r, instance_id=r,
                                   accept_thr=thr, accept_thr0=thr0, max_sweeps=budget,
                                   stop_on_first=False, chunk_sweeps=100) for r in range(runs)]
        res = xorsat.run_batch([h] * runs, cfgs, want_energy=False)
        ok = sum(1 for r in res if r.tts_sweeps >= 0)
        met.append({"w1": w1, "accept_thr0": thr0, "runs_in_ground_state_at_end": ok,
                    "quasi_greedy_runs_solved_by_then": int((times_of[w1] <= budget).sum())})
        print(f"# w1 {w1}, w0 = w1^3: {ok}/{runs} runs end in a ground state", file=sys.stderr,
              flush=True)
    return {"metric": "mean TTS (sweeps) against w1",
            "config": {"workload": f"1 planted instance, N={n}, {ncl} clones, {runs} runs per "
                                   f"w1, to first ground state (cap {cap} sweeps)"},
            "quasi_greedy": rows, "quadratic_fit_w1_min": w_opt,
            "w0_eq_w1_cubed": {"budget_sweeps": budget, "runs": runs, "rows": met}}


def workload_paper(args, xorsat, torch):
    """The paper's headline quantity on synthetic planted instances (Section "Numerical
    results", Table 1: TTS_99 of the median instance, 327,680 clones, w1 = 0.055, one run on the
    GPU at a time), at the paper's clone count unless --paper-clones says otherwise. N = 128:
    every run to its first ground state, tau of an
    instance = mean wall time of its runs, TTS_99 = ln(100) tau. N = 256: runs capped at a short
    timeout (Section "Running with a short timeout"); with few successes per instance the
    instances are pooled into one posterior (inverse-gamma with shape = successes and scale =
    total capped time)."""
    from paper_2102_09510_amd import tts_stats as ts
    from paper_2102_09510_amd.instances import THR_PAPER, gen_seed, planted_instance

    ncl = args.paper_clones
    out = {"metric": f"TTS_99 (s) of the median instance, {ncl} clones, w1 = 0.055",
           "config": {"workload": "planted instances, one run at a time"}}
    # N = 128: full runs
    n, count, runs = 128, args.paper_instances, args.paper_runs
    taus, taus_sw = [], []
    t_all = time.perf_counter()
    for k in range(count):
        inst = planted_instance(n, gen_seed(8, k))
        h = xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap)
        secs, sweeps = [], []
        for r in range(runs):
            cfg = xorsat.make_config(n_clones=ncl, seed=0x5EED + 7919 * r + 104729 * k,
                                     instance_id=k, accept_thr=THR_PAPER, max_sweeps=10**7,
                                     stop_on_first=True, chunk_sweeps=100)
            o = xorsat.run(h, cfg, want_energy=False)
            assert o.tts_sweeps >= 0
            secs.append(o.seconds)
            sweeps.append(o.tts_sweeps)
        taus.append(float(np.mean(secs)))
        taus_sw.append(float(np.mean(sweeps)))
        if k % 10 == 9:
            print(f"# N=128: {k + 1} instances, {time.perf_counter() - t_all:.1f} s",
                  file=sys.stderr, flush=True)
    ln100 = math.log(100.0)
    out["n128"] = {"instances": count, "runs_per_instance": runs,
                   "tts99_s_median": ln100 * float(np.median(taus)),
                   "tts99_s_p10_p90": [ln100 * float(np.percentile(taus, 10)),
                                       ln100 * float(np.percentile(taus, 90))],
                   "tau_sweeps_median": float(np.median(taus_sw)),
                   "paper_tts99_s_v100": 0.0275}
    # N = 256: short timeout, pooled
    n, count, cap = 256, args.paper_timeout_instances, args.paper_timeout_sweeps
    hs = []
    for k in range(count):
        inst = planted_instance(n, gen_seed(9, k))
        hs.append(xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap))
    cfgs = [xorsat.make_config(n_clones=ncl, seed=0xFACE + 104729 * k, instance_id=k,
                               accept_thr=THR_PAPER, max_sweeps=cap, stop_on_first=True,
                               chunk_sweeps=100) for k in range(count)]
    print(f"# N=256: {count} runs capped at {cap} sweeps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = []
    for g in range(0, count, 8):  # groups of 8 runs, so that progress shows
        res += xorsat.run_batch(hs[g:g + 8], cfgs[g:g + 8], want_energy=False)
        print(f"# N=256: {len(res)} runs done, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    succ = sum(1 for o in res if o.tts_sweeps >= 0)
    # seconds per sweep of one run alone at this size
    o1 = xorsat.run(hs[0], xorsat.make_config(n_clones=ncl, seed=1, instance_id=0,
                                               accept_thr=THR_PAPER, max_sweeps=2000,
                                               stop_on_first=False, chunk_sweeps=100),
                    want_energy=False)
    s_per_sweep = o1.seconds / 2000
    n256 = {"runs": count, "cap_sweeps": cap, "successes": succ, "seconds": round(dt, 1),
            "seconds_per_sweep_one_run": s_per_sweep, "paper_tts99_s_v100": 640.0}
    if succ:
        post = ts.TimeoutPosterior(succ, count, cap)
        q = [post.quantile(0.16), post.quantile(0.5), post.quantile(0.84)]
        n256.update(tau_sweeps_posterior_median=q[1], tau_sweeps_68=[q[0], q[2]],
                    tts99_s_pooled=ln100 * q[1] * s_per_sweep,
                    tts99_s_pooled_68=[ln100 * q[0] * s_per_sweep, ln100 * q[2] * s_per_sweep])
    out["n256_timeout"] = n256
    return out


def workload_paper256(args, xorsat, torch):
    """Per-instance TTS_99 at N = 256 by the paper's short-timeout protocol (Section "Running
    with a short timeout"): R runs of each instance capped at a sweep budget, tau of the instance
    from the exact posterior of its successes, TTS_99 = ln(100) tau in seconds of one run
    alone; the median over instances is the Table 1 quantity. Instances k0 .. k0 + K - 1, so
    that the set can be split over several invocations."""
    from paper_2102_09510_amd import tts_stats as ts
    from paper_2102_09510_amd.instances import THR_PAPER, gen_seed, planted_instance

    ncl, runs, cap = args.paper_clones, args.p256_runs, args.p256_cap
    k0, count = args.p256_first, args.p256_instances
    n = 256
    ln100 = math.log(100.0)
    per = []
    t_all = time.perf_counter()
    s_per_sweep = None
    for k in range(k0, k0 + count):
        inst = planted_instance(n, gen_seed(9, k))
        h = xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap)
        if s_per_sweep is None:
            # seconds per sweep of one run alone, from the second of two runs (the first one
            # pays the process's one-time set-up)
            for _ in range(2):
                o1 = xorsat.run(h, xorsat.make_config(n_clones=ncl, seed=1, instance_id=k,
                                                      accept_thr=THR_PAPER, max_sweeps=5000,
                                                      stop_on_first=False, chunk_sweeps=100),
                                want_energy=False)
            s_per_sweep = o1.seconds / 5000
        tts = []
        for g in range(0, runs, 8):  # groups of 8 runs of the instance, so that progress shows
            m = min(8, runs - g)
            cfgs = [xorsat.make_config(n_clones=ncl, seed=0xBEEF + 7919 * (g + j) + 104729 * k,
                                       instance_id=k, accept_thr=THR_PAPER, max_sweeps=cap,
                                       stop_on_first=True, chunk_sweeps=100) for j in range(m)]
            outs = xorsat.run_batch([h] * m, cfgs, want_energy=False)
            tts += [o.tts_sweeps for o in outs]
            print(f"# N=256 instance {k}: {len(tts)} runs, {sum(t >= 0 for t in tts)} solved, "
                  f"{time.perf_counter() - t_all:.0f} s", file=sys.stderr, flush=True)
        solved = [t for t in tts if t >= 0]
        rec = {"instance": k, "runs": runs, "solved": len(solved)}
        if 0 < len(solved) < runs:
            q = ts.timeout_posterior_quantiles(len(solved), runs, cap)
            rec.update(tau_sweeps=q[1], tau_sweeps_68=[q[0], q[2]])
        elif len(solved) == runs:
            rec.update(tau_sweeps=float(np.mean(solved)))  # nothing censored
        if "tau_sweeps" in rec:
            rec["tts99_s"] = ln100 * rec["tau_sweeps"] * s_per_sweep
        per.append(rec)
    done = [r["tts99_s"] for r in per if "tts99_s" in r]
    return {"metric": f"TTS_99 (s) per instance, N=256, {ncl} clones, w1 = 0.055",
            "config": {"workload": f"planted instances {k0}..{k0 + count - 1}, {runs} runs "
                                   f"each capped at {cap} sweeps"},
            "seconds_per_sweep_one_run": s_per_sweep, "instances": per,
            "tts99_s_median": float(np.median(done)) if done else None,
            "unsolved_instances": sum(1 for r in per if r["solved"] == 0),
            "paper_tts99_s_v100": 640.0}


def workload_single(args, xorsat, torch):
    """One planted N = 64 instance, 1,024 clones, first ground state or 10^5 sweeps, R seeds:
    TTS in sweeps (p50/p99), wall time per run one at a time, the R runs batched in one call,
    and the CPU oracle timed on the first runs (its TTS must equal the GPU's)."""
    from paper_2102_09510_amd.instances import THR_PAPER, gen_seed, planted_instance, run_seed

    n, ncl, runs = 64, 1024, 200
    inst = planted_instance(n, gen_seed(1, 0))
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap)

    def cfg(r):
        return xorsat.make_config(n_clones=ncl, seed=run_seed(1, 0) + r, instance_id=0,
                                  accept_thr=THR_PAPER, max_sweeps=100000, stop_on_first=True,
                                  chunk_sweeps=args.chunk or 100)

    xorsat.run(h, cfg(0))  # warm
    torch.cuda.synchronize()
    one, secs = [], []
    for r in range(runs):
        t1 = time.perf_counter()
        o = xorsat.run(h, cfg(r), want_energy=False)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t1)
        one.append(o.tts_sweeps)
    # The first batched call also pays one-time costs outside the sweeps: the process's first
    # graph instantiation and, in Python, a full garbage collection set off by the call's
    # allocations. The second, identical call shows the steady cost.
    t_batch = []
    for _ in range(2):
        t0 = time.perf_counter()
        batch = xorsat.run_batch([h] * runs, [cfg(r) for r in range(runs)], want_energy=False)
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - t0)
        assert [o.tts_sweeps for o in batch] == one
    tts = np.array(one)
    return {"metric": "TTS (sweeps, seconds) of single runs, N=64, 1024 clones",
            "config": {"workload": f"1 planted instance, N={n}, {ncl} clones, {runs} seeds, "
                                   "first ground state or 1e5 sweeps"},
            "solved": int((tts >= 0).sum()),
            "tts_sweeps_p50": pct(tts[tts >= 0], 50), "tts_sweeps_p99": pct(tts[tts >= 0], 99),
            "one_at_a_time_s_p50": pct(secs, 50), "one_at_a_time_s_p99": pct(secs, 99),
            "batched_all_runs_s": round(t_batch[1], 4),
            "batched_all_runs_first_call_s": round(t_batch[0], 4),
            "cpu_baseline": cpu_baseline_single(inst, args.cap, [cfg(r) for r in range(20)],
                                                [o.sweeps_done for o in batch[:20]], one[:20])}


def cpu_baseline_single(inst, cap, cfgs, sweeps, tts):
    """The oracle on the first single runs in full (every clone up to the GPU's end sweep),
    timed; its TTS must equal the GPU's."""
    import oracle

    threads = os.cpu_count() or 1
    perm, _ = oracle.colour(inst.tri, cap)
    t0 = time.perf_counter()
    for c, s, want in zip(cfgs, sweeps, tts):
        ref = oracle.run(inst.tri, inst.J, perm, seed=c.seed, instance_id=c.instance_id,
                         thr=c.accept_thr, n_sweeps=s, clone_count=c.n_clones, threads=threads)
        assert oracle.solve_results(ref["first_hit"])[0] == want
    dt = time.perf_counter() - t0
    return {"value": round(dt / len(cfgs), 4), "unit": "s per run", "cores": threads,
            "kind": "oracle", "sample": f"{len(cfgs)} runs in full, TTS equal to the GPU's"}


def tts_block(args, xorsat, torch):
    """TTS of the small single-instance workload (one planted N = 64 instance, 1,024 clones, to
    the first ground state or 10^5 sweeps) over many seeds, three ways on the same GPU: one run
    at a time, all runs in one batched call, and all runs submitted at once to the server. TTS
    in sweeps is identical by construction (checked); the wall-clock times differ. All runs
    arrive together, so a run's completion time is its place in the one-at-a-time sequence,
    the batched call's end, or its own completion in the server."""
    from paper_2102_09510_amd.instances import THR_PAPER, gen_seed, planted_instance, run_seed

    runs, n, ncl = args.tts_runs, 64, 1024
    inst = planted_instance(n, gen_seed(1, 0))
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=args.cap)

    def cfg(r):
        return xorsat.make_config(n_clones=ncl, seed=run_seed(1, 0) + r, instance_id=0,
                                  accept_thr=THR_PAPER, max_sweeps=100000, stop_on_first=True,
                                  chunk_sweeps=args.chunk or 100)

    xorsat.run(h, cfg(0))  # warm
    torch.cuda.synchronize()
    one, service = [], []
    for r in range(runs):
        t1 = time.perf_counter()
        o = xorsat.run(h, cfg(r), want_energy=False)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t1)
        one.append(o.tts_sweeps)
    completion = np.cumsum(service)
    batch_s = []
    for _ in range(2):  # the first call also pays one-time costs (graph instantiation)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch = xorsat.run_batch([h] * runs, [cfg(r) for r in range(runs)], want_energy=False)
        torch.cuda.synchronize()
        batch_s.append(time.perf_counter() - t0)
        assert [o.tts_sweeps for o in batch] == one
    srv = xorsat.Server(hbm_budget_bytes=1 << 30)
    t0 = time.perf_counter()
    tickets = {srv.submit(h, cfg(r), want_first_hit=False, want_energy=False): r
               for r in range(runs)}
    served = {}
    while True:
        active = srv.step()
        for c in srv.poll():
            served[tickets[c.ticket]] = c
        if active == 0:
            break
    for c in srv.poll():
        served[tickets[c.ticket]] = c
    served_s = time.perf_counter() - t0
    srv.close()
    assert [served[r].tts_sweeps for r in range(runs)] == one
    lat = [served[r].latency_s for r in range(runs)]
    tts = np.array(one)
    ok = tts[tts >= 0]

    def ms(v):
        return None if v is None else round(1e3 * v, 3)

    return {"workload": f"1 planted instance, N={n}, {ncl} clones, {runs} seeds, first ground "
                        "state or 1e5 sweeps, all runs arriving together",
            "solved": int(ok.size), "censored": int(runs - ok.size),
            "tts_sweeps_p50": pct(ok, 50), "tts_sweeps_p99": pct(ok, 99),
            "one_at_a_time": {"service_ms_p50": ms(pct(service, 50)),
                              "service_ms_p99": ms(pct(service, 99)),
                              "completion_ms_p50": ms(pct(completion, 50)),
                              "completion_ms_p99": ms(pct(completion, 99)),
                              "total_ms": ms(completion[-1])},
            "batched": {"completion_ms": ms(batch_s[1]), "total_ms": ms(batch_s[1]),
                        "first_call_ms": ms(batch_s[0])},
            "served": {"completion_ms_p50": ms(pct(lat, 50)),
                       "completion_ms_p99": ms(pct(lat, 99)), "total_ms": ms(served_s)},
            "identical_tts": True}


def headline(args, xorsat, torch):
    """The JSON line of a headline workload: W untimed steps, then K timed steps bracketed by
    device synchronisations; every sweep-chunk launch timed with HIP events on the stream it is
    launched on."""
    from paper_2102_09510_amd.instances import THR_PAPER, gen_seed, planted_instance, run_seed

    wl = args.workload
    H = HEADLINES[wl]
    count = args.instances or H["count"]
    n = args.n or H["n"]
    clones = args.clones or H["clones"]
    budget = args.budget if args.budget is not None else H["budget"]
    stop = H["stop"] and args.accept_thr0 == 0
    place = args.place_rows or wl in ("steady", "batched")
    chunk = args.chunk or H["chunk"]
    insts = [planted_instance(n, gen_seed(H["config"], k)) for k in range(count)]
    handles = [xorsat.Instance(i.tri, i.J, colour_cap=args.cap) for i in insts]

    def step(s):
        cfgs = [xorsat.make_config(n_clones=clones, seed=run_seed(H["config"], k) + s,
                                   instance_id=k, accept_thr=THR_PAPER,
                                   accept_thr0=args.accept_thr0, max_sweeps=budget,
                                   stop_on_first=stop, chunk_sweeps=chunk, place_rows=place,
                                   per_chunk=args.per_chunk)
                for k in range(count)]
        return xorsat.run_batch(handles, cfgs, want_energy=True)

    print(f"# bench {wl}: {count} x N={n} x {clones} clones, {budget} sweeps/step"
          f"{' or first ground state' if stop else ''}, warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)
    for s in range(args.warmup):
        step(1000 + s)
        torch.cuda.synchronize()
        print(f"# warmup step {s} done", file=sys.stderr, flush=True)
    xorsat.profile_read(reset=True)
    xorsat.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0
    tts = []
    censored = 0
    shape = None
    for s in range(args.steps):
        outs = step(s)
        for o in outs:
            updates += o.clone_spin_updates
            if o.tts_sweeps >= 0:
                tts.append(o.tts_sweeps)  # runs start at sweep 0
            else:
                censored += 1
        shape = (outs[0].tile_blocks, outs[0].wg_threads, outs[0].col_bytes, outs[0].rec_global)
        persistent = bool(outs[0].persistent)
        print(f"# step {s} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    xorsat.profile_enable(False)
    prof = xorsat.profile_read(reset=True)
    value = updates / dt / 1e9
    kern_rate = prof["clone_spin_updates"] / (prof["total_ms"] * 1e6) if prof["total_ms"] else 0
    # Persistent launches: one launch runs up to a whole epoch of chunks of every instance, so
    # the figures are per launch as rocprofv3 lists them. Launch per chunk: a launch covers
    # `chunk` sweeps of every instance; launches after the budget ran out (every tile exits at
    # once, a few us each) are counted apart, their time stays in.
    if persistent:
        full_launches = prof["launches"]
        per_launch_updates = prof["clone_spin_updates"] / max(full_launches, 1)
    else:
        per_launch_updates = count * clones * n * chunk
        full_launches = prof["clone_spin_updates"] / per_launch_updates
    avg_ms = prof["total_ms"] / max(full_launches, 1e-9)
    lds_tbs = ALGO_LDS_BYTES_PER_UPDATE * per_launch_updates / (avg_ms * 1e-3) / 1e12
    ops = ALGO_OPS_PER_UPDATE_W0 if args.accept_thr0 else ALGO_OPS_PER_UPDATE
    valu = ops * per_launch_updates / (avg_ms * 1e-3) / 1e12
    desc = (f"{count} planted instances, N={n}, {clones} clones each, batched, " +
            (f"{budget} sweeps per step with w0 = {args.accept_thr0}/65536" if args.accept_thr0
             else f"to first ground state or {budget} sweeps per step" if stop
             else f"{budget} sweeps per step (steady state)"))
    line = {
        "metric": "clone-spin updates/ns on 1 MI355X",
        "value": round(value, 3),
        "unit": "clone-spin updates/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic planted instances (seeded configuration model)",
        "config": {"workload": desc, "chunk_sweeps": chunk, "accept_thr": THR_PAPER,
                   "colour_cap": args.cap, "launch_shape": dict(zip(
                       ("tile_blocks", "wg_threads", "col_bytes", "rec_global"), shape)),
                   "launch": "persistent work queue" if persistent else "one per chunk",
                   **({"accept_thr0": args.accept_thr0} if args.accept_thr0 else {}),
                   **({"place_rows": True} if place else {})},
        "tts_sweeps": {"solved": len(tts), "censored": censored,
                       "p50": pct(tts, 50), "p99": pct(tts, 99)},
        "roofline": {"bound": "lds", "achieved": round(lds_tbs, 3),
                     "peak": round(LDS_PEAK_TBS, 2), "unit": "TB/s",
                     "frac": round(lds_tbs / LDS_PEAK_TBS, 4),
                     "traffic": measured_traffic(args, wl, (count, n, clones), per_launch_updates,
                                                 "qg_queue_run" if persistent else "qg_chunk"),
                     "bytes_per_update": ALGO_LDS_BYTES_PER_UPDATE,
                     "kernel": "qg_queue_run" if persistent else "qg_chunk",
                     "launches": round(full_launches, 2),
                     "launches_past_budget": 0 if persistent
                     else prof["launches"] - round(full_launches),
                     "updates_per_launch": per_launch_updates,
                     "avg_launch_ms": round(avg_ms, 3),
                     "kernel_updates_per_ns": round(kern_rate, 3),
                     "valu": {"algorithmic_ops_per_update": round(ops, 4),
                              "achieved_T_ops": round(valu, 3),
                              "peak_T_ops": round(VALU_PEAK_TOPS, 2),
                              "frac_if_full_rate": round(valu / VALU_PEAK_TOPS, 4)}},
    }
    if args.tts_runs > 0:
        print("# TTS block: one at a time, batched, served", file=sys.stderr, flush=True)
        line["tts_batched_vs_single"] = tts_block(args, xorsat, torch)
    if args.cpu_seconds > 0:
        print("# CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(insts, args, args.cpu_seconds)
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; several GPUs would each take "
                                   "a share of the 32-clone groups and combine first hits with "
                                   "one min-reduction, which is not implemented here",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2102_09510_amd import xorsat

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibrate:
        src = torch.ones(args.copy_calibrate << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return
    if args.workload not in HEADLINES:
        fn = {"uneven": workload_uneven, "serve": workload_serve, "tts": workload_tts,
              "w1scan": workload_w1scan, "paper": workload_paper,
              "paper256": workload_paper256, "single": workload_single}[args.workload]
        out = fn(args, xorsat, torch)
        out.setdefault("config", {})["colour_cap"] = args.cap
        print(json.dumps(out), flush=True)
        return
    print(json.dumps(headline(args, xorsat, torch)), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the dose engine on one MI355X.

Workload: the synthetic CT patient (256x256x128 voxels of 0.2x0.2x0.25 cm,
4 materials + density from seeded ellipsoids), a 9-beam coplanar IMRT plan with
40x40 beamlet fluence maps and the 6 MV-like triangular spectrum, run until the
mean sigma/D_max over D > D_max/2 is at most 1% (the paper's Table 3 reports
this quantity for its IMRT/VMAT plans).  One step is one such dose job with a
different seed; `value` is histories per second over the timed jobs, with the
phantom, source and tables already resident in device memory.

Also reported: the job latency (p50/p99 over the timed jobs), the roofline
position of the dominant transport kernel (HIP-event times of every launch on
the library's stream; algorithmic bytes from the kernels' own counters of voxel
lookups, queue records and tally deposits; measured HBM traffic from the
committed hardware-counter summary), and the oracle (plain CPU transport) timed
on a bounded sample of the same job.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "histories/s at 1% unc. (6MV, 256x256x128 CT phantom); p50/p99 dose-job latency"

# Algorithmic memory traffic of the transport passes (bytes per unit of work):
# every Woodcock flight and every electron step needs the density and material
# of one voxel (one packed 4-byte word), every particle taken from or put into a
# queue is a 64-byte record, and every tally deposit is one FP64 value.
BYTES_PER_VOXEL_LOOKUP = 4
BYTES_PER_RECORD = 64
BYTES_PER_DEPOSIT = 8
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
# vector-ALU lane instructions: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64
# instruction occupies a SIMD for 4 cycles; unpacked FP32 = 78.6 TFLOP/s of FMA)
PEAK_VALU_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
# the kernels and the compile-time constants they are built with: a profile is
# valid while the sha256 of these files, read in this order, is unchanged
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1107_3355_amd", "csrc", f)
                  for f in ("transport.hip", "dev_types.h")]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "traffic_ct256x256x128_imrt9.txt")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "counters_ct256x256x128_imrt9.txt")
EVENT_COST_SUMMARY = os.path.join(ROOT, "profiles", "event_cost_solo_lanes.txt")
# Regressors of a transport kernel's VALU instructions in the one-particle-per-
# wavefront form: wavefronts launched (set-up, table staging, the end of the
# pass), records loaded, and the kernel's events.
# A run's records loaded are the queue positions its passes read, empty ones
# included (with one particle per wavefront most of a wavefront's push
# reservation stays empty, and each empty position costs a refill).
EVENT_TERMS = {
    "k_photon": ("waves", "records_loaded", "flights", "compton", "photo", "pair"),
    "k_electron": ("waves", "records_loaded", "esteps", "moller", "brems"),
}
# (a pass's stores and deposits follow its interactions and steps nearly in
# proportion: as regressors they would be collinear with those counts, so the
# cost of an interaction or a step includes its pushes and deposits)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    """Oracle threads: the host cores this process may use, at most 16 (a GPU
    box gives each GPU a share of 16 cores, whatever the machine has)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(workload, seconds):
    """The oracle as it stands, on a bounded sample of the same job: a probe run
    sizes the sample so that the timed run takes about `seconds`."""
    import oracle
    from paper_1107_3355_amd import inputs as I
    threads = cpu_threads()

    def timed(n, hist0):
        t0 = time.perf_counter()
        oracle.run(I.MATERIALS, workload.phantom, workload.source, seed=7, hist0=hist0, n_hist=n,
                   n_batches=2, n_threads=threads, want_batches=False)
        return time.perf_counter() - t0

    # probes large enough (about a second on 16 threads) that the threads' start
    # and the first touches of the tables do not inflate the rate
    n1, n2 = 20_000, 200_000
    d1 = timed(n1, 0)
    d2 = timed(n2, n1)
    rate = (n2 - n1) / max(d2 - d1, 1e-3)          # setup time cancels
    n = int(max(n2, min(20_000_000, rate * seconds)))
    h0 = n1 + n2
    dt = timed(n, h0)
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "per_core": n / dt / threads, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{n} histories (ids {h0}..{h0 + n - 1}) of the same CT IMRT job, FP64 CPU "
                      f"transport on {threads} threads ({cpu_model()}; the host shows "
                      f"{os.cpu_count()} CPUs, a GPU's share is 16), {dt:.1f} s including the run set-up"}


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=float), q)) if len(a) else None


def batched_form(G, I, n_jobs, opts=None):
    """Uneven dose jobs (cubes of 48-256 voxels, 1e5-1e7 histories, spectra and
    lines, photons and electrons): all in one batched run against the same jobs
    as sequential single-job runs.  Latency of a job: from the start of the
    whole set to the job's completion."""
    ws = I.batch_jobs(n_jobs)
    log(f"batched form: {n_jobs} jobs generated ({sum(w.n_hist for w in ws):.3g} histories)")
    ctx = G.Context(0, opts=opts, materials=I.MATERIALS)
    hs = [(ctx.phantom(w.phantom), ctx.source(w.source), dict(seed=100 + k, job_id=k, n_hist=w.n_hist))
          for k, w in enumerate(ws)]
    hist = sum(w.n_hist for w in ws)
    ctx.run(hs[0][0], hs[0][1], n_hist=10_000, want_dose=False)   # tables and queues
    log("batched form: inputs on the device, batched run")
    t0 = time.perf_counter()
    res = ctx.run_batch(hs, want_dose=False)
    tb = time.perf_counter() - t0
    log(f"batched form: batched run {tb:.3f} s, now one job at a time")
    lat_b = [r["t_total_s"] for r in res]
    bal = max(abs(r["e_dep"] + r["e_esc"] - r["e_in"]) / r["e_in"] for r in res)
    repairs = sum(r["accounting_repairs"] for r in res)
    log_accounting("batched form", res)
    t0 = time.perf_counter()
    lat_s = []
    for k, (p, s, kw) in enumerate(hs):
        ctx.run(p, s, want_dose=False, **kw)
        lat_s.append(time.perf_counter() - t0)
        if k % 16 == 15:
            log(f"batched form: {k + 1} sequential jobs done")
    ts = time.perf_counter() - t0
    for p, s, _ in hs:
        p.close()
        s.close()
    ctx.close()
    return {"workload": f"{n_jobs} jobs, cubes 48-256 voxels of 0.25 cm, 1e5-1e7 histories each",
            "histories": hist,
            "batched": {"seconds": tb, "histories_per_s": hist / tb,
                        "latency_s": {"p50": pct(lat_b, 50), "p99": pct(lat_b, 99)}},
            "sequential": {"seconds": ts, "histories_per_s": hist / ts,
                           "latency_s": {"p50": pct(lat_s, 50), "p99": pct(lat_s, 99)}},
            "speedup": ts / tb, "energy_balance_max": bal, "accounting_repairs": repairs}


def source_modes(G, I, w, args):
    """The source modes of section 2.3 on the CT plan: the two beamlet samplers
    (search, Metropolis chains) and the energy intervals of the spectrum; a job
    to the target uncertainty with each, and the paper's Fig. 2 error e(N) =
    |p_f - p_f*|_2 of the beamlet frequencies of one beam after N histories."""
    import dataclasses
    ctx = G.Context(0, opts=args.opts, materials=I.MATERIALS)
    ph = ctx.phantom(w.phantom)
    out = {"workload": "CT 256x256x128 IMRT-9 to the target; Fig. 2 metric on beam 0 (40x40 beamlets)"}
    for k, strata, name in ((0, 0, "search"), (1, 0, "metropolis"), (0, 16, "search_16_energy_intervals")):
        src = dataclasses.replace(w.source, beamlet_sampler=k, spectrum_strata=strata)
        s = ctx.source(src)
        r = ctx.run(ph, s, seed=7, n_hist=args.n0, target_unc=args.target,
                    stat_min_density=args.min_density, want_dose=False)
        s.close()
        b0 = w.source.beams[0]
        one = I.Source(w.source.particle, w.source.spectrum, [b0], beamlet_sampler=k, spectrum_strata=strata)
        s1 = ctx.source(one)
        f = np.asarray(b0.intensity, dtype=np.float64).ravel()
        p_star = f / f.sum()
        errs = {}
        for n in (100_000, 1_000_000, 4_000_000):
            bl = ctx.sample_source(ph, s1, seed=11, n=n)[:, 1]
            bl = bl[bl >= 0].astype(np.int64)
            errs[str(n)] = float(np.linalg.norm(np.bincount(bl, minlength=len(f)) / max(len(bl), 1) - p_star))
        s1.close()
        out[name] = {"histories_per_s": r["histories"] / r["t_total_s"], "seconds": r["t_total_s"],
                     "histories": r["histories"], "unc": r["unc"], "fig2_error": errs}
        log(f"source modes: {name}: {r['histories'] / r['t_total_s']:.4g} hist/s, e(N) {errs}")
    # the open source interface: a phase space of 1e6 primaries recorded from the
    # plan's beams at their entry points, cycled through by the job's histories
    s0 = ctx.source(w.source)
    prim = ctx.sample_source(ph, s0, seed=13, n=1_000_000)
    s0.close()
    prim = prim[prim[:, 1] >= 0]
    rec = np.concatenate([prim[:, 2:5], prim[:, 5:8], prim[:, :1]], axis=1).astype(np.float32)
    rec[:, 3:6] /= np.linalg.norm(rec[:, 3:6].astype(np.float64), axis=1)[:, None].astype(np.float32)
    s1 = ctx.source(I.Source(w.source.particle, w.source.spectrum, [], phase_space=rec))
    r = ctx.run(ph, s1, seed=7, n_hist=args.n0, target_unc=args.target, stat_min_density=args.min_density,
                want_dose=False)
    s1.close()
    out["phase_space_1e6_records"] = {"histories_per_s": r["histories"] / r["t_total_s"], "seconds": r["t_total_s"],
                                      "histories": r["histories"], "unc": r["unc"]}
    log(f"source modes: phase space: {r['histories'] / r['t_total_s']:.4g} hist/s")
    ph.close()
    ctx.close()
    return out


def variance_reduction(G, I, w, args):
    """Primary splitting (2^k copies of weight 2^-k per history) on the CT job
    to the target uncertainty: time, histories and uncertainty for each k; the
    efficiency gain of k is the unsplit job's time over the split job's."""
    ctx = G.Context(0, opts=args.opts, materials=I.MATERIALS)
    ph, src = ctx.phantom(w.phantom), ctx.source(w.source)
    out = {"workload": "CT 256x256x128 IMRT-9 to the target, cold jobs from the same first estimate"}
    base = None
    for k in (0, 1, 2):
        r = ctx.run(ph, src, seed=17, n_hist=args.n0, target_unc=args.target,
                    stat_min_density=args.min_density, want_dose=False, split_log2=k)
        base = base or r["t_total_s"]
        out[f"split_{1 << k}"] = {"seconds": r["t_total_s"], "histories": r["histories"], "unc": r["unc"],
                                  "histories_per_s": r["histories"] / r["t_total_s"],
                                  "efficiency_gain": base / r["t_total_s"]}
        log(f"splitting {1 << k}: {r['histories']} histories in {r['t_total_s']:.3f} s, unc {r['unc']:.5f}")
    ph.close()
    src.close()
    ctx.close()
    return out


def log_accounting(what, res):
    """Report jobs whose particle accounting needed a repair, failed a check or met an anomaly
    (their signed energy balance and births - deaths gap)."""
    for k, r in enumerate(res):
        if r["accounting_repairs"] or r.get("accounting_mismatches") or r.get("transport_anomalies"):
            log(f"{what}: job {k}: accounting repairs {r['accounting_repairs']}, gap {r['accounting_gap']}, "
                f"checks failed {r.get('accounting_mismatches', 0)}, anomalies {r.get('transport_anomalies', 0)}, "
                f"balance {(r['e_dep'] + r['e_esc'] - r['e_in']) / r['e_in']:+.3e}, "
                f"histories {r['histories']}, passes {r['passes']}")


def run_stream(G, ctx, hs, times, slots, budget, label):
    """Submit the requests at their arrival times to a server with at most
    `slots` jobs running together; returns per-request latency (submission to
    completion), histories and the span from the first arrival to the last
    completion.  A long stream logs its progress about every 30 s."""
    srv = G.Server(ctx, hbm_budget_bytes=budget, max_slots=slots)
    jobs = []
    t0 = time.perf_counter()
    last = t0
    for t, (p, s, kw) in zip(times, hs):
        d = t - (time.perf_counter() - t0)
        if d > 0:
            time.sleep(d)
        jobs.append(srv.submit(p, s, want_dose=False, **{k: v for k, v in kw.items() if k != "kind"}))
        if time.perf_counter() - last > 30:
            last = time.perf_counter()
            log(f"{label}: {len(jobs)} of {len(hs)} requests submitted at {last - t0:.0f} s")
    res = []
    for k, j in enumerate(jobs):
        res.append(j.wait())
        if time.perf_counter() - last > 30:
            last = time.perf_counter()
            log(f"{label}: {k + 1} of {len(jobs)} requests done at {last - t0:.0f} s")
    wall = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    lat = [r["t_total_s"] for r in res]
    hist = sum(r["histories"] for r in res)
    log_accounting(label, res)
    kinds = [kw.get("kind", "") for _, _, kw in hs]
    log(f"{label}: p50 {pct(lat, 50):.2f} s, p99 {pct(lat, 99):.2f} s, span {wall - times[0]:.2f} s")
    # the engine's totals when the last job finished: device time of the
    # transport kernels (HIP events) and launches, over the whole stream
    engine = {k: max(r[k] for r in res) for k in ("t_kernel_s", "t_photon_s", "t_electron_s", "passes",
                                                   "graph_launches", "graphs_recorded", "passes_rebinned")}
    return {"seconds": wall, "histories_per_s": hist / max(wall - times[0], 1e-9), "engine_totals": engine,
            "latency_s": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": float(np.mean(lat)),
                          "max": float(np.max(lat))},
            "memory_high_water_bytes": info["high_water_bytes"] + info["resident_bytes"],
            "energy_balance_max": max(abs(r["e_dep"] + r["e_esc"] - r["e_in"]) / r["e_in"] for r in res),
            "accounting_repairs": sum(r["accounting_repairs"] for r in res),
            "latency_by_kind_s": {k: {"p50": pct([l for l, kk in zip(lat, kinds) if kk == k], 50),
                                      "p99": pct([l for l, kk in zip(lat, kinds) if kk == k], 99)}
                                  for k in sorted(set(kinds))},
            "latencies_s": [round(x, 4) for x in lat]}


def fifo_latencies(times, service):
    """Latencies of the requests run one at a time in arrival order, from their
    arrival times and measured alone run times (a single-server queue)."""
    done, lat = 0.0, []
    for t, s in zip(times, service):
        done = max(done, t) + s
        lat.append(done - t)
    return lat, done


# serving policies: context options and job slots
SERVE_POLICIES = {
    "per_job_launches": (None, 1),
    "shared_even": (None, 64),
    "shared_least_work_first": ('{"issue_order": 1}', 64),
    "shared_admission_order": ('{"issue_order": 2}', 64),
    "admit_while_draining": ('{"issue_order": 2, "admit_draining": 1}', 64),
    "admit_at_final_drain": ('{"issue_order": 2, "admit_draining": 2}', 64),
}


# the bench line's default set (least work first lost to even shares on p99 in
# every measurement: it starves the long VMAT jobs)
SERVE_DEFAULT = ("per_job_launches", "shared_even", "shared_admission_order", "admit_at_final_drain")


def served_form(G, I, seconds, rate, ct, opts=None, load=0.7, policies=None, service_sample=0, stated=True):
    """Poisson request stream (VMAT arcs on the 256x256x128 CT and IMRT jobs on a
    128x128x64 CT, to 1% or 2%) into a server that admits by device footprint
    and batches the admitted jobs.  The requests' run times alone give the
    service demand and the capacity (jobs/s) of one GPU for this mix (all of
    them, or the first `service_sample`); the stream is served at the stated
    rate and (load > 0), stretched in time, at `load` of the capacity (a stable
    queue), by the policies of SERVE_POLICIES: one job at a time in arrival
    order (per-job launches); up to 64 jobs sharing the device evenly, least
    remaining work first, or earliest admitted first; and admission only while
    the running jobs drain (a new job fills the device a running job leaves at
    the end of its super-round), earliest admitted first."""
    policies = policies or list(SERVE_DEFAULT)
    reqs = I.serving_requests(duration_s=seconds, rate=rate, ct=ct)
    times = [t for t, _ in reqs]
    budget = 64 << 30
    out = {"workload": f"Poisson {rate} jobs/s for {seconds} s: {len(reqs)} requests, VMAT-180 on "
                       "256x256x128 CT or IMRT-9 on 128x128x64 CT, to 1% or 2%",
           "requests": len(reqs), "hbm_budget_bytes": budget, "policies": policies}
    def merged(name):
        # the policy's options, with --opts on top
        d = json.loads(SERVE_POLICIES[name][0] or "{}")
        d.update(json.loads(opts or "{}"))
        return json.dumps(d, sort_keys=True)

    ctxs = {}
    for name in policies:
        o = merged(name)
        if o not in ctxs:
            ctxs[o] = G.Context(0, opts=o, materials=I.MATERIALS)
    hs = {o: [] for o in ctxs}
    for o, ctx in ctxs.items():
        phs = {}
        for k, (t, w) in enumerate(reqs):
            key = id(w.phantom)
            if key not in phs:
                phs[key] = ctx.phantom(w.phantom)
            hs[o].append((phs[key], ctx.source(w.source),
                          dict(seed=500 + k, job_id=k, n_hist=w.n_hist, target_unc=w.target_unc,
                               stat_min_density=0.1, kind=w.name)))
        ctx.run(hs[o][0][0], hs[o][0][1], n_hist=10_000, want_dose=False)   # tables and queues
    log(f"served form: {len(reqs)} requests prepared")
    # service demand: the requests alone, back to back
    o0 = next(iter(ctxs))
    ctx = ctxs[o0]
    n_alone = len(reqs) if service_sample <= 0 else min(service_sample, len(reqs))
    service, hist = [], 0
    for k, (p, s, kw) in enumerate(hs[o0][:n_alone]):
        a = time.perf_counter()
        r = ctx.run(p, s, want_dose=False, **{k: v for k, v in kw.items() if k != "kind"})
        service.append(time.perf_counter() - a)
        hist += r["histories"]
        log_accounting(f"served form, request {k} alone", [r])
    mean_s = float(np.mean(service))
    kinds = [w.name for _, w in reqs]
    out["service_s"] = {"requests_measured": n_alone, "mean": mean_s, "p50": pct(service, 50),
                        "max": float(np.max(service)), "total": float(np.sum(service)),
                        "each": [round(x, 4) for x in service], "kinds": kinds[:n_alone],
                        "mean_by_kind": {k: float(np.mean([x for x, kk in zip(service, kinds) if kk == k]))
                                         for k in sorted(set(kinds[:n_alone]))}}
    out["capacity_jobs_per_s"] = 1.0 / mean_s
    out["utilisation_at_stated_rate"] = rate * mean_s
    log(f"served form: mean service {mean_s:.3f} s over {n_alone} requests, capacity {1 / mean_s:.2f} "
        f"jobs/s, load {rate * mean_s:.2f} at {rate} jobs/s")
    streams = [("stated_rate", rate, times)] if stated else []
    if load > 0:
        rate_s = load / mean_s
        streams.append((f"load_{load:g}", rate_s, [t * rate / rate_s for t in times]))
    for sname, r_s, ts in streams:
        res = {"rate_jobs_per_s": r_s, "utilisation": r_s * mean_s, "arrivals_s": [round(t, 3) for t in ts]}
        if n_alone == len(reqs):
            lat, done = fifo_latencies(ts, service)
            res["one_at_a_time_replayed"] = {
                "latency_s": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": float(np.mean(lat)),
                              "max": float(np.max(lat))},
                "histories_per_s": hist / max(done - ts[0], 1e-9)}
        for name in policies:
            o, slots = merged(name), SERVE_POLICIES[name][1]
            res[name] = run_stream(G, ctxs[o], hs[o], ts, slots, budget, f"served {sname}: {name}")
        out[sname] = res
    for o, ctx in ctxs.items():
        done_ph = set()
        for p, s, _ in hs[o]:
            s.close()
            if id(p) not in done_ph:
                done_ph.add(id(p))
                p.close()
        ctx.close()
    return out


def config_rates(G, I, args):
    """Configs 1, 2A and 2B at their stated phantoms and history counts: GPU
    histories/s of a fixed-count job with the inputs resident (the dose left on
    the device), and the oracle's histories/s on a bounded sample of the same
    job (the paper's Table 2 rows, CPU against GPU, on synthetic inputs)."""
    import oracle
    threads = cpu_threads()
    cases = [("config1_water32_2MeV_parallel", I.water_cube_2mev(), 200_000, 200_000),
             ("config2A_slab100_6MVlike_point", I.slab_photon(), 10_000_000, 1_000_000),
             ("config2B_slab100_20MeV_electron_point", I.slab_electron(), 10_000_000, 100_000)]
    ctx = G.Context(0, opts=args.opts, materials=I.MATERIALS)
    out = {}
    for name, w, n, n_cpu in cases:
        p, s = ctx.phantom(w.phantom), ctx.source(w.source)
        ctx.run(p, s, n_hist=min(n, 200_000), seed=2, want_dose=False)
        t0 = time.perf_counter()
        r = ctx.run(p, s, n_hist=n, seed=1, want_dose=False)
        dt = time.perf_counter() - t0
        res = {"histories": n, "gpu_seconds": dt, "gpu_histories_per_s": n / dt,
               "energy_balance": abs(r["e_dep"] + r["e_esc"] - r["e_in"]) / r["e_in"]}
        if not args.no_cpu_baseline:
            t0 = time.perf_counter()
            oracle.run(I.MATERIALS, w.phantom, w.source, seed=7, n_hist=n_cpu, n_batches=10,
                       n_threads=threads, want_batches=False)
            dc = time.perf_counter() - t0
            res.update(oracle_histories=n_cpu, oracle_seconds=dc, oracle_histories_per_s=n_cpu / dc,
                       oracle_threads=threads, gpu_over_oracle=(n / dt) / (n_cpu / dc))
        out[name] = res
        log(f"configs: {name}: GPU {n / dt:.4g} hist/s" +
            (f", oracle {res['oracle_histories_per_s']:.4g} hist/s" if "oracle_seconds" in res else ""))
        p.close()
        s.close()
    ctx.close()
    return out


def profiled_values(path):
    """The machine-readable lines of a committed counter summary, or None when
    there is none or the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    kv = {a.strip(): b.strip() for a, b in (line.split(":", 1) for line in text.splitlines()
                                            if ":" in line and not line.startswith(" "))}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return kv if kv.get("kernel_source_sha256") == h.hexdigest() else None


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE scaled by a
    plain copy), or None."""
    kv = profiled_values(TRAFFIC_SUMMARY)
    v = kv.get(f"{kernel}_hbm_bytes_per_launch") if kv else None
    return float(v) if v else None


def measured_lane_valu_per_event(kernel):
    """Active-lane VALU instructions per flight (k_photon) or step (k_electron)
    from the committed counter summary, or None."""
    kv = profiled_values(COUNTER_SUMMARY)
    v = kv.get(f"{kernel}_lane_valu_per_event") if kv else None
    return float(v) if v else None


def measured_counters(kernel):
    """VALU busy and lane use, occupancy, L2 hit rate and atomics per second of
    `kernel` from the committed counter summary, or None."""
    kv = profiled_values(COUNTER_SUMMARY)
    if not kv:
        return None
    keys = ("valu_busy_pct", "valu_lane_use_pct", "occupancy_waves_per_cu", "l2_hit_pct", "atomics_per_s")
    if not all(f"{kernel}_{k}" in kv for k in keys):
        return None
    return {k: float(kv[f"{kernel}_{k}"]) for k in keys}


def reference_copy(nbytes):
    """One plain device-to-device copy of `nbytes` through the HIP runtime (its
    blit kernel): a kernel of known traffic that calibrates the hardware
    counters read by a profiler run of this same command."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    n = ctypes.c_size_t(nbytes)
    for ptr in (a, b):
        if hip.hipMalloc(ctypes.byref(ptr), n) != 0:
            raise RuntimeError("hipMalloc failed")
    try:
        if hip.hipMemset(a, 1, n) != 0 or hip.hipMemcpy(b, a, n, 3) != 0 or hip.hipDeviceSynchronize() != 0:
            raise RuntimeError("reference copy failed")
    finally:
        hip.hipFree(a)
        hip.hipFree(b)


def event_cost_workloads(I):
    """Jobs of varied event mixes for the event-cost fit: the CT plan at two
    sizes, configs 1, 2A and 2B, and homogeneous phantoms where one kind of
    event dominates (pair production, photoelectric absorption, electrons of
    several energies in water, bone and lung, fine and coarse voxels)."""
    def homo(mat, rho, n=(40, 40, 40), d=(0.5, 0.5, 0.5)):
        return I.homogeneous(n, d, mat, rho)

    def beam(ph, particle, e, field=4.0):
        return I.Source(particle, I.mono(e), [I.parallel_beam_z(ph, field)])

    ct = I.ct_imrt()
    small_ct = I.ct_phantom((64, 64, 32), (0.8, 0.8, 1.0))
    out = [("ct_imrt", ct.phantom, ct.source, 1_000_000),
           ("ct_imrt", ct.phantom, ct.source, 2_000_000)]
    for name, w, n in (("config1_water32_2MeV", I.water_cube_2mev(), 500_000),
                       ("config2A_slab_photon", I.slab_photon(), 500_000),
                       ("config2B_slab_electron", I.slab_electron(), 50_000)):
        out.append((name, w.phantom, w.source, n))
    bone, water, lung = homo(I.ID_BONE, 1.85), homo(I.ID_WATER, 1.0), homo(I.ID_LUNG, 0.26)
    fine = homo(I.ID_WATER, 1.0, (80, 80, 80), (0.1, 0.1, 0.1))
    coarse = homo(I.ID_WATER, 1.0, (20, 20, 40), (1.0, 1.0, 1.0))
    out += [("bone_20MeV_photons", bone, beam(bone, I.PHOTON, 20.0), 200_000),
            ("bone_80keV_photons", bone, beam(bone, I.PHOTON, 0.08), 500_000),
            ("water_300keV_photons", water, beam(water, I.PHOTON, 0.3), 500_000),
            ("small_ct_1.25MeV_photons", small_ct, beam(small_ct, I.PHOTON, 1.25, 10.0), 500_000),
            ("water_1MeV_electrons", water, beam(water, I.ELECTRON, 1.0), 200_000),
            ("bone_5MeV_electrons", bone, beam(bone, I.ELECTRON, 5.0), 100_000),
            ("lung_6MeV_electrons", lung, beam(lung, I.ELECTRON, 6.0), 100_000),
            ("water_fine_0.5MeV_electrons", fine, beam(fine, I.ELECTRON, 0.5, 1.0), 200_000),
            ("water_coarse_10MeV_electrons", coarse, beam(coarse, I.ELECTRON, 10.0), 100_000)]
    return out


def event_cost_runs(G, I):
    """The event-cost jobs in the one-particle-per-wavefront form (every
    wavefront executes exactly the instructions of its particle's path, so a
    VALU instruction counter reads the straight-line cost of the events); run
    this under a per-dispatch counter (SQ_INSTS_VALU, SQ_WAVES) and fit with
    --event-cost-fit.  Every run of the process is listed, in order, with the
    counts the fit needs."""
    ctx = G.Context(0, opts='{"solo_lanes": 1, "graphs": 0}', materials=I.MATERIALS)
    runs = []
    for k, (name, ph, src, n) in enumerate(event_cost_workloads(I)):
        p, s = ctx.phantom(ph), ctx.source(src)
        r = ctx.run(p, s, n_hist=n, seed=700 + k, want_dose=False)
        p.close()
        s.close()
        keep = ("histories", "passes_photon", "passes_electron", "events", "interactions", "records_loaded",
                "records_stored", "records_requeued", "deposits", "t_photon_s", "t_electron_s")
        runs.append(dict({k2: r[k2] for k2 in keep}, name=name))
        log(f"event cost: {name}, {n} histories, {r['passes_photon']} + {r['passes_electron']} launches")
    ctx.close()
    return runs


def event_regressors(run, kernel):
    """The counts of EVENT_TERMS[kernel] (all but 'waves') in one run."""
    k = 0 if kernel == "k_photon" else 1
    vals = dict(run["events"])
    vals.update(run["interactions"])
    # the kernel's own records and deposits (the events' deposits are both kernels')
    vals.update(records_loaded=run["records_loaded"][k], records_stored=run["records_stored"][k],
                deposits=run["deposits"][k])
    return [float(vals[t]) for t in EVENT_TERMS[kernel][1:]]


def event_cost_fit(csv_path, runs_path):
    """Instructions per history and per event of the transport kernels, from a
    rocprofv3 counter CSV (SQ_INSTS_VALU, SQ_WAVES per dispatch) of an
    --event-cost run and that run's output line.  Each wavefront carried one
    particle at a time, so its instructions are exactly those of its
    particles' paths plus the launch's fixed work.  (1) The CT plan run at two
    sizes with the same launches: the difference of the instructions over the
    difference of the histories is the straight-line cost of a history, free
    of the fixed work.  (2) A non-negative least-squares fit over all runs of
    each kernel's instructions on its wavefronts and event counts: the
    coefficient of an event type is what its path costs.  Prints the summary."""
    from scipy.optimize import nnls
    disp = read_dispatch_counters(csv_path)
    runs = bench_line(runs_path)["event_cost_runs"]
    lines, machine = [], [f"kernel_source_sha256: {kernel_source_hash()}"]
    per_kernel = {}
    for kernel, passes in (("k_photon", "passes_photon"), ("k_electron", "passes_electron")):
        ds = [disp[i] for i in sorted(disp) if kernel + "<" in disp[i]["name"]]
        assert all("true, true" in d["name"] for d in ds), "not the one-particle-per-wavefront form"
        assert len(ds) == sum(r[passes] for r in runs), (kernel, len(ds), sum(r[passes] for r in runs))
        X, y, i = [], [], 0
        for r in runs:
            part = ds[i:i + r[passes]]
            i += r[passes]
            X.append([sum(d["SQ_WAVES"] for d in part)] + event_regressors(r, kernel))
            y.append(sum(d["SQ_INSTS_VALU"] for d in part))
        per_kernel[kernel] = (np.array(X), np.array(y), passes)
    ct = [k for k, r in enumerate(runs) if r["name"] == "ct_imrt"]
    a, b = ct[0], ct[-1]
    dn = runs[b]["histories"] - runs[a]["histories"]
    lines += ["Straight-line instructions per history of the CT plan (runs of "
              f"{runs[a]['histories']} and {runs[b]['histories']} histories with the same launches):", "",
              " | kernel | launches | VALU instructions (small, large run) | per history |", " |---|---:|---:|---:|"]
    total = 0.0
    for kernel, (X, y, passes) in per_kernel.items():
        assert runs[a][passes] == runs[b][passes], "the two CT runs must have the same launches"
        v = (y[b] - y[a]) / dn
        total += v
        lines.append(f" | {kernel} | {runs[a][passes]} | {y[a]:.4g}, {y[b]:.4g} | {v:.1f} |")
        machine.append(f"{kernel}_valu_per_history: {v:.2f}")
    lines += [f" | both | | | {total:.1f} |", ""]
    for kernel, (X, y, passes) in per_kernel.items():
        # non-negative least squares (an instruction count is not negative),
        # on columns scaled to unit norm
        norm = np.linalg.norm(X, axis=0)
        keep = norm > 0
        c = np.zeros(X.shape[1])
        c[keep] = nnls(X[:, keep] / norm[keep], y)[0] / norm[keep]
        fit = X @ c
        big = y >= 0.05 * y.max()
        lines.append(f"{kernel}: VALU instructions = sum of coefficient x count over {len(runs)} runs; "
                     f"|residual| summed {np.abs(y - fit).sum() / y.sum() * 100:.1f}% of all instructions, "
                     f"at most {np.abs((y - fit) / y)[big].max() * 100:.1f}% of a run's (runs with at least 5% "
                     "of the largest run's instructions)")
        lines += [" | term | instructions each |", " |---|---:|"]
        for t, v in zip(EVENT_TERMS[kernel], c):
            lines.append(f" | {t} | {v:.1f} |")
            machine.append(f"{kernel}_cost_{t}: {v:.3f}")
        lines += ["", " | run | histories | launches | VALU instructions | fit |", " |---|---:|---:|---:|---:|"]
        for r, yy, ff in zip(runs, y, fit):
            lines.append(f" | {r['name']} | {r['histories']} | {r[passes]} | {yy:.4g} | {ff:.4g} |")
        lines.append("")
    print("\n".join(lines + ["Machine-readable values used by bench.py (valid while the kernel source hash "
                              "matches):", ""] + machine))


def measured_event_costs(kernel):
    """(straight-line instructions per CT history, {term: instructions per
    event}) of `kernel` from the committed event-cost summary, or None."""
    kv = profiled_values(EVENT_COST_SUMMARY)
    if not kv or f"{kernel}_valu_per_history" not in kv:
        return None
    return (float(kv[f"{kernel}_valu_per_history"]),
            {t: float(kv[f"{kernel}_cost_{t}"]) for t in EVENT_TERMS[kernel] if f"{kernel}_cost_{t}" in kv})


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_kernel(name):
    """'void gdpm::k_photon<true, false>(gdpm::Ctl*, ...)' -> 'k_photon'"""
    base = name.split("(")[0].split("<")[0].split()[-1]
    return base.split("::")[-1]


def read_dispatch_counters(csv_path):
    """rocprofv3 counter CSV -> {dispatch id: {"name": kernel, counter: value}}"""
    import csv
    disp = {}
    with open(csv_path) as fh:
        for row in csv.DictReader(fh):
            d = disp.setdefault(int(row["Dispatch_Id"]), {"name": row["Kernel_Name"]})
            d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    return disp


def bench_line(path):
    return json.loads(open(path).read().strip().splitlines()[-1])


def summarize_trace(stats_csv, bench_json):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run of the CT job."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    b = bench_line(bench_json)
    roof = b["roofline"]
    out = ["| kernel | calls | total ms | average us | share |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| {r['Name'].split('(')[0].replace('void ', '')} | {r['Calls']} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f}% |")
    trace_avg = {short_kernel(r["Name"]): float(r["AverageNs"]) / 1e6 for r in rows}
    k = roof["kernel"]
    out += ["", f"The bench line of the same run (HIP events on the library stream) gives "
                f"{roof['avg_launch_ms']:.3f} ms per {k} launch over {roof['launches']} launches; the "
                f"trace average is {trace_avg.get(k, float('nan')):.3f} ms.",
            f"Job: {b['config']['histories_per_job']} histories, {b['ms_per_step'] / 1e3:.3f} s, "
            f"{b['value']:.4g} histories/s under the profiler.", "",
            f"kernel_source_sha256: {kernel_source_hash()}"]
    print("\n".join(out))


def summarize_counters(bench_json, *csvs):
    """Per-launch averages of the transport and source kernels' counters
    (VALU busy and lane use, occupancy, L2 hit rate, atomics per second) from
    rocprofv3 counter CSVs of the CT job, plus the active-lane instructions per
    event that the executed-instruction roofline figure uses."""
    per = {}
    for c in csvs:
        for d in read_dispatch_counters(c).values():
            k = short_kernel(d["name"])
            if k not in ("k_photon", "k_electron", "k_source"):
                continue
            acc = per.setdefault(k, {})
            for name, v in d.items():
                if name != "name":
                    acc.setdefault(name, []).append(v)
    b = bench_line(bench_json)
    ev = b["events_per_history"]
    hist = b["config"]["histories_per_job"]
    kt = b["kernel_time_s"]
    launches = b["roofline"]["launches"]
    out = ["| kernel | VALU busy % | VALU lane use % | occupancy (waves/CU) | L2 hit % | VALU instr. per launch "
           "| atomics per s |", "|---|---:|---:|---:|---:|---:|---:|"]
    machine = [f"kernel_source_sha256: {kernel_source_hash()}"]
    for k in ("k_photon", "k_electron", "k_source"):
        a = {n: float(np.mean(v)) for n, v in per.get(k, {}).items()}
        if not a:
            continue
        hit = a["TCC_HIT_sum"] / max(a["TCC_HIT_sum"] + a["TCC_MISS_sum"], 1.0) * 100
        t = {"k_photon": kt["photon"], "k_electron": kt["electron"]}.get(k)
        atom = a["TCC_ATOMIC_sum"] * launches / t if t else float("nan")
        out.append(f"| {k} | {a['VALUBusy']:.1f} | {a['VALUUtilization']:.1f} | {a['MeanOccupancyPerCU']:.2f} | "
                   f"{hit:.1f} | {a['SQ_INSTS_VALU']:.4g} | {atom:.4g} |")
        machine += [f"{k}_valu_busy_pct: {a['VALUBusy']:.2f}", f"{k}_valu_lane_use_pct: {a['VALUUtilization']:.2f}",
                    f"{k}_occupancy_waves_per_cu: {a['MeanOccupancyPerCU']:.3f}", f"{k}_l2_hit_pct: {hit:.2f}"]
        if t:
            machine.append(f"{k}_atomics_per_s: {atom:.4e}")
            events = (ev["flights"] if k == "k_photon" else ev["esteps"]) * hist / launches
            lane = a["SQ_INSTS_VALU"] * 64 * a["VALUUtilization"] / 100 / events
            machine.append(f"{k}_lane_valu_per_event: {lane:.1f}")
    print("\n".join(out + ["", "Machine-readable values used by bench.py (valid while the kernel source hash "
                                   "matches):", ""] + machine))


def summarize_traffic(fetch_csv, write_csv, copy_mib):
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what it reads for the plain device copy of copy_mib MiB in
    the same run."""
    f, w = read_dispatch_counters(fetch_csv), read_dispatch_counters(write_csv)
    def per_kernel(disp, counter):
        out = {}
        for d in disp.values():
            out.setdefault(short_kernel(d["name"]) if "gdpm" in d["name"] else d["name"], []).append(d[counter])
        return out
    fk, wk = per_kernel(f, "FETCH_SIZE"), per_kernel(w, "WRITE_SIZE")
    copy = [n for n in fk if "copyBuffer" in n]
    big_f = max(max(fk[n]) for n in copy)
    big_w = max(max(wk[n]) for n in copy if n in wk)
    kib = copy_mib * 1024
    sf, sw = kib / big_f, kib / big_w
    out = [f"Calibration: the {copy_mib} MiB device-to-device copy read {big_f:.0f} KiB by FETCH_SIZE and wrote "
           f"{big_w:.0f} KiB by WRITE_SIZE; scale factors {sf:.4f} (fetch) and {sw:.4f} (write).", "",
           "| kernel | launches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch (scaled) |",
           "|---|---:|---:|---:|---:|"]
    machine = [f"kernel_source_sha256: {kernel_source_hash()}"]
    for k in ("k_photon", "k_electron", "k_source"):
        if k not in fk or k not in wk:
            continue
        mf, mw = float(np.mean(fk[k])), float(np.mean(wk[k]))
        b = (mf * sf + mw * sw) * 1024
        out.append(f"| {k} | {len(fk[k])} | {mf:.0f} | {mw:.0f} | {b:.4g} |")
        machine.append(f"{k}_hbm_bytes_per_launch: {b:.4e}")
    print("\n".join(out + ["", "Machine-readable values used by bench.py (valid while the kernel source hash "
                                   "matches):", ""] + machine))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--target", type=float, default=0.01)
    ap.add_argument("--n0", type=int, default=100_000_000, help="first history estimate per job")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--opts", default=None, help="context options (JSON)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB before the "
                         "timed jobs (a reference kernel of known traffic for hardware counters)")
    ap.add_argument("--batched-jobs", type=int, default=64,
                    help="jobs of the batched-form comparison (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the served request stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2.0, help="requests per second")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="utilisation of the stable stream (the stated stream stretched in time)")
    ap.add_argument("--variance-reduction", type=int, default=1,
                    help="1: also run the CT job with primary splitting (2 and 4 copies)")
    ap.add_argument("--configs", type=int, default=1,
                    help="1: also time configs 1, 2A and 2B on the GPU and the oracle")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the served form (a long stream's record), no CT jobs")
    ap.add_argument("--serve-policies", default=None,
                    help="comma-separated serving policies out of " + ",".join(SERVE_POLICIES) +
                         " (default: " + ",".join(SERVE_DEFAULT) + ")")
    ap.add_argument("--serve-service-sample", type=int, default=0,
                    help="measure the service demand on the first N requests only (0: all)")
    ap.add_argument("--serve-stated", type=int, default=1,
                    help="1: serve the stream at the stated rate (0: only the stream at --serve-load)")
    ap.add_argument("--source-modes", type=int, default=1,
                    help="1: also run the CT job with the other source modes (section 2.3)")
    ap.add_argument("--min-density", type=float, default=0.1,
                    help="voxels below this density (the air around the patient) are left out "
                         "of D_max and of the uncertainty statistic")
    ap.add_argument("--event-cost", action="store_true",
                    help="only the event-cost jobs in the one-particle-per-wavefront form (to run "
                         "under a VALU instruction counter)")
    ap.add_argument("--event-cost-fit", nargs=2, metavar=("COUNTER_CSV", "RUNS_JSON"),
                    help="fit the instructions per event from a counter CSV of an --event-cost run "
                         "and that run's output line (no GPU needed)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="print a profile summary (no GPU needed): 'trace STATS_CSV BENCH_JSON', "
                         "'counters BENCH_JSON CSV...', 'traffic FETCH_CSV WRITE_CSV COPY_MIB'")
    args = ap.parse_args()
    if args.summarize:
        kind, rest = args.summarize[0], args.summarize[1:]
        if kind == "trace":
            summarize_trace(*rest)
        elif kind == "counters":
            summarize_counters(*rest)
        elif kind == "traffic":
            summarize_traffic(rest[0], rest[1], int(rest[2]))
        else:
            ap.error(f"unknown summary {kind}")
        return
    if args.event_cost_fit:
        event_cost_fit(*args.event_cost_fit)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (histories would be "
              "sharded across GPUs by history id, with one FP64 all-reduce of the batch tallies "
              "at the end of a job). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    from paper_1107_3355_amd import gdpm as G
    from paper_1107_3355_amd import inputs as I

    if args.event_cost:
        print(json.dumps({"event_cost_runs": event_cost_runs(G, I)}), flush=True)
        return
    log("building the synthetic CT workload")
    w = I.ct_imrt(target_unc=args.target)
    if args.serve_only:
        log(f"served form only: {args.serve_seconds} s of requests at {args.serve_rate}/s")
        pols = args.serve_policies.split(",") if args.serve_policies else None
        res = served_form(G, I, args.serve_seconds, args.serve_rate, w.phantom, args.opts, args.serve_load,
                          pols, args.serve_service_sample, bool(args.serve_stated))
        print(json.dumps({"served_form": res}), flush=True)
        return
    ctx = G.Context(0, opts=args.opts, materials=I.MATERIALS)
    ph = ctx.phantom(w.phantom)
    src = ctx.source(w.source)

    def job(seed):
        # gdpm_run is blocking: it returns after the device work of the job is complete
        return ctx.run(ph, src, seed=seed, n_hist=args.n0, target_unc=args.target,
                       stat_min_density=args.min_density, want_dose=False)

    if args.copy_mib:
        reference_copy(args.copy_mib << 20)
        log(f"reference copy: {args.copy_mib} MiB read, {args.copy_mib} MiB written")

    for i in range(args.warmup):
        r = job(1000 + i)
        log(f"warmup {i}: {r['histories']} histories, unc {r['unc']:.5f}, {r['t_total_s']:.2f} s")
    # every timed job starts cold, from the same first estimate of its histories
    # (n0), as a new plan would: a first super-round of n0 histories, then the
    # histories the 1/sqrt(N) law asks for
    runs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = job(1 + i)
        runs.append(r)
        log(f"step {i}: {r['histories']} histories, unc {r['unc']:.5f}, {r['t_total_s']:.3f} s, "
            f"{r['histories'] / r['t_total_s']:.4g} hist/s")
    wall = time.perf_counter() - t0
    hist = sum(r["histories"] for r in runs)
    lat = np.array([r["t_total_s"] for r in runs])
    rates = [r["histories"] / r["t_total_s"] for r in runs]

    # roofline of the dominant transport kernel: algorithmic bytes per launch
    # over the launch's average HIP-event duration
    te = sum(r["t_electron_s"] for r in runs)
    tp = sum(r["t_photon_s"] for r in runs)
    ne = sum(r["passes_electron"] for r in runs)
    npp = sum(r["passes_photon"] for r in runs)
    ev = {k: sum(r["events"][k] for r in runs) for k in runs[0]["events"]}
    k = 1 if te >= tp else 0
    name, launches, t_k = ("k_electron", ne, te) if k else ("k_photon", npp, tp)
    lookups = ev["esteps"] if k else ev["flights"]
    nbytes = (BYTES_PER_VOXEL_LOOKUP * lookups
              + BYTES_PER_RECORD * sum(r["records_loaded"][k] + r["records_stored"][k] for r in runs)
              + BYTES_PER_DEPOSIT * sum(r["deposits"][k] for r in runs))
    avg = t_k / max(launches, 1)
    achieved = nbytes / max(launches, 1) / avg / 1e9
    hbm = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": achieved / PEAK_HBM_GBS, "algorithmic_bytes_per_launch": nbytes / max(launches, 1)}
    roof = dict(hbm, kernel=name, traffic=measured_traffic(name), counters=measured_counters(name),
                avg_launch_ms=avg * 1e3, launches=launches, share_of_kernel_time=t_k / max(te + tp, 1e-30))
    # The transport kernels are bound by vector-ALU issue (divergent scalar
    # FP32 work), not by HBM: priced as the active-lane VALU instructions one
    # transport event costs (from the committed counter profile of this kernel
    # source) times the launch's events, against the chip's lane-instruction rate.
    # Algorithmic: the straight-line VALU instructions of the launch's
    # histories (measured with one particle per wavefront, where every
    # instruction serves one particle's path; the launch's fixed work left
    # out), i.e. SURVEY-style W_h = sum over event types of count x cost.
    # Executed: the active-lane instructions the launch really issued per event
    # (queue work, job switches and whatever lanes ran beside the path).
    per_event = measured_lane_valu_per_event(name)
    costs = measured_event_costs(name)
    if costs or per_event:
        roof.update(bound="alu", peak=PEAK_VALU_TLANE, unit="T lane-instructions/s", hbm=hbm)
        roof.pop("algorithmic_bytes_per_launch")
    if per_event:
        executed = per_event * lookups / max(launches, 1) / avg / 1e12
        roof["executed"] = {"achieved": executed, "frac": executed / PEAK_VALU_TLANE,
                            "lane_valu_per_event": per_event}
        roof.update(achieved=executed, frac=executed / PEAK_VALU_TLANE)
    if costs:
        per_history, per_event_type = costs
        work = per_history * hist
        alg = work / max(launches, 1) / avg / 1e12
        roof.update(achieved=alg, frac=alg / PEAK_VALU_TLANE,
                    algorithmic_lane_instructions_per_launch=work / max(launches, 1),
                    straight_line_instructions_per_history=per_history,
                    instructions_per_event=per_event_type)
    # the kernel's FP64 tally additions per second against the measured rate of
    # scattered FP64 atomics into an array of one CT tally slot (and a small one)
    peak = ctx.atomic_rate(8 * w.phantom.nvox)
    deposits = sum(r["deposits"][k] for r in runs)
    roof["atomics"] = {"tally_atomics_per_s": deposits / max(t_k, 1e-30), "measured_peak_per_s": peak,
                       "frac": deposits / max(t_k, 1e-30) / peak,
                       "measured_peak_per_s_256KiB": ctx.atomic_rate(256 << 10),
                       "probe": f"random FP64 atomicAdd into {8 * w.phantom.nvox} B (one tally slot)"}

    out = {
        "metric": METRIC,
        "value": hist / wall,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name + "_to_1pct", "phantom_voxels": [256, 256, 128],
                   "voxel_cm": [0.2, 0.2, 0.25], "beams": 9, "beamlets": 9 * 1600,
                   "spectrum": "triangular 0.25-1.2-6 MeV", "target_unc": args.target,
                   "n_batches": 10, "histories_per_job": int(np.mean([r["histories"] for r in runs])),
                   "first_estimate": args.n0, "rounds_per_job": float(np.mean([r["rounds"] for r in runs])),
                   "stat_min_density": args.min_density,
                   "tally": "f64"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        # each timed job's own rate: the spread of the repeats
        "histories_per_s_per_job": {"min": float(min(rates)), "median": float(np.median(rates)),
                                    "max": float(max(rates))},
        "unc_reached": [r["unc"] for r in runs],
        "energy_balance_max": max(abs(r["e_dep"] + r["e_esc"] - r["e_in"]) / r["e_in"] for r in runs),
        "accounting_repairs": sum(r["accounting_repairs"] for r in runs),
        "transport_anomalies": sum(r["transport_anomalies"] for r in runs),
        "events_per_history": {k: v / hist for k, v in ev.items() if k != "histories"},
        "kernel_time_s": {"photon": tp, "electron": te},
        "roofline": roof,
    }
    if args.batched_jobs > 0:
        log(f"batched form: {args.batched_jobs} jobs")
        out["batched_form"] = batched_form(G, I, args.batched_jobs, args.opts)
        log(f"batched form: speed-up {out['batched_form']['speedup']:.2f}x over sequential runs")
    if args.source_modes:
        log("source modes: search and Metropolis beamlet sampling")
        out["source_modes"] = source_modes(G, I, w, args)
    if args.variance_reduction:
        log("variance reduction: primary splitting")
        out["variance_reduction"] = variance_reduction(G, I, w, args)
    if args.serve_seconds > 0:
        log(f"served form: {args.serve_seconds} s of requests at {args.serve_rate}/s")
        pols = args.serve_policies.split(",") if args.serve_policies else None
        out["served_form"] = served_form(G, I, args.serve_seconds, args.serve_rate, w.phantom, args.opts,
                                         args.serve_load, pols, args.serve_service_sample,
                                         bool(args.serve_stated))
    if args.configs:
        log("configs 1, 2A, 2B")
        out["configs"] = config_rates(G, I, args)
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    ph.close()
    src.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

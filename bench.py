"""Benchmark of the vacancy-jump AKMC hot path on one MI355X.

Workload: BCC 128^3 cells (4,194,304 sites), Fe-1.34Cu-0.70Ni-1.40Mn random
solid solution, 200 vacancies, binary32 energies/barriers/rates with
binary64 rate sums and time (seeded synthetic inputs, resident in HBM
before the timed region).

One step = one pass of the whole hot path: `--events` residence-time
events of the persistent event loop (rates, selection, time, swap, local
refresh) followed by one bulk rate evaluation of every site (8 jump rates
per site).  `value` is KMC events per second over the timed steps;
`rate_evals_per_s` is the bulk sweep's jump-rate evaluations per second.

The JSON line also carries:
  roofline      the bulk sweep kernel (k_rates_all) against HBM: algorithmic
                bytes per launch (1 B occupancy read + 8 rates written per
                site) over its mean kernel time from HIP events that each
                launch records at its kernel's start and end on its stream
                (akmc_rates_timing); traffic from the committed rocprofv3 counter
                summary when it still matches the kernel source;
  event_loop    per-event latency of the loop kernel;
  cpu_baseline  the CPU oracle (full rate recompute per event, binary64,
                one core) on a bounded sample of the same workload;
  cpu_baseline_local  the oracle's local-refresh mode (classical CPU AKMC
                locality, same trajectory) on a longer sample;
  forms         binary64 path, the batched replica ensemble (256 replicas
                of 16^3..48^3 cells) and the learned-barrier form, each timed
                separately outside the main timed region.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "KMC events/s + jump-rate evals/s at 4.2M sites; plain vs batched/surrogate"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_rates_all_rpv_4m_traffic.json")


def kernel_source_hash():
    """Hash of the sweep's sources without comments and layout, so that the
    stored traffic counters stay valid across edits that leave the code
    unchanged."""
    h = hashlib.sha256()
    for f in ("akmc_rates.hip", "akmc_device.hpp", "akmc_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2604_24091_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(bytes_per_launch_alg, precision_tag):
    """HBM bytes per launch from the committed counter summary, or None if
    it is missing or was taken on a different kernel source."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    r = rec.get(precision_tag)
    if not r:
        return None
    return r.get("hbm_bytes_per_launch")


def _counter_rows(run_dir, counter):
    """(kernel name, dispatch id, value) of `counter` from a rocprofv3 CSV run."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                low = {k.lower(): v for k, v in r.items()}
                if low.get("counter_name") != counter:
                    continue
                rows.append((low["kernel_name"], low.get("dispatch_id", ""), float(low["counter_value"])))
    return rows


def write_traffic(fetch_dir, write_dir, tag):
    """HBM bytes per sweep launch from two rocprofv3 --pmc runs of
    `bench.py --copy-calibration` (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch).  Each counter is scaled by the factor that makes it read
    256 MiB on the calibration pass (an elementwise add over 256 MiB of
    binary32: 256 MiB read, 256 MiB written)."""
    calib = 256 << 20
    out = {"source_hash": kernel_source_hash()}
    try:
        with open(PROFILE_TRAFFIC) as f:
            out.update({k: v for k, v in json.load(f).items() if k in ("fp32", "fp64")})
    except (OSError, ValueError):
        pass
    rec = {}
    for name, run_dir in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _counter_rows(run_dir, name)
        ew = [v for k, _, v in rows if "elementwise" in k]
        sweep = [v for k, _, v in rows if "k_rates_all" in k]
        if not ew or not sweep:
            raise SystemExit("no calibration or sweep dispatch with %s under %s" % (name, run_dir))
        factor = calib / (max(ew) * 1024.0)
        rec[name] = {"kib_per_dispatch_mean": float(np.mean(sweep)), "dispatches": len(sweep),
                     "calibration_kib": max(ew), "factor": factor,
                     "bytes_per_launch": float(np.mean(sweep)) * 1024.0 * factor}
    rec["hbm_bytes_per_launch"] = rec["FETCH_SIZE"]["bytes_per_launch"] + rec["WRITE_SIZE"]["bytes_per_launch"]
    out[tag] = rec
    out["source_hash"] = kernel_source_hash()
    with open(PROFILE_TRAFFIC, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def host_cpu():
    """Model name of the host CPU (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(spec, n_events, local=False):
    """The oracle on one host thread.  local=False: the plain oracle (full
    recompute of every rate before every event); local=True: its local
    refresh mode, the classical CPU code's locality (same trajectory)."""
    from oracle import akmc_oracle as O
    o = O.Oracle(spec, precision=0)
    t0 = time.perf_counter()
    done = o.run(n_events, local=local)
    dt = time.perf_counter() - t0
    how = ("local refresh (after each jump only the vacancies within 3 half-cells of the two "
           "exchanged sites)" if local else "full rate recompute of all 1,600 candidates per event")
    return {"value": done / dt, "unit": "events/s", "cores": 1,
            "host_cpu": host_cpu(), "host_threads": os.cpu_count(),
            "kind": "oracle-local-refresh" if local else "oracle",
            "sample": "first %d events of the same 4.2M-site lattice, binary64, %s, one thread "
                      "(%.1f s)" % (done, how, dt)}


def cpu_baseline_replicas(n_events):
    """The oracle (full rate recompute per event, binary64) on the 256-replica
    ensemble, one replica per task over every host thread (the C oracle
    releases the interpreter while it runs)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import akmc_oracle as O
    from paper_2604_24091_amd import workloads as W
    reps = W.rpv_replicas()
    oracles = [O.Oracle(r) for r in reps]
    # the machine's CPU share: at most 16 threads per GPU, whatever the host shows
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        done = sum(ex.map(lambda o: o.run(n_events), oracles))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "events/s", "cores": threads, "host_cpu": host_cpu(),
            "kind": "oracle",
            "sample": "first %d events of each of the 256 replicas (16^3..48^3 cells, 1-20 vacancies), "
                      "binary64, full rate recompute per event, one replica per task on %d threads "
                      "(%.1f s)" % (n_events, threads, dt)}


def cpu_rate_baseline(spec, occ, sites, gpu_rates):
    """The oracle's rate evaluation (binary64, one thread) on a sample of the
    sweep's sites, timed; the same oracle rates are the reference of the
    binary32 sweep's per-result error on those sites (state after the timed
    steps)."""
    from oracle import akmc_oracle as O
    from paper_2604_24091_amd import workloads as W
    o = O.Oracle(W.LatticeSpec(**{**spec.__dict__, "occ": occ}))
    t0 = time.perf_counter()
    ro, eo = o.rates_sites(sites)
    dt = time.perf_counter() - t0
    m = ro > 0
    g = gpu_rates.astype(np.float64)
    rel = np.abs(g[m] - ro[m]) / ro[m]
    base = {"value": sites.size * 8 / dt, "unit": "rate evals/s", "cores": 1, "host_cpu": host_cpu(),
            "kind": "oracle",
            "sample": "8 jump rates of %d random sites of the 4.2M-site lattice, binary64, one thread "
                      "(%.2f s)" % (sites.size, dt)}
    err = {"reference": "binary64 oracle", "sites": int(sites.size), "candidates": int(m.sum()),
           "mask_equal": bool(np.array_equal(g > 0, m)),
           "max_rel_rate": float(rel.max()), "median_rel_rate": float(np.median(rel)),
           "p999_rel_rate": float(np.quantile(rel, 0.999))}
    return base, err


def bench_forms(args, torch, akmc, W, stream):
    forms = {}
    # binary64 plain path on the same lattice.
    spec = W.rpv_4m()
    lat = akmc.Lattice(spec, precision=akmc.FP64, stream=stream)
    out = torch.empty((spec.n_sites, 8), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        lat.step(1000)
        akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(args.events)
        e1.record(stream)
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(5):
            akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, out)
        s1.record(stream)
        torch.cuda.synchronize()
    loop_s = e0.elapsed_time(e1) * 1e-3
    sweep_s = s0.elapsed_time(s1) * 1e-3 / 5
    forms["fp64"] = {"events_per_s": args.events / loop_s,
                     "rate_evals_per_s": spec.n_sites * 8 / sweep_s,
                     "sweep_gbs": spec.n_sites * 65 / sweep_s / 1e9}
    lat.close()
    del out
    forms["fp32_vs_fp64"] = bench_fp32_error(torch, akmc, W, stream)

    # The two smaller single-lattice workloads, in full.
    for name, fn, prec, n_ev in (("fe_cu_2k_fp64", W.fe_cu_2k, akmc.FP64, 10_000),
                                 ("rpv_524k_fp32", W.rpv_524k, akmc.FP32, 1_000_000)):
        sp = fn()
        lw = akmc.Lattice(sp, precision=prec, stream=stream)
        with torch.cuda.stream(stream):
            lw.step(min(n_ev, 10_000))           # warm-up launch
            torch.cuda.synchronize()
            a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lw.step(n_ev)
            b2.record(stream)
            torch.cuda.synchronize()
        dt = a.elapsed_time(b2) * 1e-3
        _, _, sm = lw.read()
        lw.close()
        forms[name] = {"events": n_ev, "sites": sp.n_sites, "vacancies": len(sp.vacancy_sites()),
                       "precision": "binary64" if prec == akmc.FP64 else
                                    "binary32 energies/rates, binary64 sums and time",
                       "events_per_s": n_ev / dt, "us_per_event": dt * 1e6 / n_ev,
                       "frozen": int(sm.frozen)}

    # Batched voxel ensemble: 256 independent replicas, one persistent launch.
    reps = W.rpv_replicas()
    params = [akmc.make_params(r, precision=akmc.FP32) for r in reps]
    nv = [int(np.count_nonzero(r.occ == 4)) for r in reps]
    ws = torch.empty(akmc.batch_workspace_bytes(params, nv), dtype=torch.uint8, device="cuda")
    b = akmc.batch_create(params, [r.occ for r in reps], ws, stream)
    chosen = akmc.batch_autotune(b, 200)
    sched = akmc.Schedule(chosen.group_lanes, chosen.waves_per_block, chosen.blocks, 1,
                          args.batch_events)
    akmc.batch_set_schedule(b, sched)
    akmc.batch_step(b, 2000)                        # warm
    torch.cuda.synchronize()
    busy0 = np.array([akmc.batch_state_read(b, r).loop_seconds for r in range(len(reps))])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    akmc.batch_step(b, args.batch_events)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3
    busy = np.array([akmc.batch_state_read(b, r).loop_seconds for r in range(len(reps))]) - busy0
    forms["batched"] = {"events_per_s": len(reps) * args.batch_events / dt,
                        "replicas": len(reps), "events_per_replica": args.batch_events,
                        "wall_s": dt,
                        "replica_seconds": {"max": float(busy.max()), "mean": float(busy.mean()),
                                            "min": float(busy.min()),
                                            "p99": float(np.quantile(busy, 0.99))},
                        "tail_max_over_mean": float(busy.max() / busy.mean()),
                        "slowest_replica_events_per_s": args.batch_events / float(busy.max()),
                        "sites_total": int(sum(r.n_sites for r in reps)),
                        "schedule": {"group_lanes": chosen.group_lanes,
                                     "waves_per_block": chosen.waves_per_block,
                                     "hipgraph": 1, "chunk_events": args.batch_events}}
    akmc.batch_destroy(b)
    del ws
    if args.surrogate_samples > 0:
        forms["surrogate"] = bench_surrogate(args, torch, akmc, W, stream)
    if args.voxel_events > 0:
        forms["voxel_ensemble"] = bench_voxels(args, torch, akmc, W, stream)
    if args.learned_events > 0:
        forms["learned_runtime"] = bench_learned(args, torch, akmc, W, stream)
    if args.far_events > 0:
        forms["pairs_to_6A"] = bench_far(args, torch, akmc, W, stream)
    return forms


def bench_far(args, torch, akmc, W, stream):
    """The costlier energy model: pair energies out to 6.0 A (six shells,
    126 changed bonds per jump instead of 26) on the 4.2M-site lattice,
    binary32 rates: event loop events/s and the rate evaluation of every
    site (the per-candidate kernel)."""
    spec = W.rpv_4m_far()
    lat = akmc.Lattice(spec, precision=akmc.FP32, stream=stream)
    out = torch.empty((spec.n_sites, 8), dtype=torch.float32, device="cuda")
    with torch.cuda.stream(stream):
        lat.step(2000)
        akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, out)
        torch.cuda.synchronize()
        a0, a1, a2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a0.record(stream)
        lat.step(args.far_events)
        a1.record(stream)
        for _ in range(3):
            akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, out)
        a2.record(stream)
        torch.cuda.synchronize()
    loop_s = a0.elapsed_time(a1) * 1e-3
    sweep_s = a1.elapsed_time(a2) * 1e-3 / 3
    lat.close()
    return {"shells": 6, "bonds_per_jump": 126, "events": args.far_events,
            "events_per_s": args.far_events / loop_s, "us_per_event": loop_s * 1e6 / args.far_events,
            "all_sites_rate_evals_per_s": spec.n_sites * 8 / sweep_s,
            "all_sites_ms": sweep_s * 1e3}


def bench_voxels(args, torch, akmc, W, stream):
    """Voxel ensemble of a wall thermal field (Sec. III-C): the Eq. 9 grid,
    one 16^3-cell replica per voxel at the voxel's temperature, every
    replica advanced to one physical-time horizon, with the persistent
    groups pulling replicas heaviest first (Eq. 10 proxy computed on the
    device) against the plain index order.  Fewer persistent groups than
    replicas, so the order decides the tail."""
    T = W.wall_thermal_field(32, 96)
    gx, gz, tv, worst = akmc.voxel_grid(T, 0.6, W.KB_EV_PER_K, args.voxel_tol)
    reps = W.voxel_replicas(tv, gx, gz, cells=16, max_vac=8)
    params = [akmc.make_params(r, precision=akmc.FP32) for r in reps]
    nv = [int(np.count_nonzero(r.occ == r.n_species - 1)) for r in reps]
    res = {"field_samples": [32, 96], "grid": [gx, gz], "voxels": len(reps),
           "eq9_tol": args.voxel_tol, "eq9_worst": worst,
           "t_min_k": float(tv.min()), "t_max_k": float(tv.max()),
           "vacancies": int(sum(nv))}
    blocks = args.voxel_blocks
    for name, order in (("priority", akmc.ORDER_PRIORITY), ("index", akmc.ORDER_INDEX)):
        ws = torch.empty(akmc.batch_workspace_bytes(params, nv), dtype=torch.uint8, device="cuda")
        b = akmc.batch_create(params, [r.occ for r in reps], ws, stream)
        akmc.batch_set_schedule(b, akmc.Schedule(64, 1, blocks, 0, 1 << 30))
        with torch.cuda.stream(stream):
            akmc.batch_priority(b)     # evaluates every replica's candidates (no events)
            torch.cuda.synchronize()
            g = np.array([akmc.batch_state_read(b, r).gamma_tot for r in range(len(reps))])
            t_end = args.voxel_events / float(np.median(g))
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            akmc.batch_run_until(b, t_end, 50 * args.voxel_events, order)
            a1.record(stream)
            torch.cuda.synchronize()
        wall = a0.elapsed_time(a1) * 1e-3
        ev = np.array([akmc.batch_state_read(b, r).n_events for r in range(len(reps))])
        busy = np.array([akmc.batch_state_read(b, r).loop_seconds for r in range(len(reps))])
        akmc.batch_destroy(b)
        del ws
        res[name] = {"wall_s": wall, "events": int(ev.sum()), "events_per_s": float(ev.sum()) / wall,
                     "events_per_replica": {"min": int(ev.min()), "median": float(np.median(ev)),
                                            "max": int(ev.max())},
                     "replica_seconds_max": float(busy.max())}
        res["t_end_s"] = t_end
    res["persistent_groups"] = blocks
    res["priority_speedup_vs_index"] = res["index"]["wall_s"] / res["priority"]["wall_s"]
    return res


def bench_learned(args, torch, akmc, W, stream):
    """AtomWorld's runtime forms on the 4.2M-site lattice: events chosen by a
    local policy network and time advanced by a Poisson network (both of
    hidden width 64 on the 64-neighbour observation, seeded weights), against
    the plain pair-rate loop on the same lattice."""
    spec = W.rpv_4m()
    rng = np.random.default_rng(2024)
    S, H = spec.n_species, 64
    nets = {}
    for name, n_out, bias in (("policy", 8, 0.0), ("poisson", 1, 1.0)):
        nb = akmc.PatchNetBlob(S, H, n_out)
        nb.set(rng.normal(0, 0.5, (64, S, H)), rng.normal(0, 0.1, H), rng.normal(0, 0.12, (H, H)),
               rng.normal(0, 0.1, H), rng.normal(0, 0.12, (H, n_out)), np.full(n_out, bias))
        nets[name] = nb
    res = {"hidden": H, "observation": "64 neighbours within 6.0 A (BCC shells 1-6)",
           "events": args.learned_events}
    for name, attach in (("pair", ()), ("policy", ("policy",)), ("poisson", ("poisson",)),
                         ("policy_poisson", ("policy", "poisson"))):
        lat = akmc.Lattice(spec, precision=akmc.FP32, stream=stream)
        if "policy" in attach:
            akmc.policy_attach(lat.h, nets["policy"].blob, 1.0)
        if "poisson" in attach:
            akmc.poisson_attach(lat.h, nets["poisson"].blob)
        with torch.cuda.stream(stream):
            lat.step(2000)
            torch.cuda.synchronize()
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            lat.step(args.learned_events)
            a1.record(stream)
            torch.cuda.synchronize()
        dt = a0.elapsed_time(a1) * 1e-3
        lat.close()
        res[name] = {"events_per_s": args.learned_events / dt, "us_per_event": dt * 1e6 / args.learned_events}
    res["policy_poisson_vs_pair"] = res["policy_poisson"]["events_per_s"] / res["pair"]["events_per_s"]
    return res


def bench_fp32_error(torch, akmc, W, stream):
    """Error of the binary32 path on the 4.2M-site lattice's initial state:
    every site's 8 rates and barriers and the vacancies' total rate against
    the binary64 path of the same library (which the parity tests hold
    within 1e-12 of the oracle)."""
    spec = W.rpv_4m()
    res = {}
    with torch.cuda.stream(stream):
        out = {}
        for prec in (akmc.FP32, akmc.FP64):
            lat = akmc.Lattice(spec, precision=prec, stream=stream)
            r, e = lat.rates(akmc.RATES_ALL_SITES, with_ea=True)
            rv = lat.rates(akmc.RATES_VACANCIES)
            torch.cuda.synchronize()
            out[prec] = (r.double(), e.double(), float(rv.double().sum()))
            lat.close()
        r32, e32, g32 = out[akmc.FP32]
        r64, e64, g64 = out[akmc.FP64]
        m = r64 > 0
        rel = ((r32 - r64).abs() / r64)[m]
        res = {"candidates": int(m.sum()), "mask_equal": bool(torch.equal(r32 > 0, m)),
               "max_rel_rate": float(rel.max()), "median_rel_rate": float(rel.median()),
               "max_abs_ea_ev": float((e32 - e64).abs()[m].max()),
               "gamma_tot_rel": abs(g32 - g64) / g64,
               "reference": "binary64 path of the same library"}
        del out, r32, e32, r64, e64, rel, m
    return res


MLP_FWD_FLOP = 2 * (160 * 128 + 128 * 128 + 128)     # per candidate, five species


def bench_surrogate(args, torch, akmc, W, stream):
    """Learned-barrier form on the same 4.2M-site lattice: training samples
    are the 8 candidates of random sites of the binary32 pair path (labels
    = pair barriers), the network is trained on the GPU, timed in bulk
    inference, and then drives the event loop (out-of-distribution
    candidates fall back to the pair barrier)."""
    S = 5
    spec = W.rpv_4m()
    rng = np.random.default_rng(2024)
    n_sites = args.surrogate_samples // 8
    with torch.cuda.stream(stream):
        lat = akmc.Lattice(spec, precision=akmc.FP32, stream=stream)
        lat.step(args.events)
        sites = torch.as_tensor(rng.choice(spec.n_sites, n_sites, replace=False).astype(np.int32),
                                device="cuda")
        env = torch.empty((n_sites * 8, 27), dtype=torch.uint8, device="cuda")
        ea = torch.empty(n_sites * 8, dtype=torch.float32, device="cuda")
        akmc.env_encode(lat.h, akmc.RATES_SITES, sites, n_sites, env, ea)
        lat.close()
        n = n_sites * 8
        n_train = (n * 9 // 10) // 256 * 256
        fin = torch.isfinite(ea[:n_train])
        mu, sigma = float(ea[:n_train][fin].mean()), float(ea[:n_train][fin].std())
        blob = torch.zeros(akmc.mlp_blob_bytes(S), dtype=torch.uint8, device="cuda")
        akmc.mlp_init(blob, S, 7, mu, sigma)
        akmc.mlp_fit_ood(blob, S, env, n_train)
        cfg = akmc.TrainCfg(batch=256, epochs=args.surrogate_epochs, lr=2e-3, lr_final=2e-5,
                            beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, shuffle=1, seed=5)
        work = torch.empty(akmc.mlp_train_workspace_bytes(S, 256), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        akmc.mlp_train(blob, S, env, ea, n_train, cfg, work)
        e1.record(stream)
        torch.cuda.synchronize()
        train_s = e0.elapsed_time(e1) * 1e-3
        pred = torch.empty(n, dtype=torch.float32, device="cuda")
        akmc.mlp_forward(blob, S, env, n, pred)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(5):
            akmc.mlp_forward(blob, S, env, n, pred)
        f1.record(stream)
        torch.cuda.synchronize()
        fwd_s = f0.elapsed_time(f1) * 1e-3 / 5
        t = ea[n_train:].double()
        m = torch.isfinite(t)
        err = pred[n_train:].double()[m] - t[m]
        rmse_mev = 1000 * float(torch.sqrt(torch.mean(err * err)))

        pair = akmc.Lattice(spec, precision=akmc.FP32, stream=stream)
        mlp = akmc.Lattice(spec, precision=akmc.FP32, stream=stream, barrier_model=akmc.BARRIER_MLP)
        akmc.mlp_attach(mlp.h, blob)
        times = {}
        for name, l in (("pair", pair), ("mlp", mlp)):
            l.step(1000)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            l.step(args.surrogate_events)
            b.record(stream)
            torch.cuda.synchronize()
            times[name] = a.elapsed_time(b) * 1e-3
        _, _, s_m = mlp.read()
        pair.close()
        mlp.close()
    fwd_flops = MLP_FWD_FLOP * n / fwd_s
    return {"samples": n, "train_samples": n_train, "epochs": args.surrogate_epochs,
            "train_s": train_s,
            "train_samples_per_s": n_train * args.surrogate_epochs / train_s,
            "train_tflops_dense_equiv": 3 * MLP_FWD_FLOP * n_train * args.surrogate_epochs / train_s / 1e12,
            "heldout_rmse_mev": rmse_mev,
            "forward_rows_per_s": n / fwd_s,
            "forward_tflops_dense_equiv": fwd_flops / 1e12,
            "forward_frac_of_bf16_peak": fwd_flops / 2.5e15,
            "loop_events_per_s": args.surrogate_events / times["mlp"],
            "pair_loop_events_per_s": args.surrogate_events / times["pair"],
            "loop_speedup_vs_pair": times["pair"] / times["mlp"],
            "ood_fallbacks_per_event": s_m.n_ood / (args.surrogate_events + 1000)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=100_000, help="events per step")
    ap.add_argument("--batch-events", type=int, default=100_000, help="events per replica (batched form)")
    ap.add_argument("--cpu-replica-events", type=int, default=3_000,
                    help="oracle events per replica of the all-core ensemble baseline")
    ap.add_argument("--cpu-rate-sites", type=int, default=100_000,
                    help="sites of the oracle's rate-evaluation sample")
    ap.add_argument("--cpu-events", type=int, default=30_000, help="oracle sample size (about 15 s)")
    ap.add_argument("--cpu-local-events", type=int, default=800_000,
                    help="sample of the oracle's local-refresh mode (about 10 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--fp64", action="store_true", help="time the binary64 path as the main line")
    ap.add_argument("--surrogate-samples", type=int, default=2_000_000,
                    help="training+held-out candidates of the learned-barrier form (0 = skip it)")
    ap.add_argument("--surrogate-epochs", type=int, default=1)
    ap.add_argument("--surrogate-events", type=int, default=20_000)
    ap.add_argument("--voxel-events", type=int, default=20_000,
                    help="median events per voxel to the ensemble's time horizon (0 = skip)")
    ap.add_argument("--voxel-tol", type=float, default=0.02, help="Eq. 9 tolerance of the voxel grid")
    ap.add_argument("--voxel-blocks", type=int, default=128, help="persistent groups of the ensemble")
    ap.add_argument("--learned-events", type=int, default=20_000,
                    help="events per form of the learned runtime (0 = skip)")
    ap.add_argument("--far-events", type=int, default=20_000,
                    help="events of the pair model out to 6.0 A (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise pass over 256 MiB (reads 256 MiB, writes "
                         "256 MiB): the reference for the HBM byte counters")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "script with --copy-calibration into the committed traffic record, then exit")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args.traffic_from[0], args.traffic_from[1], "fp64" if args.fp64 else "fp32")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path of one lattice runs on one device, and "
              "replica ensembles shard across GPUs without communication (not run here); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_24091_amd import akmc
    from paper_2604_24091_amd import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    precision = akmc.FP64 if args.fp64 else akmc.FP32
    rdt = torch.float64 if args.fp64 else torch.float32
    rbytes = 8 if args.fp64 else 4
    spec = W.rpv_4m()
    lat = akmc.Lattice(spec, precision=precision, stream=stream)
    rates = torch.empty((spec.n_sites, 8), dtype=rdt, device="cuda")
    torch.cuda.synchronize()

    def one_step(sweep_events=None):
        akmc.kmc_step(lat.h, args.events, None)
        if sweep_events is not None:
            sweep_events[0].record(stream)
        akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, rates)
        if sweep_events is not None:
            sweep_events[1].record(stream)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        sweeps = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
        loops = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)]
        for a, b in sweeps:  # create them; the sweep launches record them again
            a.record(stream)
            b.record(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            loops[k][0].record(stream)
            akmc.kmc_step(lat.h, args.events, None)
            loops[k][1].record(stream)
            # the sweep kernel's own start and end (hipExtLaunchKernel events)
            akmc.rates_timing(lat.h, sweeps[k][0], sweeps[k][1])
            akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, rates)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        akmc.rates_timing(lat.h, None, None)
    wall = t1 - t0
    sweep_each = [a.elapsed_time(b) for a, b in sweeps]
    sweep_ms = float(np.mean(sweep_each))
    loop_ms = float(np.mean([a.elapsed_time(b) for a, b in loops]))
    occ, slots, summ = lat.read()
    assert summ.n_events == args.events * (args.steps + args.warmup)
    rng = np.random.default_rng(77)
    sample_sites = np.sort(rng.choice(spec.n_sites, min(args.cpu_rate_sites, spec.n_sites),
                                      replace=False)).astype(np.int32)
    sample_rates = rates[torch.as_tensor(sample_sites.astype(np.int64), device="cuda")].double().cpu().numpy()
    # Plain fill and copy of the sweep's output array: the HBM rate this GPU
    # sustains for the same bytes, measured next to the vendor peak.
    other = torch.empty_like(rates)
    with torch.cuda.stream(stream):
        for _ in range(2):
            rates.fill_(1.0)
            other.copy_(rates)
        torch.cuda.synchronize()
        f0, f1, c1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        f0.record(stream)
        for _ in range(10):
            rates.fill_(1.0)
        f1.record(stream)
        for _ in range(10):
            other.copy_(rates)
        c1.record(stream)
        torch.cuda.synchronize()
    nbytes = rates.numel() * rates.element_size()
    fill_gbs = nbytes * 10 / (f0.elapsed_time(f1) * 1e-3) / 1e9
    copy_gbs = 2 * nbytes * 10 / (f1.elapsed_time(c1) * 1e-3) / 1e9
    del other
    assert np.array_equal(np.bincount(occ, minlength=5), np.bincount(spec.occ, minlength=5))
    lat.close()

    n_sites = spec.n_sites
    alg_bytes = n_sites * (1 + 8 * rbytes)
    achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    tag = "fp64" if args.fp64 else "fp32"
    traffic = measured_traffic(alg_bytes, tag)
    events_per_s = args.events * args.steps / wall
    line = {
        "metric": METRIC,
        "value": events_per_s,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": "rpv_4m: BCC 128^3 cells (4,194,304 sites), Fe-1.34Cu-0.70Ni-1.40Mn "
                               "at%, 200 vacancies, 563 K, seeded pair energies",
                   "events_per_step": args.events,
                   "precision": ("binary64 throughout" if args.fp64 else
                                 "binary32 energies/barriers/rates, binary64 sums and time"),
                   "step": "kmc_step(events) + rates_eval(ALL_SITES)"},
        "rate_evals_per_s": n_sites * 8 / (sweep_ms * 1e-3),
        "roofline": {"kernel": "k_rates_all (bulk sweep, 8 jump rates per site)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes,
                     "launch_ms": sweep_ms,
                     "launch_ms_each": [round(float(x), 5) for x in sweep_each],
                     "measured_fill_gbs": fill_gbs, "measured_copy_gbs": copy_gbs,
                     "frac_of_measured_fill": achieved / fill_gbs},
        "event_loop": {"kernel": "k_event_loop (one 64-lane group, persistent)",
                       "events_per_s": args.events / (loop_ms * 1e-3),
                       "us_per_event": loop_ms * 1e3 / args.events,
                       "bound": "per-event dependency chain on one CU (latency)"},
    }
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = src.numel() * 4
        del src, dst
    if not args.no_forms:
        line["forms"] = bench_forms(args, torch, akmc, W, stream)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_events)
        line["cpu_baseline_local"] = cpu_baseline(spec, args.cpu_local_events, local=True)
        line["cpu_baseline_rates"], line["fp32_vs_oracle"] = cpu_rate_baseline(
            spec, occ, sample_sites, sample_rates)
        if args.cpu_replica_events > 0:
            line["cpu_baseline_replicas"] = cpu_baseline_replicas(args.cpu_replica_events)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

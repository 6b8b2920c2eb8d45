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
                site) over its mean launch time from HIP events on its
                stream; traffic from the committed rocprofv3 counter
                summary when it still matches the kernel source;
  event_loop    per-event latency of the loop kernel;
  cpu_baseline  the CPU oracle (full rate recompute per event, binary64,
                one core) on a bounded sample of the same workload;
  forms         binary64 path, the batched replica ensemble (256 replicas
                of 16^3..48^3 cells) and the learned-barrier form, each timed
                separately outside the main timed region.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "KMC events/s + jump-rate evals/s at 4.2M sites; plain vs batched/surrogate"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_rates_all_rpv_4m_traffic.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("akmc_rates.hip", "akmc_device.hpp", "akmc_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2604_24091_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def cpu_baseline(spec, n_events):
    from oracle import akmc_oracle as O
    o = O.Oracle(spec, precision=0)
    t0 = time.perf_counter()
    done = o.run(n_events)
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": "first %d events of the same 4.2M-site lattice, binary64, full rate "
                      "recompute of all 1,600 candidates per event, one thread (%.1f s)" % (done, dt)}


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
    akmc.batch_step(b, args.batch_events)           # capture + warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    akmc.batch_step(b, args.batch_events)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3
    forms["batched"] = {"events_per_s": len(reps) * args.batch_events / dt,
                        "replicas": len(reps), "events_per_replica": args.batch_events,
                        "sites_total": int(sum(r.n_sites for r in reps)),
                        "schedule": {"group_lanes": chosen.group_lanes,
                                     "waves_per_block": chosen.waves_per_block,
                                     "hipgraph": 1}}
    akmc.batch_destroy(b)
    del ws
    return forms


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=100_000, help="events per step")
    ap.add_argument("--batch-events", type=int, default=2_000, help="events per replica (batched form)")
    ap.add_argument("--cpu-events", type=int, default=10_000, help="oracle sample size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--fp64", action="store_true", help="time the binary64 path as the main line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device-to-device copy (reference for HBM counters)")
    args = ap.parse_args()
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
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            loops[k][0].record(stream)
            akmc.kmc_step(lat.h, args.events, None)
            loops[k][1].record(stream)
            sweeps[k][0].record(stream)
            akmc.rates_eval(lat.h, akmc.RATES_ALL_SITES, None, 0, rates)
            sweeps[k][1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    wall = t1 - t0
    sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in sweeps]))
    loop_ms = float(np.mean([a.elapsed_time(b) for a, b in loops]))
    occ, slots, summ = lat.read()
    assert summ.n_events == args.events * (args.steps + args.warmup)
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
                     "launch_ms": sweep_ms},
        "event_loop": {"kernel": "k_event_loop (one 64-lane group, persistent)",
                       "events_per_s": args.events / (loop_ms * 1e-3),
                       "us_per_event": loop_ms * 1e3 / args.events,
                       "bound": "per-event dependency chain on one CU (latency)"},
    }
    if args.copy_calibration:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = src.numel()
        del src, dst
    if not args.no_forms:
        line["forms"] = bench_forms(args, torch, akmc, W, stream)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_events)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

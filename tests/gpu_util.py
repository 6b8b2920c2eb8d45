"""Helpers shared by the GPU parity tests: run the HIP path through the
C-ABI binding and compare with the oracle on the same seeded inputs."""
import sys

import numpy as np

from paper_2604_24091_amd import akmc


def banner(msg: str):
    """Names the case on stdout before each GPU step."""
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def run_gpu(spec, n_events, log=True, chunks=None, **kw):
    """Runs n_events on the GPU (optionally split into chunks) and returns
    (occ, slots, summary, log records)."""
    import torch
    lat = akmc.Lattice(spec, **kw)
    logs = []
    parts = chunks if chunks is not None else [n_events]
    assert sum(parts) == n_events
    for n in parts:
        buf = lat.step(n, log=log)
        if log:
            torch.cuda.synchronize()
            logs.append(akmc.log_to_numpy(buf, n))
    occ, slots, s = lat.read()
    lat.close()
    recs = np.concatenate(logs) if log and logs else None
    return occ, slots, s, recs


def first_divergence(gpu_log, orc_log):
    keys = ["n", "slot", "dir", "from_site", "to_site", "species"]
    n = min(len(gpu_log), len(orc_log))
    for k in keys:
        bad = np.flatnonzero(gpu_log[k][:n] != orc_log[k][:n])
        if bad.size:
            return int(bad[0])
    return None


def near_tie(oracle_mod, spec, gpu_log, e, precision=0, rel=1e-12):
    """True if, at event e of the trajectory both sides agree on up to e,
    the target u1*Gamma_tot lies within `rel` (relative to Gamma_tot) of a
    boundary of the cumulative rate sums: a selection that rounding alone
    can flip."""
    o = oracle_mod.Oracle(spec, precision=precision)
    if e > 0:
        o.follow(gpu_log[:e])
    rates, _ = o.rates_vacancies()
    r = rates.reshape(-1)
    cum = np.cumsum(r)
    g = cum[-1]
    u1, _ = oracle_mod.uniforms(spec.seed, spec.stream_id, int(o.state.n))
    target = u1 * g
    return bool(np.min(np.abs(cum - target)) <= rel * g)

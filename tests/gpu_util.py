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
    """Earliest event at which any recorded field differs (or the shorter
    log ends), or None."""
    keys = ["n", "slot", "dir", "from_site", "to_site", "species"]
    n = min(len(gpu_log), len(orc_log))
    first = None
    for k in keys:
        bad = np.flatnonzero(gpu_log[k][:n] != orc_log[k][:n])
        if bad.size and (first is None or bad[0] < first):
            first = int(bad[0])
    if first is None and len(gpu_log) != len(orc_log):
        first = n
    return first


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


def assert_matches_oracle(oracle_mod, spec, gpu, n_events, precision=0, time_mode=0, rtol=None):
    """The GPU run gpu = (occ, slots, summary, log) against the oracle on the
    same inputs.  If both trajectories agree, the final state, digest, time
    and the per-event totals must match.  If they part at some event, that
    event must be a near tie (the target within rtol of a cumulative-sum
    boundary, which the rounding order of the sums alone can flip), and the
    whole GPU log is then replayed by the oracle's follow mode: every later
    event is still checked against the oracle's rates of the state it was
    taken from.  Returns the number of events at which the GPU's choice lies
    outside its exact interval (0 unless a near tie was met)."""
    occ_g, slots_g, s_g, log_g = gpu
    if rtol is None:
        rtol = 1e-12 if precision == 0 else 1e-5
    o = oracle_mod.Oracle(spec, precision=precision, time_mode=time_mode)
    done, log_o = o.run(n_events, log=True)
    assert done == n_events == len(log_g)
    e = first_divergence(log_g, log_o)
    if e is None:
        assert np.array_equal(occ_g, o.occ)
        assert np.array_equal(slots_g, o.slots)
        assert s_g.digest == o.state.digest
        assert s_g.n_events == o.state.n
        np.testing.assert_allclose(log_g["gamma_tot"], log_o["gamma_tot"], rtol=rtol)
        np.testing.assert_allclose(log_g["dt"], log_o["dt"], rtol=rtol)
        assert abs(s_g.t - o.state.t) <= rtol * abs(o.state.t)
        assert abs(s_g.gamma_tot - o.state.gamma_tot) <= rtol * o.state.gamma_tot
        return 0
    assert near_tie(oracle_mod, spec, log_g, e, precision, rel=rtol), \
        "divergence at event %d is not a near tie" % e
    print("[gpu-case] near tie at event %d: following the GPU log from there" % e, flush=True)
    f = oracle_mod.Oracle(spec, precision=precision, time_mode=time_mode)
    res = f.follow(log_g)
    assert res["mismatches"] == 0
    assert res["max_select_violation"] <= rtol
    assert res["max_gamma_rel"] <= rtol and res["max_dt_rel"] <= rtol
    assert res["n_differ"] <= 1 + n_events // 100000
    assert np.array_equal(occ_g, f.occ) and np.array_equal(slots_g, f.slots)
    assert s_g.digest == f.state.digest and s_g.n_events == f.state.n
    assert abs(s_g.t - f.state.t) <= rtol * abs(f.state.t)
    return res["n_differ"]


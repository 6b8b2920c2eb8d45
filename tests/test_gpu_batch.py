"""GPU parity of the batched replica ensemble (akmc_batch_*).

Every replica of a batch must end bit for bit where a standalone lattice
with the same parameters ends (occupancy, slots, digest, time), for every
launch schedule; replicas are checked against the oracle too.
"""
import numpy as np
import pytest

from paper_2604_24091_amd import akmc
from paper_2604_24091_amd import workloads as W
from tests.gpu_util import assert_matches_oracle, banner, run_gpu

pytestmark = pytest.mark.gpu


def _batch(specs, n_events, sched=None, chunks=None, precision=akmc.FP64):
    import torch
    params = [akmc.make_params(s, precision=precision) for s in specs]
    nv = [int(np.count_nonzero(s.occ == s.n_species - 1)) for s in specs]
    nbytes = akmc.batch_workspace_bytes(params, nv)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = akmc.batch_create(params, [s.occ for s in specs], ws)
    if sched is not None:
        akmc.batch_set_schedule(b, sched)
    for n in (chunks or [n_events]):
        akmc.batch_step(b, n)
    out = []
    for r, s in enumerate(specs):
        occ = np.empty(s.n_sites, np.uint8)
        sl = np.empty(max(nv[r], 1), np.int32)
        summ = akmc.batch_state_read(b, r, occ, sl)
        out.append((occ, sl[:nv[r]], summ))
    akmc.batch_destroy(b)
    return out


def _small_replicas(n_rep=24, seed=5):
    specs = W.rpv_replicas(n_rep=n_rep, seed=seed, cells_range=(4, 12), max_vac=20)
    return specs


@pytest.mark.parametrize("lanes,waves,graph", [(8, 1, 0), (16, 2, 0), (32, 1, 1), (64, 4, 0), (8, 4, 1)])
def test_batch_equals_standalone(lanes, waves, graph):
    banner("batch lanes=%d waves=%d graph=%d" % (lanes, waves, graph))
    specs = _small_replicas()
    n = 3000
    sched = akmc.Schedule(lanes, waves, 0, graph, 1000)
    res = _batch(specs, n, sched)
    for r in (0, 5, 11, 23):
        occ, sl, s, _ = run_gpu(specs[r], n, log=False)
        bo, bsl, bs = res[r]
        assert np.array_equal(bo, occ) and np.array_equal(bsl, sl)
        assert bs.digest == s.digest and bs.t == s.t and bs.n_events == s.n_events == n


def test_batch_schedules_agree_and_match_oracle(oracle_mod):
    banner("batch schedules vs oracle")
    specs = _small_replicas(n_rep=12, seed=9)
    n = 2000
    a = _batch(specs, n, akmc.Schedule(8, 1, 0, 0, 700))
    b = _batch(specs, n, akmc.Schedule(64, 2, 3, 0, 2000))
    for r in range(len(specs)):
        assert np.array_equal(a[r][0], b[r][0])
        assert a[r][2].digest == b[r][2].digest and a[r][2].t == b[r][2].t
    # Replicas against the oracle: the standalone run with its event log
    # ends where the replica ends, and that log is checked event by event
    # (a near tie is verified and then followed to the end, never skipped).
    for r in (0, 3, 7, 11):
        gpu = run_gpu(specs[r], n)
        assert np.array_equal(gpu[0], a[r][0]) and gpu[2].digest == a[r][2].digest
        assert gpu[2].t == a[r][2].t
        assert_matches_oracle(oracle_mod, specs[r], gpu, n)


def test_batch_autotune_keeps_results():
    banner("batch autotune")
    import torch
    specs = _small_replicas(n_rep=16, seed=13)
    params = [akmc.make_params(s) for s in specs]
    nv = [int(np.count_nonzero(s.occ == 4)) for s in specs]
    ws = torch.empty(akmc.batch_workspace_bytes(params, nv), dtype=torch.uint8, device="cuda")
    b = akmc.batch_create(params, [s.occ for s in specs], ws)
    chosen = akmc.batch_autotune(b, 100)        # 8 trials x 100 events
    assert chosen.group_lanes in (8, 16, 32, 64) and chosen.waves_per_block in (1, 2)
    akmc.batch_step(b, 200)
    occ = np.empty(specs[3].n_sites, np.uint8)
    s = akmc.batch_state_read(b, 3, occ)
    akmc.batch_destroy(b)
    ref = run_gpu(specs[3], 1000, log=False)
    assert np.array_equal(occ, ref[0]) and s.digest == ref[2].digest


def test_batch_fp32_equals_standalone():
    banner("batch fp32")
    specs = _small_replicas(n_rep=10, seed=17)
    res = _batch(specs, 2000, akmc.Schedule(16, 1, 0, 0, 2000), precision=akmc.FP32)
    for r in (0, 9):
        occ, sl, s, _ = run_gpu(specs[r], 2000, log=False, precision=akmc.FP32)
        assert np.array_equal(res[r][0], occ) and res[r][2].digest == s.digest


def test_batch_up_to_the_vacancy_limit_fits_lds():
    """Replicas up to the vacancy limit (512): a schedule whose groups need
    more LDS than a workgroup has is refused (UNSUPPORTED), the initial
    schedule and the autotuner use only schedules that fit, and every
    replica still ends where its standalone run ends."""
    import torch
    banner("batch up to the vacancy limit")
    rng = np.random.default_rng(23)
    specs = [W.random_lattice(rng, (12, 12, 12), 5, nv, solute_total=0.2)
             for nv in (akmc.MAX_VACANCIES, 300, 40, 3)]
    params = [akmc.make_params(s) for s in specs]
    nv = [int(np.count_nonzero(s.occ == 4)) for s in specs]
    ws = torch.empty(akmc.batch_workspace_bytes(params, nv), dtype=torch.uint8, device="cuda")
    b = akmc.batch_create(params, [s.occ for s in specs], ws)
    for lanes, waves in ((8, 1), (16, 1), (64, 4)):
        with pytest.raises(akmc.AkmcError):
            akmc.batch_set_schedule(b, akmc.Schedule(lanes, waves, 0, 0, 1000))
    akmc.batch_step(b, 300)                     # initial schedule
    chosen = akmc.batch_autotune(b, 100)
    assert chosen.group_lanes >= 32
    akmc.batch_step(b, 400)
    outs = []
    for r, s in enumerate(specs):
        occ = np.empty(s.n_sites, np.uint8)
        outs.append((occ, akmc.batch_state_read(b, r, occ)))
    akmc.batch_destroy(b)
    n = outs[0][1].n_events
    assert all(o[1].n_events == n for o in outs) and n >= 1000
    for r in range(len(specs)):
        occ, _, s, _ = run_gpu(specs[r], n, log=False)
        assert np.array_equal(outs[r][0], occ) and outs[r][1].digest == s.digest


def test_replica_ensemble_production_run():
    """The 256-replica ensemble (16^3..48^3 cells, 1-20 vacancies, 523-593 K)
    as a production run: 10^5 binary32 events per replica under the
    autotuned schedule with graph replay; every replica conserves its
    species and ran every event, and three replicas (the first, a middle
    and the last in creation order) end bit for bit where their standalone
    runs end."""
    import torch
    banner("batch ensemble production 1e5 events per replica")
    specs = W.rpv_replicas()
    params = [akmc.make_params(s, precision=akmc.FP32) for s in specs]
    nv = [int(np.count_nonzero(s.occ == 4)) for s in specs]
    ws = torch.empty(akmc.batch_workspace_bytes(params, nv), dtype=torch.uint8, device="cuda")
    b = akmc.batch_create(params, [s.occ for s in specs], ws)
    chosen = akmc.batch_autotune(b, 100)
    akmc.batch_set_schedule(b, akmc.Schedule(chosen.group_lanes, chosen.waves_per_block, chosen.blocks,
                                             1, 20_000))
    akmc.batch_step(b, 100_000)
    outs = []
    for r, s in enumerate(specs):
        occ = np.empty(s.n_sites, np.uint8)
        summ = akmc.batch_state_read(b, r, occ)
        outs.append((occ, summ))
        assert summ.frozen == 0
        assert np.array_equal(np.bincount(occ, minlength=5), np.bincount(s.occ, minlength=5))
    akmc.batch_destroy(b)
    n = outs[0][1].n_events
    assert n == 100_000 + 8 * 100 and all(o[1].n_events == n for o in outs)
    for r in (0, 128, 255):
        occ, _, s, _ = run_gpu(specs[r], n, log=False, precision=akmc.FP32)
        assert np.array_equal(outs[r][0], occ) and outs[r][1].digest == s.digest and outs[r][1].t == s.t

"""GPU parity of the pair model out to 6.0 A (six shells, n_shells = 6)
against the oracle: rates and barriers of site lists and of every site
(binary64 within 1e-12, binary32 within 1e-5 of the binary64 oracle), the
event loop's trajectory (binary64: bit-exact up to near ties, followed to
the end), LOCAL == FULL and chunked == unchunked bit for bit, the loop's
barriers, and a 128^3-cell lattice followed event by event in binary32."""
import numpy as np
import pytest

from paper_2604_24091_amd import akmc
from paper_2604_24091_amd import workloads as W
from tests.gpu_util import assert_matches_oracle, banner, run_gpu

pytestmark = pytest.mark.gpu


def _far(rng, dims, S, nv, solute_total=0.3):
    spec = W.random_lattice(rng, dims, S, nv, solute_total=solute_total)
    spec.eps_far = W.far_tables(rng, S)
    return spec


@pytest.mark.parametrize("precision", [akmc.FP64, akmc.FP32])
def test_far_rates_match_oracle(oracle_mod, precision):
    import torch
    banner("far rates precision=%d" % precision)
    rng = np.random.default_rng(21)
    spec = _far(rng, (5, 6, 7), 5, 9)
    lat = akmc.Lattice(spec, precision=precision)
    try:
        sites = np.concatenate([rng.integers(0, spec.n_sites, 200), [0, spec.n_sites - 1]])
        r_s, e_s = lat.rates(akmc.RATES_SITES, sites, with_ea=True)
        r_a, e_a = lat.rates(akmc.RATES_ALL_SITES, with_ea=True)
        r_v = lat.rates(akmc.RATES_VACANCIES)
        torch.cuda.synchronize()
        r_s, e_s = r_s.double().cpu().numpy(), e_s.double().cpu().numpy()
        r_a, e_a = r_a.double().cpu().numpy(), e_a.double().cpu().numpy()
        r_v = r_v.double().cpu().numpy()
    finally:
        lat.close()
    o = oracle_mod.Oracle(spec)
    ro_a, eo_a = o.rates_sites(np.arange(spec.n_sites, dtype=np.int32))
    tol, etol = (1e-12, 1e-12) if precision == akmc.FP64 else (1e-5, 1e-6)
    for r, e, ro, eo in ((r_a, e_a, ro_a, eo_a), (r_s, e_s, ro_a[sites], eo_a[sites]),
                         (r_v, None, ro_a[o.slots], None)):
        m = ro > 0
        assert np.array_equal(r > 0, m)
        assert np.max(np.abs(r[m] - ro[m]) / ro[m]) <= tol
        if e is not None:
            assert np.max(np.abs(e[m] - eo[m])) <= etol and np.all(np.isinf(e[~m]))
    if precision == akmc.FP32:
        o32 = oracle_mod.Oracle(spec, precision=1)
        r32, _ = o32.rates_sites(np.arange(spec.n_sites, dtype=np.int32))
        m = r32 > 0
        assert np.max(np.abs(r_a[m] - r32[m]) / r32[m]) <= 1e-5


@pytest.mark.parametrize("refresh", [akmc.REFRESH_LOCAL, akmc.REFRESH_FULL])
def test_far_loop_matches_oracle_fp64(oracle_mod, refresh):
    banner("far loop fp64 refresh=%d" % refresh)
    rng = np.random.default_rng(22)
    spec = _far(rng, (6, 6, 6), 5, 12)
    gpu = run_gpu(spec, 3000, precision=akmc.FP64, refresh=refresh)
    assert_matches_oracle(oracle_mod, spec, gpu, 3000)


def test_far_local_equals_full_and_chunks():
    banner("far local == full, chunks")
    rng = np.random.default_rng(23)
    spec = _far(rng, (5, 5, 6), 4, 40, solute_total=0.2)    # crowded: many slots refreshed
    a = run_gpu(spec, 2000, log=False, precision=akmc.FP64, refresh=akmc.REFRESH_LOCAL)
    b = run_gpu(spec, 2000, log=False, precision=akmc.FP64, refresh=akmc.REFRESH_FULL)
    c = run_gpu(spec, 2000, log=False, precision=akmc.FP64, chunks=[1, 700, 1299])
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and a[2].digest == x[2].digest and a[2].t == x[2].t


def test_far_loop_barriers(oracle_mod):
    banner("far loop barriers")
    import torch
    rng = np.random.default_rng(24)
    spec = _far(rng, (6, 7, 6), 5, 10)
    lat = akmc.Lattice(spec, precision=akmc.FP64)
    lat.step(1500)
    ea = lat.barriers().double().cpu().numpy()
    occ, slots, _ = lat.read()
    lat.close()
    o = oracle_mod.Oracle(W.LatticeSpec(**{**spec.__dict__, "occ": occ}))
    _, eo = o.rates_sites(slots)
    m = np.isfinite(eo)
    assert np.array_equal(np.isfinite(ea), m)
    assert np.max(np.abs(ea[m] - eo[m])) <= 1e-12


def test_far_loop_fp32_on_the_4m_lattice(oracle_mod):
    """The 128^3-cell workload with pairs out to 6.0 A, binary32 rates:
    3,000 events followed by the binary64 oracle."""
    banner("far loop rpv_4m fp32 3000")
    spec = W.rpv_4m_far()
    occ, slots, s, log = run_gpu(spec, 3000, precision=akmc.FP32)
    f = oracle_mod.Oracle(spec)
    res = f.follow(log)
    print("[gpu-case] far 4m follow: %s" % res, flush=True)
    assert res["mismatches"] == 0
    assert res["max_select_violation"] <= 1e-5
    assert res["max_gamma_rel"] <= 1e-5 and res["max_dt_rel"] <= 1e-5
    assert res["n_differ"] <= 3
    assert np.array_equal(occ, f.occ) and s.digest == f.state.digest

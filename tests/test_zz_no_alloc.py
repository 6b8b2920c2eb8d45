"""The allocation-free cluster histogram (akmc_cluster_hist_noalloc, scratch
held by the library in its own device code object) against the entry point
with a caller scratch buffer (akmc_cluster_hist), through the C ABI: integer
work, so bin for bin.  Two calls in a row share the library's scratch; the
second is on a smaller lattice, so what the first left behind must not leak
into it.  Also: a lattice above the scratch's limit is refused with a clear
error."""
import numpy as np
import pytest

from paper_2604_24091_amd import akmc
from paper_2604_24091_amd import workloads as W
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def _both(lat, species, max_size):
    import torch
    ref = lat.clusters(species, max_size)
    got = torch.full((max_size + 1,), -7, dtype=torch.int64, device=lat.ws.device)
    akmc.cluster_hist_noalloc(lat.h, species, max_size, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_matches_scratch_entry_point_on_two_calls(oracle_mod):
    banner("cluster_hist_noalloc: 64^3 cells then 12x10x8")
    big = W.random_lattice(np.random.default_rng(31), (64, 64, 64), 4, 20, solute_total=0.2)
    small = W.random_lattice(np.random.default_rng(32), (12, 10, 8), 5, 7, solute_total=0.4)
    for spec, species, max_size in ((big, 1, 4096), (small, 2, 64)):
        lat = akmc.Lattice(spec)
        try:
            ref, got = _both(lat, species, max_size)
            occ, _, _ = lat.read()
        finally:
            lat.close()
        assert np.array_equal(got, ref), (spec.dims, species)
        n, oracle_hist = oracle_mod.Oracle(spec).cluster_hist(species, max_size, occ)
        assert np.array_equal(got, oracle_hist)
        assert int(got.sum()) == n > 0


def test_noalloc_after_events_and_at_the_limit(oracle_mod):
    """The 128^3-cell production lattice (exactly the scratch limit) after
    some events, then a smaller one again."""
    banner("cluster_hist_noalloc: 128^3 cells after 2000 events, then 16^3")
    for spec, n_ev in ((W.rpv_4m(), 2000), (W.random_lattice(np.random.default_rng(33), (16, 16, 16),
                                                            4, 3, solute_total=0.1), 500)):
        assert spec.n_sites <= akmc.CLUSTER_STATIC_MAX_SITES
        lat = akmc.Lattice(spec)
        try:
            lat.step(n_ev)
            ref, got = _both(lat, 1, 256)
        finally:
            lat.close()
        assert np.array_equal(got, ref)
        assert got[0] == 0 and got.sum() > 0


def test_noalloc_refuses_lattices_above_its_scratch():
    banner("cluster_hist_noalloc: refusal above the limit")
    spec = W.pure_fe((130, 128, 128), 1, 5)
    assert spec.n_sites > akmc.CLUSTER_STATIC_MAX_SITES
    lat = akmc.Lattice(spec)
    try:
        import torch
        hist = torch.zeros(9, dtype=torch.int64, device=lat.ws.device)
        with pytest.raises(akmc.AkmcError) as e:
            akmc.cluster_hist_noalloc(lat.h, 0, 8, hist)
        assert e.value.status == akmc.ERR_UNSUPPORTED
        assert "AKMC_CLUSTER_STATIC_MAX_SITES" in str(e.value)
    finally:
        lat.close()

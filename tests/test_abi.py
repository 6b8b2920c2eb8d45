"""The C-ABI library loads, exports every function include/akmc.h declares,
and rejects bad arguments on the host before touching a GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_2604_24091_amd import akmc
from paper_2604_24091_amd import workloads as W


def test_library_exports_every_declared_symbol():
    names = akmc.header_functions()
    assert len(names) >= 15
    L = akmc.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    assert akmc.status_string(akmc.OK) == "ok"
    assert "frozen" in akmc.status_string(akmc.ERR_FROZEN)


def test_workspace_bytes_and_validation():
    spec = W.fe_cu_2k()
    p = akmc.make_params(spec)
    n = akmc.workspace_bytes(p, 1)
    assert n >= spec.n_sites
    bad = akmc.make_params(spec)
    bad.lx = 2
    with pytest.raises(akmc.AkmcError) as e:
        akmc.workspace_bytes(bad, 1)
    assert e.value.status == akmc.ERR_INVALID and "edges" in str(e.value)
    bad = akmc.make_params(spec)
    bad.eps1[1] += 0.1            # breaks symmetry
    with pytest.raises(akmc.AkmcError):
        akmc.workspace_bytes(bad, 1)
    bad = akmc.make_params(spec)
    bad.temperature = -1.0
    with pytest.raises(akmc.AkmcError):
        akmc.workspace_bytes(bad, 1)
    with pytest.raises(akmc.AkmcError):
        akmc.workspace_bytes(p, akmc.MAX_VACANCIES + 1)


def test_create_rejects_null_and_bad_codes_without_gpu():
    spec = W.fe_cu_2k()
    p = akmc.make_params(spec)
    L = akmc.lib()
    h = C.c_void_p()
    st = L.akmc_lattice_create(C.byref(p), None, None, None, 0, None, C.byref(h))
    assert st == akmc.ERR_INVALID
    occ = spec.occ.copy()
    occ[5] = 9
    fake_ws = C.c_void_p(256 * 1024)     # never dereferenced: validation fails first
    st = L.akmc_lattice_create(C.byref(p), occ.ctypes.data, None, fake_ws, 1 << 20, None, C.byref(h))
    assert st == akmc.ERR_INVALID and "code" in akmc.last_error()
    st = L.akmc_lattice_create(C.byref(p), spec.occ.ctypes.data, None, fake_ws, 16, None, C.byref(h))
    assert st == akmc.ERR_WORKSPACE
    misaligned = C.c_void_p(256 * 1024 + 8)
    st = L.akmc_lattice_create(C.byref(p), spec.occ.ctypes.data, None, misaligned, 1 << 20, None, C.byref(h))
    assert st == akmc.ERR_INVALID
    bad_slots = np.array([0], dtype=np.int32)
    st = L.akmc_lattice_create(C.byref(p), spec.occ.ctypes.data, bad_slots.ctypes.data, fake_ws, 1 << 20, None, C.byref(h))
    assert st == akmc.ERR_INVALID


def test_struct_sizes_match_header():
    assert C.sizeof(akmc.Event) == 40
    assert C.sizeof(akmc.Params) == (4 * 4 + 8 * (64 + 64 + 8) + 8 * 3 + 8 * 2 + 8 * 3 + 4 * 4
                                     + 4 * 2 + 8 * 4 * 64)


def test_null_handles_are_rejected_without_gpu():
    """Every entry point that takes a lattice or batch handle checks it
    first: NULL gives ERR_INVALID and touches no device."""
    L = akmc.lib()
    calls = [
        lambda: L.akmc_rates_eval(None, 0, None, 0, None, None),
        lambda: L.akmc_rates_timing(None, None, None),
        lambda: L.akmc_kmc_step(None, 1, None),
        lambda: L.akmc_state_read(None, None, None, None),
        lambda: L.akmc_cluster_scratch_bytes(None, None),
        lambda: L.akmc_cluster_hist(None, 1, 8, None, None, 0),
        lambda: L.akmc_lattice_destroy(None),
        lambda: L.akmc_env_encode(None, 0, None, 0, None, None),
        lambda: L.akmc_mlp_attach(None, None),
        lambda: L.akmc_batch_set_schedule(None, None),
        lambda: L.akmc_batch_step(None, 1),
        lambda: L.akmc_batch_autotune(None, 1, None),
        lambda: L.akmc_batch_state_read(None, 0, None, None, None),
        lambda: L.akmc_batch_destroy(None),
        lambda: L.akmc_cluster_hist_noalloc(None, 1, 8, None),
        lambda: L.akmc_kmc_run_until(None, 1.0, 1, None),
        lambda: L.akmc_batch_priority(None, None, None),
        lambda: L.akmc_batch_run_until(None, 1.0, 1, 0),
        lambda: L.akmc_patchnet_eval(None, None, None, 0, None),
        lambda: L.akmc_policy_attach(None, None, 1.0),
        lambda: L.akmc_poisson_attach(None, None),
        lambda: L.akmc_patchnet_blob_bytes(5, 0, 8, None),
        lambda: L.akmc_patchnet_blob_bytes(5, 16, 3, None),
        lambda: L.akmc_patchnet_blob_bytes(5, 12, 8, None),
        lambda: L.akmc_voxel_grid(None, 1, 1, 0.6, 1e-4, 0.1, None, None, None, None),
    ]
    for call in calls:
        assert call() == akmc.ERR_INVALID
        assert akmc.last_error()


def test_params_checks_of_the_far_pair_model():
    """n_shells must be 2 or 6; the six-shell model needs edges of 5 cells
    and symmetric far tables (host-side checks, no GPU)."""
    spec = W.random_lattice(np.random.default_rng(3), (5, 5, 5), 4, 2)
    spec.eps_far = W.far_tables(np.random.default_rng(4), 4)
    p = akmc.make_params(spec)
    assert p.n_shells == 6 and akmc.workspace_bytes(p, 2) > 0
    bad = akmc.make_params(spec)
    bad.n_shells = 3
    with pytest.raises(akmc.AkmcError):
        akmc.workspace_bytes(bad, 2)
    bad = akmc.make_params(spec)
    bad.eps_far[2][1] += 0.01
    with pytest.raises(akmc.AkmcError) as e:
        akmc.workspace_bytes(bad, 2)
    assert "symmetric" in str(e.value)
    small = W.random_lattice(np.random.default_rng(5), (4, 5, 5), 4, 2)
    small.eps_far = spec.eps_far
    with pytest.raises(akmc.AkmcError) as e:
        akmc.workspace_bytes(akmc.make_params(small), 2)
    assert "5 cells" in str(e.value)

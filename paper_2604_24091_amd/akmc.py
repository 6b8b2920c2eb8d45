"""Python binding of libakmc.so (include/akmc.h).

Argument marshalling only: every step of the path runs in the HIP
library.  Device buffers are torch tensors on a ROCm device (PyTorch owns
device memory); the HIP stream is torch's current stream unless given.
Importing this module never falls back to anything: if libakmc.so is
missing it raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libakmc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "akmc.h")

OK, ERR_INVALID, ERR_WORKSPACE, ERR_HIP, ERR_FROZEN, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
REFRESH_LOCAL, REFRESH_FULL = 0, 1
TIME_STOCHASTIC, TIME_MEAN = 0, 1
BARRIER_PAIR, BARRIER_MLP = 0, 1
RATES_VACANCIES, RATES_SITES, RATES_ALL_SITES = 0, 1, 2
ORDER_PRIORITY, ORDER_INDEX, ORDER_CREATE = 0, 1, 2
MAX_VACANCIES = 512
CLUSTER_STATIC_MAX_SITES = 4194304


class Params(C.Structure):
    _fields_ = [("lx", C.c_int32), ("ly", C.c_int32), ("lz", C.c_int32),
                ("n_species", C.c_int32),
                ("eps1", C.c_double * 64), ("eps2", C.c_double * 64), ("e0", C.c_double * 8),
                ("nu", C.c_double), ("temperature", C.c_double), ("kb", C.c_double),
                ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("event_counter0", C.c_int64), ("time0", C.c_double), ("digest0", C.c_uint64),
                ("precision", C.c_int32), ("refresh", C.c_int32), ("time_mode", C.c_int32),
                ("barrier_model", C.c_int32), ("n_shells", C.c_int32), ("pad_", C.c_int32),
                ("eps_far", (C.c_double * 64) * 4)]


class Event(C.Structure):
    _fields_ = [("n", C.c_int64), ("slot", C.c_int32), ("from_site", C.c_int32),
                ("to_site", C.c_int32), ("dir", C.c_uint8), ("species", C.c_uint8),
                ("pad", C.c_uint8 * 2), ("gamma_tot", C.c_double), ("dt", C.c_double)]


class Summary(C.Structure):
    _fields_ = [("t", C.c_double), ("n_events", C.c_int64), ("gamma_tot", C.c_double),
                ("digest", C.c_uint64), ("species_count", C.c_int64 * 8),
                ("n_neg_barrier", C.c_int64), ("n_neg_reverse", C.c_int64), ("n_ood", C.c_int64),
                ("n_vacancies", C.c_int32), ("frozen", C.c_int32), ("loop_seconds", C.c_double)]


class TrainCfg(C.Structure):
    _fields_ = [("batch", C.c_int32), ("epochs", C.c_int32), ("lr", C.c_float),
                ("lr_final", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("weight_decay", C.c_float), ("shuffle", C.c_int32),
                ("pad_", C.c_int32), ("seed", C.c_uint64)]


class Schedule(C.Structure):
    _fields_ = [("group_lanes", C.c_int32), ("waves_per_block", C.c_int32),
                ("blocks", C.c_int32), ("use_graph", C.c_int32), ("chunk_events", C.c_int64)]


EVENT_DTYPE = np.dtype([("n", "<i8"), ("slot", "<i4"), ("from_site", "<i4"),
                        ("to_site", "<i4"), ("dir", "u1"), ("species", "u1"),
                        ("pad", "u1", (2,)), ("gamma_tot", "<f8"), ("dt", "<f8")])
assert EVENT_DTYPE.itemsize == C.sizeof(Event) == 40


class AkmcError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__("%s failed: %s (%s)" % (what, status_string(status), detail))
        self.status = status


_lib = None


def lib():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libakmc.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        P = C.POINTER(Params)
        L.akmc_workspace_bytes.argtypes = [P, C.c_int32, C.POINTER(sz)]
        L.akmc_lattice_create.argtypes = [P, vp, vp, vp, sz, vp, C.POINTER(vp)]
        L.akmc_rates_eval.argtypes = [vp, C.c_int32, vp, C.c_int64, vp, vp]
        L.akmc_rates_timing.argtypes = [vp, vp, vp]
        L.akmc_kmc_step.argtypes = [vp, C.c_int64, vp]
        L.akmc_kmc_run_until.argtypes = [vp, C.c_double, C.c_int64, vp]
        L.akmc_voxel_grid.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), vp,
                                      C.POINTER(C.c_double)]
        L.akmc_batch_priority.argtypes = [vp, vp, vp]
        L.akmc_batch_run_until.argtypes = [vp, C.c_double, C.c_int64, C.c_int32]
        L.akmc_patchnet_blob_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(sz)]
        L.akmc_patchnet_set.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.akmc_patchnet_get.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32), vp]
        L.akmc_patchnet_eval.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.akmc_policy_attach.argtypes = [vp, vp, C.c_float]
        L.akmc_poisson_attach.argtypes = [vp, vp]
        L.akmc_state_read.argtypes = [vp, vp, vp, C.POINTER(Summary)]
        L.akmc_loop_barriers.argtypes = [vp, vp]
        L.akmc_lattice_destroy.argtypes = [vp]
        L.akmc_cluster_scratch_bytes.argtypes = [vp, C.POINTER(sz)]
        L.akmc_cluster_hist.argtypes = [vp, C.c_int32, C.c_int64, vp, vp, sz]
        L.akmc_cluster_hist_noalloc.argtypes = [vp, C.c_int32, C.c_int64, vp]
        L.akmc_batch_workspace_bytes.argtypes = [C.c_int32, P, vp, C.POINTER(sz)]
        L.akmc_batch_create.argtypes = [C.c_int32, P, vp, vp, vp, sz, vp, C.POINTER(vp)]
        L.akmc_batch_set_schedule.argtypes = [vp, C.POINTER(Schedule)]
        L.akmc_batch_step.argtypes = [vp, C.c_int64]
        L.akmc_batch_autotune.argtypes = [vp, C.c_int64, C.POINTER(Schedule)]
        L.akmc_batch_state_read.argtypes = [vp, C.c_int32, vp, vp, C.POINTER(Summary)]
        L.akmc_batch_destroy.argtypes = [vp]
        i32 = C.c_int32
        L.akmc_mlp_blob_bytes.argtypes = [i32, C.POINTER(sz)]
        L.akmc_mlp_param_count.argtypes = [i32, C.POINTER(i32)]
        L.akmc_mlp_init.argtypes = [vp, i32, C.c_uint64, C.c_float, C.c_float, vp]
        L.akmc_mlp_set_params.argtypes = [vp, i32, vp, C.c_float, C.c_float, vp]
        L.akmc_mlp_get_params.argtypes = [vp, i32, vp, C.POINTER(C.c_float), C.POINTER(C.c_float), vp]
        L.akmc_env_encode.argtypes = [vp, i32, vp, C.c_int64, vp, vp]
        L.akmc_mlp_fit_ood.argtypes = [vp, i32, vp, C.c_int64, vp]
        L.akmc_mlp_forward.argtypes = [vp, i32, vp, C.c_int64, vp, vp]
        L.akmc_mlp_train_workspace_bytes.argtypes = [i32, i32, C.POINTER(sz)]
        L.akmc_mlp_train.argtypes = [vp, i32, vp, vp, C.c_int64, C.POINTER(TrainCfg), vp, vp, sz, vp]
        L.akmc_mlp_grad.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, sz, vp]
        L.akmc_mlp_attach.argtypes = [vp, vp]
        for name in ("akmc_mlp_blob_bytes", "akmc_mlp_param_count", "akmc_mlp_init",
                     "akmc_mlp_set_params", "akmc_mlp_get_params", "akmc_env_encode",
                     "akmc_mlp_fit_ood", "akmc_mlp_forward", "akmc_mlp_train_workspace_bytes",
                     "akmc_mlp_train", "akmc_mlp_grad", "akmc_mlp_attach"):
            getattr(L, name).restype = C.c_int32
        L.akmc_status_string.argtypes = [C.c_int32]
        L.akmc_status_string.restype = C.c_char_p
        L.akmc_last_error.restype = C.c_char_p
        for name in ("akmc_workspace_bytes", "akmc_lattice_create", "akmc_rates_eval",
                     "akmc_rates_timing", "akmc_kmc_step", "akmc_loop_barriers", "akmc_state_read",
                     "akmc_lattice_destroy", "akmc_cluster_scratch_bytes", "akmc_cluster_hist",
                     "akmc_cluster_hist_noalloc", "akmc_kmc_run_until", "akmc_voxel_grid",
                     "akmc_batch_priority", "akmc_batch_run_until", "akmc_patchnet_blob_bytes",
                     "akmc_patchnet_set", "akmc_patchnet_get", "akmc_patchnet_eval",
                     "akmc_policy_attach", "akmc_poisson_attach",
                     "akmc_batch_workspace_bytes", "akmc_batch_create", "akmc_batch_set_schedule",
                     "akmc_batch_step", "akmc_batch_autotune", "akmc_batch_state_read",
                     "akmc_batch_destroy"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/akmc.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:akmc_status|const char \*)\s*(akmc_\w+)\s*\(", text, re.M)))


def status_string(s: int) -> str:
    return lib().akmc_status_string(s).decode()


def last_error() -> str:
    return lib().akmc_last_error().decode()


def _check(status: int, what: str):
    if status != OK:
        raise AkmcError(status, what, last_error())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_params(spec, precision: int = FP64, refresh: int = REFRESH_LOCAL,
                time_mode: int = TIME_STOCHASTIC, barrier_model: int = BARRIER_PAIR,
                event_counter0: int = 0, time0: float = 0.0, digest0: int = 0) -> Params:
    """Params from a workloads.LatticeSpec (or any object with the same fields)."""
    p = Params()
    p.lx, p.ly, p.lz = (int(v) for v in spec.dims)
    S = int(spec.n_species)
    p.n_species = S
    e1 = np.asarray(spec.eps1, dtype=np.float64).reshape(S, S)
    e2 = np.asarray(spec.eps2, dtype=np.float64).reshape(S, S)
    for a in range(S):
        for b in range(S):
            p.eps1[a * S + b] = e1[a, b]
            p.eps2[a * S + b] = e2[a, b]
    for a, v in enumerate(np.asarray(spec.e0, dtype=np.float64)):
        p.e0[a] = v
    p.nu = float(spec.nu)
    p.temperature = float(spec.temperature)
    p.kb = float(spec.kb)
    p.seed = int(spec.seed) & (2**64 - 1)
    p.stream_id = int(spec.stream_id) & (2**64 - 1)
    p.event_counter0 = int(event_counter0)
    p.time0 = float(time0)
    p.digest0 = int(digest0) & (2**64 - 1)
    p.precision = int(precision)
    p.refresh = int(refresh)
    p.time_mode = int(time_mode)
    p.barrier_model = int(barrier_model)
    far = getattr(spec, "eps_far", None)
    p.n_shells = 2 if far is None else 6
    if far is not None:
        far = np.asarray(far, dtype=np.float64).reshape(4, S, S)
        for m in range(4):
            for a in range(S):
                for b in range(S):
                    p.eps_far[m][a * S + b] = far[m, a, b]
    return p


# ------------------------------------------------------------- C calls

def workspace_bytes(params: Params, n_vac: int) -> int:
    n = C.c_size_t()
    _check(lib().akmc_workspace_bytes(C.byref(params), int(n_vac), C.byref(n)), "workspace_bytes")
    return n.value


def lattice_create(params: Params, occ_host: np.ndarray, ws, stream=None,
                   slot_sites: Optional[np.ndarray] = None) -> int:
    occ = np.ascontiguousarray(occ_host, dtype=np.uint8)
    sl = None if slot_sites is None else np.ascontiguousarray(slot_sites, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().akmc_lattice_create(C.byref(params), occ.ctypes.data,
                                     None if sl is None else sl.ctypes.data, _ptr(ws), ws.numel(),
                                     _stream(stream), C.byref(h)), "lattice_create")
    return h.value


def rates_eval(h: int, mode: int, sites, n_sites: int, rates_out, ea_out=None):
    _check(lib().akmc_rates_eval(h, int(mode), _ptr(sites), int(n_sites), _ptr(rates_out),
                                 _ptr(ea_out)), "rates_eval")


def rates_timing(h: int, start=None, stop=None):
    """Events (torch.cuda.Event, already recorded once so that they exist)
    that every later ALL_SITES launch on h records at its kernel's start and
    end; None, None stops it."""
    def ev(e):
        return None if e is None else C.c_void_p(e.cuda_event)
    _check(lib().akmc_rates_timing(h, ev(start), ev(stop)), "rates_timing")


def kmc_step(h: int, n_events: int, log=None):
    _check(lib().akmc_kmc_step(h, int(n_events), _ptr(log)), "kmc_step")


def kmc_run_until(h: int, t_end: float, max_events: int, log=None):
    _check(lib().akmc_kmc_run_until(h, float(t_end), int(max_events), _ptr(log)), "kmc_run_until")


def voxel_grid(T: np.ndarray, e_eff: float, kb: float, tol: float):
    """(n_x, n_z, voxel temperatures [n_z*n_x], worst Eq. 9 variation) of a
    field T[nz][nx] (host call)."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    nz, nx = T.shape
    out = np.zeros(nx * nz, dtype=np.float64)
    gx, gz, worst = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().akmc_voxel_grid(T.ctypes.data, nx, nz, float(e_eff), float(kb), float(tol),
                                 C.byref(gx), C.byref(gz), out.ctypes.data, C.byref(worst)),
           "voxel_grid")
    return gx.value, gz.value, out[:gx.value * gz.value].copy(), worst.value


def patchnet_blob_bytes(S: int, H: int, n_out: int) -> int:
    n = C.c_size_t()
    _check(lib().akmc_patchnet_blob_bytes(int(S), int(H), int(n_out), C.byref(n)), "patchnet_blob_bytes")
    return n.value


def patchnet_set(blob, S: int, H: int, n_out: int, params: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().akmc_patchnet_set(_ptr(blob), int(S), int(H), int(n_out), p.ctypes.data), "patchnet_set")


def patchnet_get(blob):
    S, H, no = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().akmc_patchnet_get(_ptr(blob), C.byref(S), C.byref(H), C.byref(no), None), "patchnet_get")
    n = 64 * S.value * H.value + H.value + H.value * H.value + H.value + H.value * no.value + no.value
    out = np.zeros(n, dtype=np.float32)
    _check(lib().akmc_patchnet_get(_ptr(blob), None, None, None, out.ctypes.data), "patchnet_get")
    return S.value, H.value, no.value, out


def patchnet_eval(h: int, blob, sites, n_sites: int, out):
    _check(lib().akmc_patchnet_eval(h, _ptr(blob), _ptr(sites), int(n_sites), _ptr(out)), "patchnet_eval")


def policy_attach(h: int, blob, tau: float = 1.0):
    _check(lib().akmc_policy_attach(h, _ptr(blob), C.c_float(tau)), "policy_attach")


def poisson_attach(h: int, blob):
    _check(lib().akmc_poisson_attach(h, _ptr(blob)), "poisson_attach")


def batch_priority(b: int, w_out=None, order_out=None):
    _check(lib().akmc_batch_priority(b, _ptr(w_out), _ptr(order_out)), "batch_priority")


def batch_run_until(b: int, t_end: float, max_events_per_replica: int, order: int = ORDER_PRIORITY):
    _check(lib().akmc_batch_run_until(b, float(t_end), int(max_events_per_replica), int(order)),
           "batch_run_until")


def loop_barriers(h: int, ea_out):
    """Barriers [n_vac][8] the event loop last evaluated (device tensor of
    the handle's rate precision)."""
    _check(lib().akmc_loop_barriers(h, _ptr(ea_out)), "loop_barriers")


def state_read(h: int, occ_host: Optional[np.ndarray] = None,
               slots_host: Optional[np.ndarray] = None) -> Summary:
    s = Summary()
    _check(lib().akmc_state_read(h, None if occ_host is None else occ_host.ctypes.data,
                                 None if slots_host is None else slots_host.ctypes.data,
                                 C.byref(s)), "state_read")
    return s


def lattice_destroy(h: int):
    _check(lib().akmc_lattice_destroy(h), "lattice_destroy")


def cluster_scratch_bytes(h: int) -> int:
    out = C.c_size_t(0)
    _check(lib().akmc_cluster_scratch_bytes(h, C.byref(out)), "cluster_scratch_bytes")
    return out.value


def cluster_hist(h: int, species: int, max_size: int, hist_out, scratch, scratch_bytes: int):
    _check(lib().akmc_cluster_hist(h, int(species), int(max_size), _ptr(hist_out), _ptr(scratch),
                                   int(scratch_bytes)), "cluster_hist")


def cluster_hist_noalloc(h: int, species: int, max_size: int, hist_out):
    _check(lib().akmc_cluster_hist_noalloc(h, int(species), int(max_size), _ptr(hist_out)),
           "cluster_hist_noalloc")


def batch_workspace_bytes(params: Sequence[Params], n_vac: Sequence[int]) -> int:
    arr = (Params * len(params))(*params)
    nv = np.ascontiguousarray(n_vac, dtype=np.int32)
    n = C.c_size_t()
    _check(lib().akmc_batch_workspace_bytes(len(params), arr, nv.ctypes.data, C.byref(n)),
           "batch_workspace_bytes")
    return n.value


def batch_create(params: Sequence[Params], occs: Sequence[np.ndarray], ws, stream=None,
                 slot_sites: Optional[Sequence] = None) -> int:
    arr = (Params * len(params))(*params)
    occs = [np.ascontiguousarray(o, dtype=np.uint8) for o in occs]
    ptrs = (C.c_void_p * len(occs))(*[o.ctypes.data for o in occs])
    sptrs = None
    if slot_sites is not None:
        sl = [None if x is None else np.ascontiguousarray(x, dtype=np.int32) for x in slot_sites]
        sptrs = (C.c_void_p * len(sl))(*[None if x is None else x.ctypes.data for x in sl])
    b = C.c_void_p()
    _check(lib().akmc_batch_create(len(params), arr, ptrs, sptrs, _ptr(ws), ws.numel(),
                                   _stream(stream), C.byref(b)), "batch_create")
    return b.value


def batch_set_schedule(b: int, sched: Schedule):
    _check(lib().akmc_batch_set_schedule(b, C.byref(sched)), "batch_set_schedule")


def batch_step(b: int, n_events_per_replica: int):
    _check(lib().akmc_batch_step(b, int(n_events_per_replica)), "batch_step")


def batch_autotune(b: int, trial_events: int) -> Schedule:
    s = Schedule()
    _check(lib().akmc_batch_autotune(b, int(trial_events), C.byref(s)), "batch_autotune")
    return s


def batch_state_read(b: int, r: int, occ_host: Optional[np.ndarray] = None,
                     slots_host: Optional[np.ndarray] = None) -> Summary:
    s = Summary()
    _check(lib().akmc_batch_state_read(b, int(r), None if occ_host is None else occ_host.ctypes.data,
                                       None if slots_host is None else slots_host.ctypes.data,
                                       C.byref(s)), "batch_state_read")
    return s


def batch_destroy(b: int):
    _check(lib().akmc_batch_destroy(b), "batch_destroy")


def mlp_blob_bytes(S: int) -> int:
    n = C.c_size_t()
    _check(lib().akmc_mlp_blob_bytes(int(S), C.byref(n)), "mlp_blob_bytes")
    return n.value


def mlp_param_count(S: int) -> int:
    n = C.c_int32()
    _check(lib().akmc_mlp_param_count(int(S), C.byref(n)), "mlp_param_count")
    return n.value


def mlp_init(blob, S: int, seed: int, mu: float, sigma: float, stream=None):
    _check(lib().akmc_mlp_init(_ptr(blob), int(S), int(seed), float(mu), float(sigma), _stream(stream)),
           "mlp_init")


def mlp_set_params(blob, S: int, params: np.ndarray, mu: float, sigma: float, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().akmc_mlp_set_params(_ptr(blob), int(S), p.ctypes.data, float(mu), float(sigma),
                                     _stream(stream)), "mlp_set_params")


def mlp_get_params(blob, S: int, stream=None):
    p = np.empty(mlp_param_count(S), dtype=np.float32)
    mu, sg = C.c_float(), C.c_float()
    _check(lib().akmc_mlp_get_params(_ptr(blob), int(S), p.ctypes.data, C.byref(mu), C.byref(sg),
                                     _stream(stream)), "mlp_get_params")
    return p, mu.value, sg.value


def env_encode(h: int, mode: int, sites, n_sites: int, env_out, ea_out=None):
    _check(lib().akmc_env_encode(h, int(mode), _ptr(sites), int(n_sites), _ptr(env_out), _ptr(ea_out)),
           "env_encode")


def mlp_fit_ood(blob, S: int, env, n: int, stream=None):
    _check(lib().akmc_mlp_fit_ood(_ptr(blob), int(S), _ptr(env), int(n), _stream(stream)), "mlp_fit_ood")


def mlp_forward(blob, S: int, env, n: int, ea_out, stream=None):
    _check(lib().akmc_mlp_forward(_ptr(blob), int(S), _ptr(env), int(n), _ptr(ea_out), _stream(stream)),
           "mlp_forward")


def mlp_train_workspace_bytes(S: int, batch: int) -> int:
    n = C.c_size_t()
    _check(lib().akmc_mlp_train_workspace_bytes(int(S), int(batch), C.byref(n)), "mlp_train_workspace_bytes")
    return n.value


def mlp_train(blob, S: int, env, ea, n: int, cfg: TrainCfg, work, loss=None, stream=None):
    _check(lib().akmc_mlp_train(_ptr(blob), int(S), _ptr(env), _ptr(ea), int(n), C.byref(cfg),
                                _ptr(loss), _ptr(work), work.numel(), _stream(stream)), "mlp_train")


def mlp_grad(blob, S: int, env, ea, n: int, grad_out, work, loss=None, stream=None):
    _check(lib().akmc_mlp_grad(_ptr(blob), int(S), _ptr(env), _ptr(ea), int(n), _ptr(grad_out),
                               _ptr(loss), _ptr(work), work.numel(), _stream(stream)), "mlp_grad")


def mlp_attach(h: int, blob):
    _check(lib().akmc_mlp_attach(h, _ptr(blob)), "mlp_attach")


def pack_params(p: dict) -> np.ndarray:
    """Flat binary32 parameter vector in the library's order from a dict with
    W1 (K1 x 128), b1, W2 (128 x 128), b2, w3, b3."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "w3", "b3")]).astype(np.float32)


def unpack_params(v: np.ndarray, S: int) -> dict:
    k1 = 32 * ((27 * S + 31) // 32)
    H = 128
    out, o = {}, 0
    for k, shape in (("W1", (k1, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


# ------------------------------------------------------ conveniences

class Lattice:
    """One lattice on the current ROCm device (workspace owned by torch)."""

    def __init__(self, spec, device="cuda", stream=None, slot_sites=None, **kw):
        import torch
        self.spec = spec
        self.params = make_params(spec, **kw)
        self.n_vac = int(np.count_nonzero(spec.occ == spec.n_species - 1))
        nbytes = workspace_bytes(self.params, self.n_vac)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.h = lattice_create(self.params, spec.occ, self.ws, stream, slot_sites)
        self.n_sites = spec.n_sites

    def close(self):
        if getattr(self, "h", None):
            lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rate_dtype(self):
        import torch
        return torch.float32 if self.params.precision == FP32 else torch.float64

    def rates(self, mode=RATES_VACANCIES, sites=None, with_ea=False):
        import torch
        dev = self.ws.device
        if mode == RATES_VACANCIES:
            n = self.n_vac
        elif mode == RATES_ALL_SITES:
            n = self.n_sites
        else:
            sites = torch.as_tensor(np.asarray(sites, dtype=np.int32), device=dev)
            n = sites.numel()
        out = torch.empty((n, 8), dtype=self.rate_dtype(), device=dev)
        ea = torch.empty_like(out) if with_ea else None
        rates_eval(self.h, mode, sites, n, out, ea)
        return (out, ea) if with_ea else out

    def barriers(self):
        """Device [n_vac][8] barriers the event loop last evaluated."""
        import torch
        out = torch.empty((max(self.n_vac, 1), 8), dtype=self.rate_dtype(), device=self.ws.device)
        loop_barriers(self.h, out)
        return out[:self.n_vac]

    def step(self, n_events: int, log: bool = False):
        import torch
        buf = None
        if log:
            buf = torch.empty((max(n_events, 1), 40), dtype=torch.uint8, device=self.ws.device)
        kmc_step(self.h, n_events, buf)
        return buf

    def run_until(self, t_end: float, max_events: int, log: bool = False):
        import torch
        buf = None
        if log:
            buf = torch.empty((max(max_events, 1), 40), dtype=torch.uint8, device=self.ws.device)
        kmc_run_until(self.h, t_end, max_events, buf)
        return buf

    def clusters(self, species: int = 1, max_size: int = 64):
        """Device int64[max_size + 1] cluster-size histogram of `species`."""
        import torch
        dev = self.ws.device
        nb = cluster_scratch_bytes(self.h)
        # Kept with the lattice: the launch is asynchronous on its stream.
        if getattr(self, "_cc_scratch", None) is None:
            self._cc_scratch = torch.empty(nb, dtype=torch.uint8, device=dev)
        hist = torch.empty(max_size + 1, dtype=torch.int64, device=dev)
        cluster_hist(self.h, species, max_size, hist, self._cc_scratch, nb)
        return hist

    def read(self):
        occ = np.empty(self.n_sites, dtype=np.uint8)
        slots = np.empty(max(self.n_vac, 1), dtype=np.int32)
        s = state_read(self.h, occ, slots)
        return occ, slots[:self.n_vac], s


class PatchNetBlob:
    """A local patch network in device memory (akmc_patchnet_set layout):
    policy (n_out = 8) or Poisson network (n_out = 1)."""

    def __init__(self, S: int, H: int, n_out: int, device="cuda"):
        import torch
        self.S, self.H, self.n_out = int(S), int(H), int(n_out)
        self.blob = torch.zeros(patchnet_blob_bytes(S, H, n_out), dtype=torch.uint8, device=device)

    def set(self, w1, b1, w2, b2, w3, b3):
        """w1 [64][S][H], b1 [H], w2 [H][H], b2 [H], w3 [H][n_out], b3 [n_out]."""
        flat = np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in (w1, b1, w2, b2, w3, b3)])
        patchnet_set(self.blob, self.S, self.H, self.n_out, flat)

    def get(self):
        """The stored (bfloat16-rounded) parameters as the six arrays."""
        S, H, no, v = patchnet_get(self.blob)
        out, o = [], 0
        for shape in ((64, S, H), (H,), (H, H), (H,), (H, no), (no,)):
            n = int(np.prod(shape))
            out.append(v[o:o + n].reshape(shape).copy())
            o += n
        return out


def log_to_numpy(buf, n: int) -> np.ndarray:
    """Device event-log buffer (uint8 [n, 40]) to a structured numpy array."""
    raw = buf[:n].cpu().numpy().reshape(-1)
    return raw.view(EVENT_DTYPE).copy()

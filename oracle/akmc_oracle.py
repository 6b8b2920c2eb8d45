"""ctypes wrapper around the C oracle (akmc_oracle.c).

TEST INFRASTRUCTURE (see oracle/__init__.py).  Inputs come from
paper_2604_24091_amd.workloads.LatticeSpec objects or plain numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None


class OrcParams(C.Structure):
    _fields_ = [("lx", C.c_int32), ("ly", C.c_int32), ("lz", C.c_int32),
                ("n_species", C.c_int32),
                ("eps1", C.c_double * 64), ("eps2", C.c_double * 64),
                ("e0", C.c_double * 8),
                ("nu", C.c_double), ("temperature", C.c_double), ("kb", C.c_double),
                ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("precision", C.c_int32), ("time_mode", C.c_int32),
                ("n_shells", C.c_int32), ("pad_", C.c_int32), ("epsx", (C.c_double * 64) * 4)]


class OrcEvent(C.Structure):
    _fields_ = [("n", C.c_int64), ("slot", C.c_int32), ("from_site", C.c_int32),
                ("to_site", C.c_int32), ("dir", C.c_uint8), ("species", C.c_uint8),
                ("pad", C.c_uint8 * 2), ("gamma_tot", C.c_double), ("dt", C.c_double)]


class OrcState(C.Structure):
    _fields_ = [("n", C.c_int64), ("t", C.c_double), ("digest", C.c_uint64),
                ("gamma_tot", C.c_double), ("n_neg_evaluated", C.c_int64)]


class OrcPatchNet(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("hidden", C.c_int32), ("n_out", C.c_int32),
                ("pad_", C.c_int32),
                ("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p),
                ("b2", C.c_void_p), ("w3", C.c_void_p), ("b3", C.c_void_p)]


class PatchNet:
    """Weights of a local patch network (policy: n_out = 8; Poisson
    network: n_out = 1) as binary32 arrays: w1 [64][S][H], b1 [H],
    w2 [H][H], b2 [H], w3 [H][n_out], b3 [n_out]."""

    def __init__(self, w1, b1, w2, b2, w3, b3):
        self.w1 = np.ascontiguousarray(w1, dtype=np.float32)
        self.b1 = np.ascontiguousarray(b1, dtype=np.float32)
        self.w2 = np.ascontiguousarray(w2, dtype=np.float32)
        self.b2 = np.ascontiguousarray(b2, dtype=np.float32)
        self.w3 = np.ascontiguousarray(w3, dtype=np.float32)
        self.b3 = np.ascontiguousarray(b3, dtype=np.float32)
        self.S = self.w1.shape[1]
        self.H = self.w1.shape[2]
        self.n_out = self.w3.shape[1]
        assert self.w1.shape[0] == 64 and self.w2.shape == (self.H, self.H)
        assert self.b1.shape == (self.H,) and self.b2.shape == (self.H,)
        assert self.w3.shape[0] == self.H and self.b3.shape == (self.n_out,)
        self.c = OrcPatchNet(self.S, self.H, self.n_out, 0,
                             *(a.ctypes.data for a in (self.w1, self.b1, self.w2, self.b2,
                                                       self.w3, self.b3)))


EVENT_DTYPE = np.dtype([("n", "<i8"), ("slot", "<i4"), ("from_site", "<i4"),
                        ("to_site", "<i4"), ("dir", "u1"), ("species", "u1"),
                        ("pad", "u1", (2,)), ("gamma_tot", "<f8"), ("dt", "<f8")])
assert EVENT_DTYPE.itemsize == C.sizeof(OrcEvent) == 40

FNV_OFFSET = 0xCBF29CE484222325

_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        P = C.POINTER(OrcParams)
        L.orc_site.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_site.restype = C.c_int32
        L.orc_nbr1.argtypes = [P, C.c_int32, C.c_int]
        L.orc_nbr1.restype = C.c_int32
        L.orc_nbr2.argtypes = [P, C.c_int32, C.c_int]
        L.orc_nbr2.restype = C.c_int32
        L.orc_delta_e.argtypes = [P, _u8p, C.c_int32, C.c_int]
        L.orc_delta_e.restype = C.c_double
        L.orc_candidate.argtypes = [P, _u8p, C.c_int32, C.c_int,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_candidate.restype = None
        L.orc_rates_sites.argtypes = [P, _u8p, _i32p, C.c_int64, _f64p, C.c_void_p]
        L.orc_rates_sites.restype = None
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_philox4x64_10.restype = None
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_int64,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_uniforms.restype = None
        L.orc_fnv1a.argtypes = [C.c_uint64, _u8p, C.c_int64]
        L.orc_fnv1a.restype = C.c_uint64
        L.orc_digest_event.argtypes = [C.c_uint64, C.c_int32, C.c_int32]
        L.orc_digest_event.restype = C.c_uint64
        L.orc_select.argtypes = [_f64p, C.c_int64, C.c_double, C.POINTER(C.c_double)]
        L.orc_select.restype = C.c_int64
        L.orc_gamma_tot.argtypes = [P, _u8p, _i32p, C.c_int32]
        L.orc_gamma_tot.restype = C.c_double
        L.orc_run.argtypes = [P, _u8p, _i32p, C.c_int32, C.POINTER(OrcState),
                              C.c_int64, C.c_void_p]
        L.orc_run.restype = C.c_int64
        L.orc_run_local.argtypes = L.orc_run.argtypes
        L.orc_run_local.restype = C.c_int64
        L.orc_run_until.argtypes = [P, _u8p, _i32p, C.c_int32, C.POINTER(OrcState),
                                    C.c_double, C.c_int64, C.c_void_p]
        L.orc_run_until.restype = C.c_int64
        L.orc_follow.argtypes = [P, _u8p, _i32p, C.c_int32, C.POINTER(OrcState),
                                 C.c_int64, C.c_void_p, _f64p]
        L.orc_follow.restype = None
        L.orc_cluster_hist.argtypes = [P, _u8p, C.c_int, _i64p, C.c_int64]
        L.orc_cluster_hist.restype = C.c_int64
        L.orc_encode_env.argtypes = [P, _u8p, C.c_int32, C.c_int, _u8p]
        L.orc_encode_env.restype = None
        L.orc_encode_env_sites.argtypes = [P, _u8p, _i32p, C.c_int64, _u8p]
        L.orc_encode_env_sites.restype = None
        L.orc_barrier_counts.argtypes = [P, _u8p, _i32p, C.c_int32, _i64p]
        L.orc_barrier_counts.restype = None
        NP = C.POINTER(OrcPatchNet)
        L.orc_obs_offset.argtypes = [C.c_int, _i32p]
        L.orc_obs_offset.restype = None
        L.orc_observation.argtypes = [P, _u8p, C.c_int32, _u8p]
        L.orc_observation.restype = None
        L.orc_patchnet_forward.argtypes = [NP, _u8p, np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")]
        L.orc_patchnet_forward.restype = None
        L.orc_policy_weights.argtypes = [P, _u8p, C.c_int32, NP, C.c_float, _f64p,
                                         np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")]
        L.orc_policy_weights.restype = None
        L.orc_poisson_u.argtypes = [P, _u8p, _i32p, C.c_int32, NP]
        L.orc_poisson_u.restype = C.c_double
        L.orc_poisson_dt.argtypes = [C.c_double] * 4
        L.orc_poisson_dt.restype = C.c_double
        L.orc_run_learned.argtypes = [P, _u8p, _i32p, C.c_int32, C.POINTER(OrcState), C.c_int64,
                                      C.c_void_p, C.c_void_p, C.c_float, C.c_void_p]
        L.orc_run_learned.restype = C.c_int64
        L.orc_follow_learned.argtypes = [P, _u8p, _i32p, C.c_int32, C.POINTER(OrcState), C.c_int64,
                                         C.c_void_p, C.c_void_p, C.c_float, C.c_void_p, _f64p]
        L.orc_follow_learned.restype = None
        _lib = L
    return _lib


def make_params(spec, precision: int = 0, time_mode: int = 0,
                temperature: Optional[float] = None) -> OrcParams:
    p = OrcParams()
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
    p.temperature = float(spec.temperature if temperature is None else temperature)
    p.kb = float(spec.kb)
    p.seed = int(spec.seed) & (2**64 - 1)
    p.stream_id = int(spec.stream_id) & (2**64 - 1)
    p.precision = int(precision)
    p.time_mode = int(time_mode)
    # the pair model out to 6.0 A: shells 3..6 from spec.eps_far [4][S][S]
    far = getattr(spec, "eps_far", None)
    p.n_shells = 2 if far is None else 6
    if far is not None:
        far = np.asarray(far, dtype=np.float64).reshape(4, S, S)
        for m in range(4):
            for a in range(S):
                for b in range(S):
                    p.epsx[m][a * S + b] = far[m, a, b]
    return p


class Oracle:
    """One lattice state advanced by the plain full-recompute AKMC loop."""

    def __init__(self, spec, precision: int = 0, time_mode: int = 0):
        self.spec = spec
        self.p = make_params(spec, precision, time_mode)
        self.occ = np.ascontiguousarray(spec.occ, dtype=np.uint8).copy()
        self.slots = np.flatnonzero(self.occ == spec.n_species - 1).astype(np.int32)
        self.state = OrcState(0, 0.0, FNV_OFFSET, 0.0, 0)

    # geometry --------------------------------------------------------------
    def nbr1(self, site: int, k: int) -> int:
        return lib().orc_nbr1(C.byref(self.p), site, k)

    def nbr2(self, site: int, m: int) -> int:
        return lib().orc_nbr2(C.byref(self.p), site, m)

    # rates -----------------------------------------------------------------
    def delta_e(self, i: int, k: int, occ=None) -> float:
        occ = self.occ if occ is None else occ
        return lib().orc_delta_e(C.byref(self.p), occ, int(i), int(k))

    def rates_sites(self, sites, occ=None):
        occ = self.occ if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        n = sites.size
        rates = np.zeros((n, 8), dtype=np.float64)
        ea = np.zeros((n, 8), dtype=np.float64)
        lib().orc_rates_sites(C.byref(self.p), occ, sites, n, rates,
                              ea.ctypes.data_as(C.c_void_p))
        return rates, ea

    def rates_vacancies(self):
        return self.rates_sites(self.slots)

    def gamma_tot(self) -> float:
        return lib().orc_gamma_tot(C.byref(self.p), self.occ, self.slots, self.slots.size)

    # events ----------------------------------------------------------------
    def run(self, n_events: int, log: bool = False, local: bool = False):
        """n_events events; local=True refreshes after each jump only the
        slots within reach of the exchanged sites (same trajectory)."""
        buf = np.zeros(max(n_events, 1), dtype=EVENT_DTYPE) if log else None
        fn = lib().orc_run_local if local else lib().orc_run
        done = fn(C.byref(self.p), self.occ, self.slots, self.slots.size,
                  C.byref(self.state), int(n_events),
                  buf.ctypes.data_as(C.c_void_p) if log else None)
        if log:
            return done, buf[:max(done, 0)]
        return done

    def run_until(self, t_end: float, max_events: int, log: bool = False):
        """Events while t < t_end, at most max_events (the last event is the
        one that reaches t_end)."""
        buf = np.zeros(max(max_events, 1), dtype=EVENT_DTYPE) if log else None
        done = lib().orc_run_until(C.byref(self.p), self.occ, self.slots, self.slots.size,
                                   C.byref(self.state), C.c_double(t_end), int(max_events),
                                   buf.ctypes.data_as(C.c_void_p) if log else None)
        if log:
            return done, buf[:max(done, 0)]
        return done

    def observation(self, i: int, occ=None):
        occ = self.occ if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        out = np.zeros(64, dtype=np.uint8)
        lib().orc_observation(C.byref(self.p), occ, int(i), out)
        return out

    def policy_weights(self, pol: "PatchNet", inv_tau: float, occ=None):
        """[n_vac][8] selection weights exp(z_hat) and logits of the current
        slots (weight 0 for an inadmissible jump)."""
        occ = self.occ if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        nv = self.slots.size
        w = np.zeros((nv, 8), dtype=np.float64)
        z = np.zeros((nv, 8), dtype=np.float32)
        for v in range(nv):
            wv = np.zeros(8, dtype=np.float64)
            zv = np.zeros(8, dtype=np.float32)
            lib().orc_policy_weights(C.byref(self.p), occ, int(self.slots[v]), C.byref(pol.c),
                                     C.c_float(inv_tau), wv, zv)
            w[v], z[v] = wv, zv
        return w, z

    def poisson_u(self, pn: "PatchNet") -> float:
        return lib().orc_poisson_u(C.byref(self.p), self.occ, self.slots, self.slots.size,
                                   C.byref(pn.c))

    def run_learned(self, n_events: int, pol: Optional["PatchNet"] = None, inv_tau: float = 1.0,
                    pn: Optional["PatchNet"] = None, log: bool = False):
        """Events chosen by the policy (or by the rates without one), time by
        Eq. 7 with a Poisson network (or by time_mode without one)."""
        buf = np.zeros(max(n_events, 1), dtype=EVENT_DTYPE) if log else None
        done = lib().orc_run_learned(C.byref(self.p), self.occ, self.slots, self.slots.size,
                                     C.byref(self.state), int(n_events),
                                     buf.ctypes.data_as(C.c_void_p) if log else None,
                                     C.cast(C.byref(pol.c), C.c_void_p) if pol else None,
                                     C.c_float(inv_tau),
                                     C.cast(C.byref(pn.c), C.c_void_p) if pn else None)
        if log:
            return done, buf[:max(done, 0)]
        return done

    def follow_learned(self, log_records, pol: Optional["PatchNet"] = None, inv_tau: float = 1.0,
                       pn: Optional["PatchNet"] = None):
        recs = np.ascontiguousarray(log_records, dtype=EVENT_DTYPE)
        out = np.zeros(5, dtype=np.float64)
        lib().orc_follow_learned(C.byref(self.p), self.occ, self.slots, self.slots.size,
                                 C.byref(self.state), recs.size, recs.ctypes.data_as(C.c_void_p),
                                 C.cast(C.byref(pol.c), C.c_void_p) if pol else None,
                                 C.c_float(inv_tau),
                                 C.cast(C.byref(pn.c), C.c_void_p) if pn else None, out)
        return {"max_select_violation": out[0], "max_gamma_rel": out[1],
                "max_dt_rel": out[2], "mismatches": int(out[3]), "n_differ": int(out[4])}

    def follow(self, log_records):
        recs = np.ascontiguousarray(log_records, dtype=EVENT_DTYPE)
        out = np.zeros(5, dtype=np.float64)
        lib().orc_follow(C.byref(self.p), self.occ, self.slots, self.slots.size,
                         C.byref(self.state), recs.size,
                         recs.ctypes.data_as(C.c_void_p), out)
        return {"max_select_violation": out[0], "max_gamma_rel": out[1],
                "max_dt_rel": out[2], "mismatches": int(out[3]), "n_differ": int(out[4])}

    def cluster_hist(self, species: int = 1, max_size: int = 64, occ=None):
        occ = self.occ if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        hist = np.zeros(max_size + 1, dtype=np.int64)
        n = lib().orc_cluster_hist(C.byref(self.p), occ, int(species), hist, max_size)
        return n, hist

    def encode_env(self, i: int, k: int, occ=None):
        occ = self.occ if occ is None else occ
        out = np.zeros(27, dtype=np.uint8)
        lib().orc_encode_env(C.byref(self.p), occ, int(i), int(k), out)
        return out

    def encode_env_sites(self, sites, occ=None):
        """Slot codes of the 8 candidates of every listed site: [n][8][27]."""
        occ = self.occ if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        out = np.zeros((sites.size, 8, 27), dtype=np.uint8)
        lib().orc_encode_env_sites(C.byref(self.p), occ, sites, sites.size, out)
        return out

    def barrier_counts(self):
        """(candidates with Ea < 0, candidates with Ea < dE) of the current
        slots, admissible jumps only."""
        out = np.zeros(2, dtype=np.int64)
        lib().orc_barrier_counts(C.byref(self.p), self.occ, self.slots, self.slots.size, out)
        return int(out[0]), int(out[1])


def patchnet_forward(net: PatchNet, codes) -> np.ndarray:
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    out = np.zeros(net.n_out, dtype=np.float32)
    lib().orc_patchnet_forward(C.byref(net.c), c, out)
    return out


def obs_offsets() -> np.ndarray:
    out = np.zeros((64, 3), dtype=np.int32)
    for m in range(64):
        o = np.zeros(3, dtype=np.int32)
        lib().orc_obs_offset(m, o)
        out[m] = o
    return out


def poisson_dt(u_s: float, g_s: float, u_s1: float, g_s1: float) -> float:
    return lib().orc_poisson_dt(u_s, g_s, u_s1, g_s1)


def philox(counter, key):
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(ctr, k, out)
    return out


def uniforms(seed: int, stream_id: int, n: int):
    u1, u2 = C.c_double(), C.c_double()
    lib().orc_uniforms(seed, stream_id, n, C.byref(u1), C.byref(u2))
    return u1.value, u2.value


def fnv1a(data: bytes, h: int = FNV_OFFSET) -> int:
    arr = np.frombuffer(bytes(data), dtype=np.uint8).copy() if data else np.zeros(1, np.uint8)
    return lib().orc_fnv1a(h, arr, len(data))


def digest_event(h: int, from_site: int, to_site: int) -> int:
    """One event of the trajectory digest (orc_digest_event)."""
    return lib().orc_digest_event(h, int(from_site), int(to_site))


def select(rates, u1: float):
    r = np.ascontiguousarray(rates, dtype=np.float64)
    g = C.c_double()
    c = lib().orc_select(r, r.size, float(u1), C.byref(g))
    return c, g.value

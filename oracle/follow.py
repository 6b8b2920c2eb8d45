"""Plain replay of an event log against barriers from any barrier model.

TEST INFRASTRUCTURE: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.

The C oracle's follow mode replays a log against the pair model's rates.
This module does the same for a barrier model given as a Python function
(the learned barrier with its pair-model fallback, for instance), in
binary64, with every rate recomputed before every event:
  rate        r = nu * exp(-(Ea / kT)) (Eq. 8); an inadmissible jump
              (Ea = +inf, the feasibility mask of Eq. 1) has r = +0;
  selection   the candidates compete system-wide (Eq. 2 with logits ln r):
              candidate c is a valid choice for the uniform u1 when
              C_{c-1} <= u1 * Gamma_tot < C_c, with C the running sums
              over c = 8*slot + k, left to right;
  time        dt = -ln(u2) / Gamma_tot (mean 1/Gamma_tot, Eq. 5), or
              1/Gamma_tot in mean-time mode.
Every recorded event is checked against these quantities of the state it
was taken from, then its swap is applied.
"""
from __future__ import annotations

import math

import numpy as np

from . import akmc_oracle as O


class Follower:
    """A lattice state that replays event logs.

    barriers(occ, slots) -> float64 [nv][8] barriers of the current
    candidates (+inf for an inadmissible jump)."""

    def __init__(self, spec, barriers, time_mode: int = 0):
        self.spec = spec
        self.barriers = barriers
        self.time_mode = int(time_mode)
        self.occ = np.ascontiguousarray(spec.occ, dtype=np.uint8).copy()
        self.slots = np.flatnonzero(self.occ == spec.n_species - 1).astype(np.int32)
        self.n = 0
        self.t = 0.0
        self.digest = O.FNV_OFFSET
        self.kt = float(spec.kb) * float(spec.temperature)
        self.geo = O.Oracle(spec)      # neighbour geometry and uniforms only

    def rates(self):
        ea = np.asarray(self.barriers(self.occ, self.slots), dtype=np.float64).reshape(-1)
        r = np.zeros_like(ea)
        ok = np.isfinite(ea)
        r[ok] = float(self.spec.nu) * np.exp(-(ea[ok] / self.kt))
        return r, ea

    def follow(self, log):
        """Replays `log` (EVENT_DTYPE records) from the current state.
        Returns the largest selection-interval violation relative to
        Gamma_tot, the largest relative differences of the recorded
        Gamma_tot and dt, the number of structural mismatches (then the
        replay stops) and the number of choices outside their exact
        interval."""
        out = {"max_select_violation": 0.0, "max_gamma_rel": 0.0, "max_dt_rel": 0.0,
               "mismatches": 0, "n_differ": 0, "events": 0}
        V = self.spec.n_species - 1
        for ev in np.asarray(log):
            r, _ = self.rates()
            g = 0.0
            for x in r:               # left to right
                g += x
            u1, u2 = O.uniforms(self.spec.seed, self.spec.stream_id, self.n)
            c = int(ev["slot"]) * 8 + int(ev["dir"])
            ok = int(ev["n"]) == self.n and 0 <= int(ev["slot"]) < self.slots.size and int(ev["dir"]) < 8
            if ok:
                before = 0.0
                for x in r[:c]:
                    before += x
                after = before + r[c]
                target = u1 * g
                viol = max(0.0, before - target, target - after)
                out["max_select_violation"] = max(out["max_select_violation"], viol / g)
                out["n_differ"] += int(viol > 0.0)
                ok = r[c] > 0.0
                dt = 1.0 / g if self.time_mode == 1 else -math.log(u2) / g
                out["max_gamma_rel"] = max(out["max_gamma_rel"], abs(float(ev["gamma_tot"]) - g) / g)
                out["max_dt_rel"] = max(out["max_dt_rel"], abs(float(ev["dt"]) - dt) / dt)
                i = int(self.slots[ev["slot"]])
                j = self.geo.nbr1(i, int(ev["dir"]))
                ok = ok and int(ev["from_site"]) == i and int(ev["to_site"]) == j and \
                    int(ev["species"]) == int(self.occ[j])
            if not ok:
                out["mismatches"] += 1
                break
            self.occ[i] = self.occ[j]
            self.occ[j] = V
            self.slots[ev["slot"]] = j
            self.digest = O.digest_event(self.digest, i, j)
            self.t += dt
            self.n += 1
            out["events"] += 1
        return out

"""Seeded synthetic inputs for the vacancy-jump AKMC path.

This module only draws inputs: occupancies, pair-energy tables, barrier
offsets, temperatures and replica shapes.  It holds none of the method's
arithmetic (no energies, barriers, rates, sums or selection), so both the
HIP library and the CPU oracle can be fed from it without sharing code.

Workload shapes follow the alloy systems the paper studies: Fe-based BCC
RPV steels with Cu, Ni and Mn solutes (Sec. IV-B, the A508-3 composition)
at service temperatures around 285-304 C (Sec. I), with a point-defect
(vacancy) population in the appm range used for training (Sec. IV-C).
The paper's own ab initio energy landscape and validation data are not
available; the pair energies here are seeded uniform draws that stand in
for them (same shapes, same species set).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

# Species codes.  The last code of a system is always the vacancy.
FE, CU, NI, MN = 0, 1, 2, 3

KB_EV_PER_K = 8.617333262e-5  # CODATA 2018 Boltzmann constant in eV/K


@dataclasses.dataclass
class LatticeSpec:
    """One periodic BCC lattice and its energy model (host-side inputs)."""

    dims: tuple                 # (lx, ly, lz) cubic cells
    n_species: int              # S, vacancy code = S - 1
    eps1: np.ndarray            # (S, S) symmetric 1NN pair energies, eV
    eps2: np.ndarray            # (S, S) symmetric 2NN pair energies, eV
    e0: np.ndarray              # (S - 1,) barrier offsets per migrating species, eV
    nu: float                   # attempt frequency, Hz
    temperature: float          # K
    occ: np.ndarray             # uint8[2 * lx * ly * lz], sublattice-major
    seed: int = 0               # Philox key word 0
    stream_id: int = 0          # Philox key word 1
    kb: float = KB_EV_PER_K
    # Pair model out to 6.0 A: (4, S, S) symmetric energies of shells 3..6
    # (None: first and second neighbours only)
    eps_far: Optional[np.ndarray] = None

    @property
    def n_sites(self) -> int:
        lx, ly, lz = self.dims
        return 2 * lx * ly * lz

    @property
    def vacancy(self) -> int:
        return self.n_species - 1

    def vacancy_sites(self) -> np.ndarray:
        return np.flatnonzero(self.occ == self.vacancy).astype(np.int32)


def pair_tables(rng: np.random.Generator, n_species: int, lo: float = -0.80,
                hi: float = -0.40):
    """Symmetric 1NN and 2NN pair tables, one uniform draw per unordered pair
    (vacancy pairs included)."""
    out = []
    for _shell in range(2):
        t = np.zeros((n_species, n_species), dtype=np.float64)
        for a in range(n_species):
            for b in range(a, n_species):
                v = rng.uniform(lo, hi)
                t[a, b] = v
                t[b, a] = v
        out.append(t)
    return out[0], out[1]


def occupancy(rng: np.random.Generator, dims: Sequence[int], n_species: int,
              solute_fractions: dict, n_vac: int) -> np.ndarray:
    """Random solid solution with exact counts.

    Species s (a solute) gets floor(x_s * N + 0.5) sites, the vacancy code
    gets n_vac sites, species 0 (Fe) fills the rest; positions come from one
    seeded permutation of all N sites.
    """
    lx, ly, lz = dims
    n = 2 * lx * ly * lz
    counts = np.zeros(n_species, dtype=np.int64)
    for s, x in solute_fractions.items():
        counts[s] = int(np.floor(x * n + 0.5))
    counts[n_species - 1] = n_vac
    counts[0] = n - counts[1:].sum()
    if counts[0] < 0:
        raise ValueError("solute + vacancy counts exceed the lattice")
    labels = np.repeat(np.arange(n_species, dtype=np.uint8), counts)
    perm = rng.permutation(n)
    occ = np.empty(n, dtype=np.uint8)
    occ[perm] = labels
    return occ


# ---------------------------------------------------------------------------
# The five workloads.  Each is named by what it is and its sizes.
# ---------------------------------------------------------------------------

def fe_cu_2k(seed: int = 1000) -> LatticeSpec:
    """Fe-1.0Cu, 10^3 BCC cells (2,000 sites), one vacancy, 3 species."""
    rng = np.random.default_rng(seed)
    eps1, eps2 = pair_tables(rng, 3)
    occ = occupancy(rng, (10, 10, 10), 3, {CU: 0.010}, 1)
    return LatticeSpec(dims=(10, 10, 10), n_species=3, eps1=eps1, eps2=eps2,
                       e0=np.array([0.62, 0.53]), nu=6.0e12, temperature=563.0,
                       occ=occ, seed=seed, stream_id=0)


def _rpv_alloy_model(rng: np.random.Generator):
    eps1, eps2 = pair_tables(rng, 5)
    e0 = rng.uniform(0.50, 0.70, size=4)
    return eps1, eps2, e0


RPV_FRACTIONS = {CU: 0.0134, NI: 0.0070, MN: 0.0140}


def rpv_alloy(cells: int, n_vac: int, seed: int) -> LatticeSpec:
    """Fe-1.34Cu-0.70Ni-1.40Mn random solid solution, cells^3 BCC cells."""
    rng = np.random.default_rng(seed)
    eps1, eps2, e0 = _rpv_alloy_model(rng)
    occ = occupancy(rng, (cells, cells, cells), 5, RPV_FRACTIONS, n_vac)
    return LatticeSpec(dims=(cells, cells, cells), n_species=5, eps1=eps1,
                       eps2=eps2, e0=e0, nu=6.0e12, temperature=563.0, occ=occ,
                       seed=seed, stream_id=0)


def far_tables(rng: np.random.Generator, n_species: int, scale=(0.10, 0.06, 0.04, 0.03)) -> np.ndarray:
    """Symmetric pair energies of shells 3..6 (eV), i.i.d. U[-c, c] per
    unordered pair with c shrinking with distance: a stand-in for a
    longer-ranged landscape (vacancy rows included)."""
    out = np.zeros((4, n_species, n_species))
    for m, c in enumerate(scale):
        for a in range(n_species):
            for b in range(a, n_species):
                out[m, a, b] = out[m, b, a] = rng.uniform(-c, c)
    return out


def rpv_alloy_far(cells: int, n_vac: int, seed: int) -> LatticeSpec:
    """The Fe-1.34Cu-0.70Ni-1.40Mn solid solution with the pair model out to
    6.0 A (shells 1-6, the 64-neighbour range of Sec. IV-C)."""
    spec = rpv_alloy(cells, n_vac, seed)
    spec.eps_far = far_tables(np.random.default_rng(seed + 7919), 5)
    return spec


def rpv_4m_far(seed: int = 1005) -> LatticeSpec:
    """128^3 cells, 200 vacancies, pairs out to 6.0 A."""
    return rpv_alloy_far(128, 200, seed)


def rpv_524k(seed: int = 1001) -> LatticeSpec:
    """64^3 cells (524,288 sites), 10 vacancies."""
    return rpv_alloy(64, 10, seed)


def rpv_4m(seed: int = 1002) -> LatticeSpec:
    """128^3 cells (4,194,304 sites), 200 vacancies."""
    return rpv_alloy(128, 200, seed)


def rpv_replicas(n_rep: int = 256, seed: int = 1003,
                 cells_range=(16, 48), max_vac: int = 20) -> List[LatticeSpec]:
    """Independent replicas of uneven size (a voxel ensemble).

    Each replica draws its own edge length in cells_range (inclusive), Cu in
    [0.5, 2.0] at%, Ni and Mn in [0, 1.5] at% each, 1..max_vac vacancies and
    T in [523, 593] K.  All replicas share one alloy energy model; replica r
    uses Philox stream r.
    """
    rng = np.random.default_rng(seed)
    eps1, eps2, e0 = _rpv_alloy_model(rng)
    reps = []
    for r in range(n_rep):
        L = int(rng.integers(cells_range[0], cells_range[1] + 1))
        fr = {CU: rng.uniform(0.005, 0.020), NI: rng.uniform(0.0, 0.015),
              MN: rng.uniform(0.0, 0.015)}
        nv = int(rng.integers(1, max_vac + 1))
        T = float(rng.uniform(523.0, 593.0))
        occ = occupancy(rng, (L, L, L), 5, fr, nv)
        reps.append(LatticeSpec(dims=(L, L, L), n_species=5, eps1=eps1,
                                eps2=eps2, e0=e0, nu=6.0e12, temperature=T,
                                occ=occ, seed=seed, stream_id=r))
    return reps


def wall_thermal_field(nx: int = 32, nz: int = 96, t_inlet: float = 533.0,
                       t_outlet: float = 593.0, wall_drop: float = 10.0) -> np.ndarray:
    """Temperature samples T[z][x] (K) over a section of a reactor-vessel
    wall: x runs through the wall from the inner to the outer surface, z along
    the axis over the core belt.  A stand-in for the CAP1400 service field of
    Sec. IV-B, whose data the paper does not give: the inner surface follows
    the coolant from inlet to outlet temperature along z (cosine heating
    shape) and the wall cools linearly by wall_drop toward its outer surface,
    which spans the 523-593 K range of the replica ensembles."""
    x = (np.arange(nx) + 0.5) / nx
    z = (np.arange(nz) + 0.5) / nz
    tz = t_inlet + (t_outlet - t_inlet) * 0.5 * (1.0 - np.cos(np.pi * z))
    return tz[:, None] - wall_drop * x[None, :]


def voxel_replicas(temps: Sequence[float], n_x: int, n_z: int, cells: int = 16,
                   seed: int = 1004, max_vac: int = 8,
                   mu_wall: float = 2.0) -> List[LatticeSpec]:
    """One replica per voxel of an n_x by n_z wall grid (voxel b*n_x + a at
    temps[b*n_x + a]).  Vacancy counts follow a synthetic neutron flux of
    the Eq. 11 shape, phi = exp(-mu_wall x) f(z) with a cosine axial profile
    peaking mid-belt: nv = max(1, round(max_vac phi / phi_max)) (Eq. 12
    ties the initial vacancy concentration to the local conditions without
    a formula).  Compositions are drawn around the RPV solute fractions;
    one alloy energy model for all; replica r uses Philox stream r."""
    rng = np.random.default_rng(seed)
    eps1, eps2, e0 = _rpv_alloy_model(rng)
    reps = []
    for b in range(n_z):
        for a in range(n_x):
            xv = (a + 0.5) / n_x
            zv = (b + 0.5) / n_z
            phi = np.exp(-mu_wall * xv) * np.sin(np.pi * zv)
            nv = max(1, int(round(max_vac * phi)))
            fr = {CU: rng.uniform(0.005, 0.020), NI: rng.uniform(0.0, 0.015),
                  MN: rng.uniform(0.0, 0.015)}
            occ = occupancy(rng, (cells, cells, cells), 5, fr, nv)
            reps.append(LatticeSpec(dims=(cells, cells, cells), n_species=5, eps1=eps1,
                                    eps2=eps2, e0=e0, nu=6.0e12,
                                    temperature=float(temps[b * n_x + a]), occ=occ,
                                    seed=seed, stream_id=len(reps)))
    return reps


def random_lattice(rng: np.random.Generator, dims, n_species: int,
                   n_vac: int, solute_total: float = 0.3,
                   temperature: float = 563.0) -> LatticeSpec:
    """Small test lattice: heavy solute loading so every species and many
    mixed environments occur even on 3^3..6^3 cells."""
    eps1, eps2 = pair_tables(rng, n_species)
    e0 = rng.uniform(0.50, 0.70, size=n_species - 1)
    fr = {}
    if n_species > 2:
        per = solute_total / (n_species - 2)
        for s in range(1, n_species - 1):
            fr[s] = per
    occ = occupancy(rng, dims, n_species, fr, n_vac)
    return LatticeSpec(dims=tuple(dims), n_species=n_species, eps1=eps1,
                       eps2=eps2, e0=e0, nu=6.0e12, temperature=temperature,
                       occ=occ, seed=int(rng.integers(0, 2**63)), stream_id=0)


def pure_fe(dims, n_vac: int = 1, seed: int = 7, n_species: int = 3,
            temperature: float = 563.0, e0_fe: float = 0.62) -> LatticeSpec:
    """All-Fe lattice with vacancies at seeded positions (closed-form cases)."""
    rng = np.random.default_rng(seed)
    eps1, eps2 = pair_tables(rng, n_species)
    e0 = np.full(n_species - 1, 0.55)
    e0[0] = e0_fe
    lx, ly, lz = dims
    n = 2 * lx * ly * lz
    occ = np.zeros(n, dtype=np.uint8)
    occ[rng.choice(n, size=n_vac, replace=False)] = n_species - 1
    return LatticeSpec(dims=tuple(dims), n_species=n_species, eps1=eps1,
                       eps2=eps2, e0=e0, nu=6.0e12, temperature=temperature,
                       occ=occ, seed=seed, stream_id=0)


WORKLOADS = {
    "fe_cu_2k": fe_cu_2k,
    "rpv_524k": rpv_524k,
    "rpv_4m": rpv_4m,
}

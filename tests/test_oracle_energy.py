"""Pins of the oracle's lattice, energy change, barrier and rate.

Oracle functions pinned here: orc_site/orc_nbr1/orc_nbr2 (lattice reading),
orc_delta_e and orc_candidate (bond-count energy change, Kang-Weinberg
barrier, Arrhenius rate of Eq. 8, feasibility mask of Eq. 1).
"""
import math

import numpy as np
import pytest

from paper_2604_24091_amd import workloads as W
from tests import bruteforce as BF

DIMS = [(3, 3, 3), (3, 4, 5), (4, 4, 4), (5, 3, 4)]


@pytest.mark.parametrize("dims", DIMS)
def test_neighbour_tables_match_cartesian_shells(oracle_mod, dims):
    spec = W.pure_fe(dims)
    o = oracle_mod.Oracle(spec)
    adj1, adj2, disp = BF.shells(dims)
    n = spec.n_sites
    assert adj1.sum(1).tolist() == [8] * n
    assert adj2.sum(1).tolist() == [6] * n
    for s in range(n):
        n1 = [o.nbr1(s, k) for k in range(8)]
        n2 = [o.nbr2(s, m) for m in range(6)]
        assert sorted(n1) == sorted(np.flatnonzero(adj1[s]).tolist())
        assert sorted(n2) == sorted(np.flatnonzero(adj2[s]).tolist())
        for k, q in enumerate(n1):
            sx, sy, sz = disp[s, q]
            assert (4 * (sx > 0) + 2 * (sy > 0) + (sz > 0)) == k
        want = [(2, 0, 0), (-2, 0, 0), (0, 2, 0), (0, -2, 0), (0, 0, 2), (0, 0, -2)]
        assert [tuple(disp[s, q]) for q in n2] == want


@pytest.mark.parametrize("dims,S,nv,seed", [((3, 3, 3), 3, 3, 1), ((3, 4, 5), 5, 6, 2),
                                            ((4, 4, 4), 5, 8, 3), ((5, 5, 5), 5, 10, 4),
                                            ((4, 3, 3), 4, 2, 5)])
def test_delta_e_equals_whole_lattice_brute_force(oracle_mod, dims, S, nv, seed):
    rng = np.random.default_rng(seed)
    spec = W.random_lattice(rng, dims, S, nv, solute_total=0.4)
    o = oracle_mod.Oracle(spec)
    adj1, adj2, _ = BF.shells(dims)
    e_before = BF.total_energy(spec.occ, spec.eps1, spec.eps2, adj1, adj2)
    V = S - 1
    checked = 0
    for i in o.slots:
        for k in range(8):
            j = o.nbr1(int(i), k)
            de = o.delta_e(int(i), k)
            if spec.occ[j] == V:
                assert math.isnan(de)
                continue
            after = spec.occ.copy()
            after[i], after[j] = after[j], after[i]
            e_after = BF.total_energy(after, spec.eps1, spec.eps2, adj1, adj2)
            assert abs((e_after - e_before) - de) < 1e-10, (i, k)
            checked += 1
    assert checked > 0


def _worked_example(oracle_mod):
    """All-Fe lattice (Fe, Cu, V), vacancy at site 0 and one Cu on the
    (+,+,+) first neighbour of the vacancy."""
    spec = W.pure_fe((6, 6, 6), n_vac=0, seed=11)
    o = oracle_mod.Oracle(spec)
    occ = np.zeros(spec.n_sites, dtype=np.uint8)
    occ[0] = 2
    cu_site = o.nbr1(0, 7)
    occ[cu_site] = 1
    return spec, o, occ


def test_worked_example_single_cu(oracle_mod):
    spec, o, occ = _worked_example(oracle_mod)
    e1, e2 = spec.eps1, spec.eps2
    FE, CU, V = 0, 1, 2
    # (1) Cu jumps into the vacancy: every changed bond sees only Fe, dE = 0.
    assert o.delta_e(0, 7, occ) == 0.0
    # (2) Fe from a direction differing from (+,+,+) in one sign: Cu is a
    #     first neighbour of the vacancy and a second neighbour of that Fe.
    d1 = (e1[FE, CU] - e1[V, CU]) - (e1[FE, FE] - e1[V, FE])
    d2 = (e2[FE, CU] - e2[V, CU]) - (e2[FE, FE] - e2[V, FE])
    for k in (3, 5, 6):
        assert abs(o.delta_e(0, k, occ) - (d1 - d2)) < 1e-15
    # (3) Fe from the other four directions: only the first-shell Cu bond.
    for k in (0, 1, 2, 4):
        assert abs(o.delta_e(0, k, occ) - d1) < 1e-15
    # Barrier of the Cu jump is its own E0 (Kang-Weinberg with dE = 0).
    p = o.p
    kt = spec.kb * spec.temperature
    rates, ea = o.rates_sites(np.array([0], np.int32), occ)
    assert ea[0, 7] == spec.e0[CU]
    assert rates[0, 7] == pytest.approx(spec.nu * math.exp(-spec.e0[CU] / kt), rel=1e-15)


def test_pure_fe_rate_closed_form(oracle_mod):
    """Pure Fe: every admissible jump has Ea = E0(Fe) and the Eq. 8 rate."""
    spec = W.fe_cu_2k()
    spec.occ[:] = 0
    spec.occ[123] = 2
    o = oracle_mod.Oracle(spec)
    rates, ea = o.rates_vacancies()
    kt = 8.617333262e-5 * 563.0
    r = 6.0e12 * math.exp(-0.62 / kt)
    assert np.all(ea == 0.62)
    np.testing.assert_allclose(rates, r, rtol=1e-15)
    # Numbers for this parameter set: kT = 0.0485156 eV, r = 1.6909e7 Hz.
    assert kt == pytest.approx(0.0485156, abs=1e-7)
    assert r == pytest.approx(1.6909e7, rel=1e-4)
    assert o.gamma_tot() == pytest.approx(8 * r, rel=1e-15)


def test_vacancy_targets_are_masked(oracle_mod):
    rng = np.random.default_rng(9)
    spec = W.random_lattice(rng, (4, 4, 4), 3, 0)
    spec.occ[:] = 0
    o = oracle_mod.Oracle(spec)
    spec.occ[0] = 2
    for k in (1, 4, 6):
        spec.occ[o.nbr1(0, k)] = 2
    o = oracle_mod.Oracle(spec)
    rates, ea = o.rates_sites(np.array([0], np.int32))
    for k in range(8):
        if k in (1, 4, 6):
            assert rates[0, k] == 0.0 and math.isinf(ea[0, k])
        else:
            assert rates[0, k] > 0.0


@pytest.mark.parametrize("S,seed", [(3, 21), (5, 22)])
def test_detailed_balance(oracle_mod, S, seed):
    """The reverse jump has exactly the opposite bond counts, so
    dE_rev = -dE bit for bit and r_fwd / r_rev = exp(-dE / kT)."""
    rng = np.random.default_rng(seed)
    spec = W.random_lattice(rng, (5, 5, 5), S, 12, solute_total=0.5)
    o = oracle_mod.Oracle(spec)
    kt = spec.kb * spec.temperature
    V = S - 1
    n = 0
    for i in o.slots:
        for k in range(8):
            j = o.nbr1(int(i), k)
            if spec.occ[j] == V:
                continue
            de = o.delta_e(int(i), k)
            after = spec.occ.copy()
            after[i], after[j] = after[j], after[i]
            de_rev = o.delta_e(j, 7 - k, after)
            assert de_rev == -de
            r_f, _ = o.rates_sites(np.array([i], np.int32))
            r_b, _ = o.rates_sites(np.array([j], np.int32), after)
            ratio = r_f[0, k] / r_b[0, 7 - k]
            assert ratio == pytest.approx(math.exp(-de / kt), rel=1e-12)
            n += 1
    assert n > 20


def test_arrhenius_slope_and_sensitivity(oracle_mod):
    """Eq. 8: ln r is linear in 1/T with slope -Ea/kB; Eq. 9: the relative
    rate change for a small dT is Ea dT / (kB T^2)."""
    rng = np.random.default_rng(31)
    spec = W.random_lattice(rng, (4, 4, 4), 5, 4, solute_total=0.4)
    sites = np.flatnonzero(spec.occ == 4).astype(np.int32)
    Ts = np.array([523.0, 543.0, 563.0, 583.0, 603.0])
    logs = []
    for T in Ts:
        spec.temperature = T
        o = oracle_mod.Oracle(spec)
        r, ea = o.rates_sites(sites)
        logs.append(np.log(r[r > 0]))
        ea0 = ea[r > 0]
    logs = np.array(logs)
    slope = np.polyfit(1.0 / Ts, logs, 1)[0]
    np.testing.assert_allclose(slope, -ea0 / spec.kb, rtol=1e-9)
    T, dT = 563.0, 1e-3
    spec.temperature = T
    r0, ea = oracle_mod.Oracle(spec).rates_sites(sites)
    spec.temperature = T + dT
    r1, _ = oracle_mod.Oracle(spec).rates_sites(sites)
    m = r0 > 0
    rel = (r1[m] - r0[m]) / r0[m]
    np.testing.assert_allclose(rel, ea[m] * dT / (spec.kb * T * T), rtol=1e-4)


def test_binary32_mode_error_against_binary64(oracle_mod):
    """The binary32 rate mode stays within 1e-5 relative of binary64 on a
    heavily alloyed lattice (the stated error of the binary32 form)."""
    rng = np.random.default_rng(41)
    spec = W.random_lattice(rng, (12, 12, 12), 5, 0, solute_total=0.3)
    sites = np.arange(spec.n_sites, dtype=np.int32)
    r64, e64 = oracle_mod.Oracle(spec, precision=0).rates_sites(sites)
    r32, e32 = oracle_mod.Oracle(spec, precision=1).rates_sites(sites)
    m = r64 > 0
    assert np.array_equal(m, r32 > 0)
    rel = np.abs(r32[m] - r64[m]) / r64[m]
    assert rel.max() < 1e-5
    assert np.abs(e32[m] - e64[m]).max() < 1e-6


def test_encode_env_matches_bond_counts(oracle_mod):
    """The 27-slot surrogate input carries exactly the species of the bonds
    the jump changes: its group counts reproduce the oracle's energy change,
    and the frame reflection makes the (+,+,+) jump encode unchanged."""
    rng = np.random.default_rng(51)
    spec = W.random_lattice(rng, (4, 5, 4), 5, 6, solute_total=0.5)
    o = oracle_mod.Oracle(spec)
    S, V = 5, 4
    D1 = spec.eps1 - spec.eps1[V][None, :]
    D2 = spec.eps2 - spec.eps2[V][None, :]
    for i in o.slots:
        for k in range(8):
            env = o.encode_env(int(i), k)
            j = o.nbr1(int(i), k)
            assert env[0] == spec.occ[j]
            if env[0] == V:
                continue
            A = env[0]
            c = lambda sl: np.bincount(env[sl], minlength=S).astype(float)
            dn1 = c(slice(1, 8)) - c(slice(14, 21))
            dn2 = c(slice(8, 14)) - c(slice(21, 27))
            de = dn1 @ D1[A] + dn2 @ D2[A]
            assert abs(de - o.delta_e(int(i), k)) < 1e-12
            # N1(i) without j and N1(j) without i hold the right sites.
            n1i = sorted(spec.occ[[o.nbr1(int(i), q) for q in range(8) if q != k]])
            assert sorted(env[1:8]) == n1i
            n1j = sorted(spec.occ[[o.nbr1(j, q) for q in range(8) if q != 7 - k]])
            assert sorted(env[14:21]) == n1j
    # Reflection: the (+,+,+) jump is its own frame.
    i = int(o.slots[0])
    env = o.encode_env(i, 7)
    assert env[1:8].tolist() == [spec.occ[o.nbr1(i, d)] for d in range(7)]
    assert env[8:14].tolist() == [spec.occ[o.nbr2(i, m)] for m in range(6)]


def test_encode_env_is_reflection_invariant(oracle_mod):
    """Mirroring the lattice through the vacancy along the axes where jump k
    points negative turns jump k into the (+,+,+) jump; the encodings of the
    two must be identical."""
    rng = np.random.default_rng(52)
    dims = (4, 4, 4)
    spec = W.random_lattice(rng, dims, 5, 3, solute_total=0.6)
    o = oracle_mod.Oracle(spec)
    pos = BF.positions(dims)
    box = 2 * np.array(dims)
    index = {tuple(p): s for s, p in enumerate(pos)}
    for i in o.slots:
        pi = pos[i]
        for k in range(8):
            flip = np.array([(k >> 2) & 1 == 0, (k >> 1) & 1 == 0, k & 1 == 0])
            mpos = np.where(flip[None, :], 2 * pi[None, :] - pos, pos) % box
            mocc = np.empty_like(spec.occ)
            for s in range(spec.n_sites):
                mocc[index[tuple(mpos[s])]] = spec.occ[s]
            assert np.array_equal(o.encode_env(int(i), k), o.encode_env(int(i), 7, mocc))

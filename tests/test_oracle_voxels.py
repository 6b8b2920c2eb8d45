"""Pins of the voxel-ensemble oracle (oracle/voxels.py) and of the oracle's
time-horizon run (orc_run_until): the temperature-guided discretisation of
Sec. III-C1 (Eq. 9), the workload proxy of Sec. III-C2 (Eq. 10), and the
rule that a voxel advanced to a physical time stops at the first event that
reaches it.  Each pin is a closed form or a property the passage fixes, not
a second copy of the oracle's code."""
import math

import numpy as np
import pytest

from oracle import voxels as VX
from paper_2604_24091_amd import workloads as W

KB = 8.617333262e-5


def test_constant_field_is_one_voxel():
    T = np.full((12, 7), 563.0)
    nx, nz, tv, worst = VX.discretize(T, 0.6, KB, 1e-3)
    assert (nx, nz) == (1, 1) and tv[0] == 563.0 and worst == 0.0


@pytest.mark.parametrize("mx,mz", [(2, 1), (1, 3), (2, 3), (4, 2)])
def test_staircase_field_needs_exactly_its_steps(mx, mz):
    """A field constant on an mx-by-mz grid of blocks, with steps far above
    the tolerance, is split exactly along its steps: any grid with fewer
    voxels puts a step inside some voxel.  The voxel temperatures are the
    block values themselves."""
    nx, nz = 4 * mx, 3 * mz
    T = np.empty((nz, nx))
    for z in range(nz):
        for x in range(nx):
            T[z, x] = 540.0 + 10.0 * (x * mx // nx) + 25.0 * (z * mz // nz)
    gx, gz, tv, worst = VX.discretize(T, 0.6, KB, 1e-3)
    assert (gx, gz) == (mx, mz)
    want = [540.0 + 10.0 * a + 25.0 * b for b in range(mz) for a in range(mx)]
    assert list(tv) == want and worst == 0.0
    # A tolerance above every step's variation keeps one voxel.
    assert VX.discretize(T, 0.6, KB, 10.0)[:2] == (1, 1)


def test_eq9_is_the_first_order_log_rate_variation(oracle_mod):
    """Eq. 9 against Eq. 8 itself: the pure-Fe rate (every jump at E0) at T
    and T + dT, from the oracle's rate function, gives
    ln(r(T+dT)/r(T)) = E dT / (kB T (T+dT)); Eq. 9's E dT/(kB T^2) agrees to
    first order in dT/T."""
    for dT in (0.01, 0.1, 1.0):
        rates = []
        for T in (563.0, 563.0 + dT):
            spec = W.pure_fe((4, 4, 4), 1, 5, temperature=T, e0_fe=0.62)
            r, _ = oracle_mod.Oracle(spec).rates_vacancies()
            rates.append(r[0, 0])
        exact = math.log(rates[1] / rates[0])
        eq9 = VX.eq9_variation(0.62, KB, 563.0, 563.0, 563.0 + dT)
        assert abs(eq9 - exact) <= 2.0 * (dT / 563.0) * exact + 1e-12


def test_linear_field_voxels_bound_the_exact_rate_spread():
    """Whatever grid is chosen, every voxel's exact rate spread,
    (E/kB)(1/T_min - 1/T_max), stays within the tolerance up to the
    first-order error of Eq. 9, and one voxel fewer along the wall fails."""
    nx, nz = 24, 8
    T = np.array([[553.0 + 1.5 * x + 0.25 * z for x in range(nx)] for z in range(nz)])
    tol = 4e-2
    gx, gz, tv, worst = VX.discretize(T, 0.6, KB, tol)
    assert worst <= tol
    for m, lo, hi in VX.voxel_stats(T, gx, gz):
        exact = (0.6 / KB) * (1.0 / lo - 1.0 / hi)
        assert exact <= tol * (1.0 + 2.0 * (hi - lo) / lo)
        assert lo <= m <= hi
    assert gx > 1
    assert max(VX.eq9_variation(0.6, KB, m, lo, hi)
               for m, lo, hi in VX.voxel_stats(T, gx - 1, gz)) > tol


def test_priority_closed_forms(oracle_mod):
    """Pure Fe: every admissible jump has Ea = E0(Fe), so E_v = E0 and
    W_v = M_v exp(-E0/kT) with M_v = 8 per isolated vacancy; two vacancies
    on neighbouring sites lose the jump onto each other (Eq. 1 mask)."""
    spec = W.pure_fe((6, 6, 6), 3, 9, temperature=573.0, e0_fe=0.62)
    o = oracle_mod.Oracle(spec)
    _, ea = o.rates_vacancies()
    kT = KB * 573.0
    m, e, w = VX.priority(ea, kT)
    near = any(o.nbr1(int(a), k) == int(b) for a in o.slots for b in o.slots for k in range(8))
    assert not near
    assert m == 24 and np.all(ea == 0.62)
    assert abs(e - 0.62) <= 24 * 2.0 ** -52           # a sum of 24 equal terms, then / 24
    assert abs(w / (24 * math.exp(-(0.62 / kT))) - 1.0) <= 1e-13
    occ = np.zeros(2 * 6 ** 3, dtype=np.uint8)
    i = 37
    j = o.nbr1(i, 5)
    occ[[i, j]] = 2
    spec2 = W.LatticeSpec(dims=(6, 6, 6), n_species=3, eps1=spec.eps1, eps2=spec.eps2,
                          e0=spec.e0, nu=spec.nu, temperature=573.0, occ=occ, seed=1,
                          stream_id=0)
    _, ea2 = oracle_mod.Oracle(spec2).rates_vacancies()
    m2, _, _ = VX.priority(ea2, kT)
    assert m2 == 14
    m0, e0, w0 = VX.priority(np.full((2, 8), np.inf), kT)
    assert m0 == 0 and math.isnan(e0) and w0 == 0.0


def test_dispatch_order_heaviest_first_ties_by_index():
    assert VX.dispatch_order([1.0, 3.0, 3.0, 0.0, 2.0]) == [1, 2, 4, 0, 3]
    assert VX.dispatch_order([]) == []


def test_run_until_stops_at_the_event_that_reaches_the_horizon(oracle_mod):
    """Mean-time mode in pure Fe with one vacancy: every event adds
    dt = 1/G with the same G = 8 r0, so a horizon of (K + 1/2)/G is reached
    by event K + 1 exactly."""
    spec = W.pure_fe((5, 5, 5), 1, 3, temperature=563.0, e0_fe=0.62)
    o = oracle_mod.Oracle(spec, time_mode=1)
    g = o.gamma_tot()
    K = 37
    done, log = o.run_until((K + 0.5) / g, 10 ** 6, log=True)
    assert done == K + 1 and np.all(log["dt"] == 1.0 / g)
    t_before = o.state.t - log["dt"][-1]
    assert t_before < (K + 0.5) / g <= o.state.t
    # Already past the horizon: nothing happens.
    assert o.run_until((K + 0.5) / g, 10) == 0


def test_run_until_equals_fixed_count_and_chunks(oracle_mod):
    """Stochastic time on an alloy: the run to a horizon is the fixed-count
    run of the same length, bit for bit, and splitting it by max_events
    changes nothing."""
    spec = W.random_lattice(np.random.default_rng(77), (6, 6, 6), 4, 6, solute_total=0.1)
    a = oracle_mod.Oracle(spec)
    t_end = 2.0e-6
    n, log = a.run_until(t_end, 10 ** 6, log=True)
    assert n > 10 and a.state.t >= t_end and a.state.t - log["dt"][-1] < t_end
    b = oracle_mod.Oracle(spec)
    assert b.run(n) == n
    assert b.state.digest == a.state.digest and b.state.t == a.state.t
    assert np.array_equal(b.occ, a.occ)
    c = oracle_mod.Oracle(spec)
    total = 0
    while True:
        d = c.run_until(t_end, 7)
        total += d
        if d < 7:
            break
    assert total == n and c.state.digest == a.state.digest and c.state.t == a.state.t

"""Pins of the oracle's pair model out to 6.0 A (six shells, the 64
neighbours of Sec. IV-C's observation range): the local energy change of
every jump against the whole-lattice brute-force energy difference
(independent Cartesian shells), detailed balance, the first-two-shell model
as its special case, and the local-refresh reach."""
import math

import numpy as np
import pytest

from paper_2604_24091_amd import workloads as W
from tests import bruteforce as BF


def _far_spec(rng, dims, S, nv, solute_total=0.4):
    spec = W.random_lattice(rng, dims, S, nv, solute_total=solute_total)
    spec.eps_far = W.far_tables(rng, S)
    return spec


@pytest.mark.parametrize("dims,S,nv,seed", [((5, 5, 5), 3, 3, 1), ((5, 6, 5), 5, 6, 2),
                                            ((6, 5, 7), 4, 5, 3), ((6, 6, 6), 5, 9, 4)])
def test_delta_e_equals_whole_lattice_brute_force(oracle_mod, dims, S, nv, seed):
    rng = np.random.default_rng(seed)
    spec = _far_spec(rng, dims, S, nv)
    o = oracle_mod.Oracle(spec)
    adj = BF.shells6(dims)
    eps = [np.asarray(spec.eps1), np.asarray(spec.eps2)] + [spec.eps_far[m] for m in range(4)]
    e0 = BF.total_energy6(spec.occ, eps, adj)
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
            e1 = BF.total_energy6(after, eps, adj)
            assert abs((e1 - e0) - de) < 1e-10, (i, k, e1 - e0, de)
            checked += 1
    assert checked > 0
    # the far shells matter: with them dropped the energy change differs
    near = W.LatticeSpec(**{**spec.__dict__, "eps_far": None})
    on = oracle_mod.Oracle(near)
    diffs = [abs(on.delta_e(int(i), k) - o.delta_e(int(i), k)) for i in o.slots for k in range(8)
             if spec.occ[o.nbr1(int(i), k)] != V]
    assert max(diffs) > 1e-3


def test_two_shell_model_is_the_special_case(oracle_mod):
    """Zero energies beyond the second shell give the first-two-shell
    model's rates and barriers bit for bit."""
    rng = np.random.default_rng(9)
    spec = W.random_lattice(rng, (6, 6, 6), 5, 8, solute_total=0.3)
    far = W.LatticeSpec(**{**spec.__dict__, "eps_far": np.zeros((4, 5, 5))})
    r2, e2 = oracle_mod.Oracle(spec).rates_vacancies()
    r6, e6 = oracle_mod.Oracle(far).rates_vacancies()
    assert np.array_equal(r2, r6) and np.array_equal(e2, e6)


def test_detailed_balance_far(oracle_mod):
    """dE of the reverse jump is -dE bit for bit (integer counts negate),
    and r_f / r_b = exp(-dE/kT)."""
    rng = np.random.default_rng(10)
    spec = _far_spec(rng, (6, 6, 6), 5, 6)
    o = oracle_mod.Oracle(spec)
    V = spec.n_species - 1
    kT = spec.kb * spec.temperature
    n = 0
    for i in o.slots:
        for k in range(8):
            j = o.nbr1(int(i), k)
            if spec.occ[j] == V:
                continue
            de = o.delta_e(int(i), k)
            after = spec.occ.copy()
            after[i], after[j] = after[j], after[i]
            de_rev = o.delta_e(int(j), 7 - k, occ=after)
            assert de_rev == -de
            A = int(spec.occ[j])
            rf = spec.nu * math.exp(-(spec.e0[A] + 0.5 * de) / kT)
            rb = spec.nu * math.exp(-(spec.e0[A] - 0.5 * de) / kT)
            assert abs(rf / rb / math.exp(-de / kT) - 1) < 1e-12
            n += 1
    assert n > 20


def test_local_refresh_reach_far(oracle_mod):
    """With vacancies packed closely, the local-refresh mode (reach 5
    half-cells) gives the full recompute's trajectory bit for bit."""
    rng = np.random.default_rng(11)
    spec = _far_spec(rng, (5, 5, 5), 4, 30, solute_total=0.3)
    a = oracle_mod.Oracle(spec)
    b = oracle_mod.Oracle(spec)
    na, la = a.run(400, log=True)
    nb, lb = b.run(400, log=True, local=True)
    assert na == nb == 400
    assert np.array_equal(la["to_site"], lb["to_site"]) and a.state.digest == b.state.digest

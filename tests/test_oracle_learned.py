"""Pins of the oracle's learned runtime forms (orc_observation,
orc_patchnet_forward, orc_policy_weights, orc_poisson_u, orc_poisson_dt,
orc_run_learned): the 64-neighbour observation of Sec. IV-C, the masked and
temperature-scaled policy with a system-wide softmax (Eq. 1-2) and its
zero-shot size invariance (Eq. 4), and Poisson-time alignment (Eq. 5-7).
Anchors: an independent Cartesian neighbour search, numpy evaluations of the
network and of the softmax, closed forms, and an exactly solved mean
first-passage problem."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2604_24091_amd import workloads as W

A_LAT = 2.866   # Angstrom


def _net(rng, S, H, n_out, scale=0.5, bias3=0.0):
    from oracle import akmc_oracle as O

    def bf(a):   # values exactly representable in bfloat16
        a = np.asarray(a, dtype=np.float32)
        return (a.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
    return O.PatchNet(bf(rng.normal(0, scale, (64, S, H))), rng.normal(0, 0.1, H),
                      bf(rng.normal(0, scale / 4, (H, H))), rng.normal(0, 0.1, H),
                      bf(rng.normal(0, scale / 4, (H, n_out))),
                      np.full(n_out, bias3, dtype=np.float32))


def _cart(o, spec, s):
    lx, ly, lz = spec.dims
    nc = lx * ly * lz
    b, r = divmod(int(s), nc)
    x, r = r % lx, r // lx
    y, z = r % ly, r // ly
    return np.array([x + 0.5 * b, y + 0.5 * b, z + 0.5 * b]) * A_LAT


def test_observation_is_the_6A_neighbourhood(oracle_mod):
    """The 64 observed sites of a vacancy are exactly the sites within
    6.0 A (minimum image), in the six shells 8/6/12/24/8/6 at
    a sqrt(3)/2, a, a sqrt(2), a sqrt(11)/2, a sqrt(3), 2a; the next shell
    (a sqrt(19)/2 = 6.25 A) is left out."""
    spec = W.random_lattice(np.random.default_rng(3), (5, 6, 7), 4, 2)
    o = oracle_mod.Oracle(spec)
    occ = np.arange(spec.n_sites) % 251          # site-distinguishing codes only for the mapping
    lx, ly, lz = spec.dims
    box = np.array([lx, ly, lz]) * A_LAT
    for i in (0, 17, spec.n_sites - 1, spec.n_sites // 2 + 3):
        ci = _cart(o, spec, i)
        d = np.array([_cart(o, spec, s) for s in range(spec.n_sites)]) - ci
        d -= box * np.round(d / box)
        r = np.sqrt((d ** 2).sum(1))
        near = set(np.flatnonzero((r > 0) & (r <= 6.0)).tolist())
        offs = oracle_mod.obs_offsets()
        got = []
        for m in range(64):
            # site of offset m, found by its Cartesian displacement
            want = offs[m] * (A_LAT / 2)
            hit = np.flatnonzero(np.all(np.abs(d - want) < 1e-9, axis=1))
            assert hit.size == 1
            got.append(int(hit[0]))
        assert set(got) == near and len(got) == 64
        radii = np.sqrt((offs.astype(float) ** 2).sum(1)) * A_LAT / 2
        assert np.all(np.diff(radii) >= -1e-12)
        shells = np.unique(np.round(radii, 6), return_counts=True)
        want_r = A_LAT * np.array([math.sqrt(3) / 2, 1, math.sqrt(2), math.sqrt(11) / 2,
                                   math.sqrt(3), 2])
        assert np.allclose(shells[0], want_r) and list(shells[1]) == [8, 6, 12, 24, 8, 6]
        codes = o.observation(i, occ=(occ % 256).astype(np.uint8))
        assert list(codes) == [occ[g] % 256 for g in got]


def test_network_matches_a_dense_one_hot_evaluation(oracle_mod):
    """The gather-sum first layer equals the one-hot input times W1; the
    whole forward equals a float64 evaluation to binary32 rounding."""
    rng = np.random.default_rng(5)
    for S, H, n_out in ((3, 16, 8), (5, 64, 8), (5, 32, 1)):
        net = _net(rng, S, H, n_out)
        for _ in range(5):
            codes = rng.integers(0, S, 64).astype(np.uint8)
            x = np.zeros(64 * S)
            x[np.arange(64) * S + codes] = 1.0
            h1 = np.maximum(net.b1 + x @ net.w1.reshape(64 * S, H).astype(np.float64), 0)
            h2 = np.maximum(net.b2 + h1 @ net.w2.astype(np.float64), 0)
            y = net.b3 + h2 @ net.w3.astype(np.float64)
            got = oracle_mod.patchnet_forward(net, codes)
            assert np.allclose(got, y, rtol=1e-5, atol=1e-5 * max(1.0, np.abs(y).max()))


def test_policy_mask_and_temperature(oracle_mod):
    """Eq. 1: a jump onto a vacancy gets weight 0; the others exp(z/tau).
    tau -> infinity makes every admissible jump equally likely."""
    rng = np.random.default_rng(8)
    spec = W.random_lattice(rng, (5, 5, 5), 4, 12, solute_total=0.3)
    o = oracle_mod.Oracle(spec)
    net = _net(rng, 4, 32, 8)
    w, z = o.policy_weights(net, np.float32(1.0 / 0.7))
    V = spec.n_species - 1
    masked = 0
    for v, i in enumerate(o.slots):
        for k in range(8):
            if o.occ[o.nbr1(int(i), k)] == V:
                assert w[v, k] == 0.0
                masked += 1
            else:
                zz = float(np.float32(z[v, k] * np.float32(1.0 / 0.7)))
                assert abs(w[v, k] / math.exp(zz) - 1.0) <= 1e-15
    assert masked > 0
    w0, _ = o.policy_weights(net, 0.0)
    assert set(np.unique(w0).tolist()) <= {0.0, 1.0}


def test_policy_selection_frequencies_follow_the_softmax(oracle_mod):
    """Eq. 2: the first event drawn from one state over many random streams
    has the distribution softmax(z_hat) over all candidates (chi-square)."""
    rng = np.random.default_rng(9)
    spec = W.random_lattice(rng, (5, 5, 5), 3, 3, solute_total=0.4)
    net = _net(rng, 3, 16, 8, scale=0.8)
    base = oracle_mod.Oracle(spec)
    w, _ = base.policy_weights(net, 1.0)
    p = (w / w.sum()).ravel()
    counts = np.zeros(p.size)
    n = 4000
    for sid in range(n):
        spec.stream_id = sid
        o = oracle_mod.Oracle(spec)
        done, log = o.run_learned(1, pol=net, inv_tau=1.0, log=True)
        assert done == 1
        counts[int(log["slot"][0]) * 8 + int(log["dir"][0])] += 1
    assert np.all(counts[p == 0] == 0)
    live = p > 0
    chi = stats.chisquare(counts[live], n * p[live])
    assert chi.pvalue > 1e-3, chi


def test_policy_is_size_invariant_eq4(oracle_mod):
    """Eq. 4: the probability of choosing direction k from a vacancy context
    depends only on the context's frequency and its logits.  A lattice tiled
    2x2x2 has the same context frequencies, so every (context, k) keeps its
    probability (the 8 copies of a vacancy together)."""
    rng = np.random.default_rng(10)
    small = W.random_lattice(rng, (5, 5, 6), 4, 4, solute_total=0.3)
    net = _net(rng, 4, 32, 8)
    lx, ly, lz = small.dims
    occ = small.occ.reshape(2, lz, ly, lx)
    big_occ = np.tile(occ, (1, 2, 2, 2)).reshape(-1)
    big = W.LatticeSpec(dims=(2 * lx, 2 * ly, 2 * lz), n_species=small.n_species,
                        eps1=small.eps1, eps2=small.eps2, e0=small.e0, nu=small.nu,
                        temperature=small.temperature, occ=big_occ, seed=1, stream_id=0)
    os_, ob = oracle_mod.Oracle(small), oracle_mod.Oracle(big)
    ws, _ = os_.policy_weights(net, 1.3)
    wb, _ = ob.policy_weights(net, 1.3)
    ps = ws / ws.sum()
    pb = wb / wb.sum()
    agg = np.zeros_like(ps)
    for v, s in enumerate(ob.slots):
        b, r = divmod(int(s), 8 * lx * ly * lz)
        x, r = r % (2 * lx), r // (2 * lx)
        y, z = r % (2 * ly), r // (2 * ly)
        small_site = b * lx * ly * lz + ((z % lz) * ly + (y % ly)) * lx + (x % lx)
        agg[int(np.flatnonzero(os_.slots == small_site)[0])] += pb[v]
    assert np.allclose(agg, ps, rtol=1e-12, atol=0)


def test_poisson_time_constant_network_closed_form(oracle_mod):
    """A Poisson network that outputs a constant c gives u(s) = n_v c, so
    Eq. 7 reads dtau = n_v c (1/Gamma(s) - 1/Gamma(s')) for every event."""
    rng = np.random.default_rng(11)
    spec = W.random_lattice(rng, (5, 5, 5), 4, 3, solute_total=0.2)
    S, H = spec.n_species, 16
    from oracle import akmc_oracle as O
    c = 0.8125
    pn = O.PatchNet(np.zeros((64, S, H)), np.zeros(H), np.zeros((H, H)), np.zeros(H),
                    np.zeros((H, 1)), np.array([c]))
    o = oracle_mod.Oracle(spec)
    assert o.poisson_u(pn) == 3 * c
    done, log = o.run_learned(60, pn=pn, log=True)
    assert done == 60
    g = np.append(log["gamma_tot"], o.state.gamma_tot)
    want = (3 * c - (g[:-1] / g[1:]) * (3 * c)) / g[:-1]
    assert np.allclose(log["dt"], want, rtol=1e-13, atol=1e-13 * np.abs(want).max())
    assert np.all(log["dt"] == want)


def test_poisson_time_telescopes(oracle_mod):
    """Eq. 6-7: dtau = tau(s) - tau(s') with tau = u/Gamma, so the times of
    a trajectory sum to u(s_0)/Gamma(s_0) - u(s_N)/Gamma(s_N) for any
    network."""
    rng = np.random.default_rng(12)
    spec = W.random_lattice(rng, (5, 5, 6), 4, 4, solute_total=0.2)
    pn = _net(rng, spec.n_species, 32, 1, scale=0.3, bias3=2.0)
    o = oracle_mod.Oracle(spec)
    u0, g0 = o.poisson_u(pn), o.gamma_tot()
    done, log = o.run_learned(200, pn=pn, log=True)
    uN, gN = o.poisson_u(pn), o.gamma_tot()
    lhs = math.fsum(log["dt"])
    rhs = u0 / g0 - uN / gN
    assert abs(lhs - rhs) <= 1e-9 * max(abs(u0 / g0), abs(uN / gN))


def test_poisson_time_with_the_exact_first_passage_time(oracle_mod):
    """Eq. 5 solved exactly: one vacancy walks in pure Fe around one Cu atom
    until it becomes a first neighbour of the Cu (the absorbing set).  The
    mean first-passage times tau solve sum_a Gamma_a (tau(s') - tau(s)) = -1;
    with u = Gamma tau, Eq. 7's increment averaged over the next event is
    the classical mean residence time 1/Gamma(s) in every transient state,
    and tau(s) - tau(s') is what Eq. 7 returns."""
    spec = W.pure_fe((4, 4, 4), 1, 3, n_species=3)
    n = spec.n_sites
    cu = 5
    base = np.zeros(n, dtype=np.uint8)
    base[cu] = 1
    o = oracle_mod.Oracle(spec)
    absorbing = {o.nbr1(cu, k) for k in range(8)}
    trans = [s for s in range(n) if s != cu and s not in absorbing]
    idx = {s: a for a, s in enumerate(trans)}
    M = np.zeros((len(trans), len(trans)))
    rhs = -np.ones(len(trans))
    rates = {}
    for s in trans:
        occ = base.copy()
        occ[s] = 2
        r, _ = o.rates_sites(np.array([s], dtype=np.int32), occ=occ)
        rates[s] = r[0]
        a = idx[s]
        for k in range(8):
            t = o.nbr1(s, k)
            M[a, a] -= r[0, k]
            if t in idx:
                M[a, idx[t]] += r[0, k]
    tau = np.linalg.solve(M, rhs)
    for s in trans[::7]:
        g = float(rates[s].sum())
        us = g * tau[idx[s]]
        mean = 0.0
        for k in range(8):
            t = o.nbr1(s, k)
            if t in idx:
                gt = float(rates[t].sum())
                ut = gt * tau[idx[t]]
            else:
                gt, ut = 1.0, 0.0            # absorbed: tau(s') = 0
            d = oracle_mod.poisson_dt(us, g, ut, gt)
            assert abs(d - (tau[idx[s]] - (tau[idx[t]] if t in idx else 0.0))) <= 1e-9 * tau.max()
            mean += rates[s][k] / g * d
        assert abs(mean * g - 1.0) <= 1e-9


def test_follow_learned_accepts_its_own_log_and_flags_a_wrong_one(oracle_mod):
    """The learned follow mode replays a run's own log with no violation
    and exact times, and flags a log whose choice was altered."""
    rng = np.random.default_rng(13)
    spec = W.random_lattice(rng, (5, 5, 5), 4, 3, solute_total=0.2)
    pol = _net(rng, spec.n_species, 16, 8, scale=0.6)
    pn = _net(rng, spec.n_species, 16, 1, scale=0.3, bias3=1.5)
    a = oracle_mod.Oracle(spec)
    done, log = a.run_learned(300, pol=pol, inv_tau=1.25, pn=pn, log=True)
    assert done == 300
    f = oracle_mod.Oracle(spec)
    res = f.follow_learned(log, pol=pol, inv_tau=1.25, pn=pn)
    assert res["mismatches"] == 0 and res["n_differ"] == 0
    assert res["max_select_violation"] == 0.0 and res["max_dt_rel"] == 0.0
    assert res["max_gamma_rel"] == 0.0
    assert f.state.digest == a.state.digest and f.state.t == a.state.t
    bad = log.copy()
    e = 120
    alt = [k for k in range(8) if k != int(bad["dir"][e])]
    bad["dir"][e] = alt[0]
    g = oracle_mod.Oracle(spec)
    res = g.follow_learned(bad, pol=pol, inv_tau=1.25, pn=pn)
    assert res["mismatches"] == 1 or res["n_differ"] >= 1

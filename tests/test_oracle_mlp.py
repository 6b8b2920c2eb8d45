"""Pins of the surrogate's binary64 oracle (oracle/mlp.py): encoding,
GELU, gradients (central finite differences and an independent autograd),
AdamW (closed-form first step and an independent library optimizer)."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _data(rng, n, S=5):
    env = rng.integers(0, S, size=(n, 27))
    env[:, 0] = rng.integers(0, S - 1, size=n)
    return env, rng.uniform(0.4, 0.8, size=n)


def test_one_hot_layout():
    env = np.arange(27) % 5
    x = M.one_hot(env[None, :], 5)
    assert x.shape == (1, 160)
    assert x.sum() == 27 and np.all(x[0, 135:] == 0)
    for s in range(27):
        assert x[0, s * 5 + env[s]] == 1.0


def test_gelu_tanh_close_to_erf_gelu():
    from scipy.special import erf
    z = np.linspace(-6, 6, 2001)
    exact = 0.5 * z * (1 + erf(z / math.sqrt(2)))
    assert np.max(np.abs(M.gelu(z) - exact)) < 1e-3
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, atol=1e-8)


def test_bf16_rounding():
    # bfloat16 keeps 8 significant bits: spacing 2^-7 just above 1.
    assert M.bf16(1.0) == 1.0
    assert M.bf16(1.0 + 2 ** -9) == 1.0                      # below half a spacing
    assert M.bf16(1.0 + 2 ** -8) == 1.0                      # tie, rounds to even
    assert M.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6        # tie, rounds to even
    assert M.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7
    assert M.bf16(-3.0) == -3.0
    x = np.random.default_rng(0).normal(size=1000)
    assert np.max(np.abs(M.bf16(x) - x) / np.abs(x)) <= 2 ** -8


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(5, rng, mu=0.6, sigma=0.05)
    for k in M.PARAM_KEYS:
        p[k] = p[k] + rng.normal(scale=0.05, size=p[k].shape)
    env, ea = _data(rng, 16)
    x = M.one_hot(env, 5)
    _, g = M.loss_and_grads(p, x, ea)
    h = 1e-6
    for k in M.PARAM_KEYS:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        if k == "W1":                                   # rows that are hit by the inputs
            hit = np.flatnonzero(x.sum(0) > 0)
            idx = np.array([r * M.HID + c for r, c in zip(rng.choice(hit, 12), rng.integers(0, M.HID, 12))])
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = M.loss_and_grads(p, x, ea)
            flat[i] = old - h
            lm, _ = M.loss_and_grads(p, x, ea)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, i, fd, an)


def test_gradients_match_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    p = M.init_params(5, rng, mu=0.6, sigma=0.05)
    env, ea = _data(rng, 32)
    x = M.one_hot(env, 5)
    loss, g = M.loss_and_grads(p, x, ea)
    T = {k: torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in M.PARAM_KEYS}
    xt = torch.tensor(x)
    z1 = xt @ T["W1"] + T["b1"]
    h1 = torch.nn.functional.gelu(z1, approximate="tanh")
    z2 = h1 @ T["W2"] + T["b2"]
    h2 = torch.nn.functional.gelu(z2, approximate="tanh")
    y = h2 @ T["w3"] + T["b3"][0]
    t = (torch.tensor(ea) - p["mu"]) / p["sigma"]
    L = torch.mean((y - t) ** 2)
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    for k in M.PARAM_KEYS:
        np.testing.assert_allclose(g[k], T[k].grad.numpy(), rtol=1e-10, atol=1e-13)


def test_adamw_first_step_closed_form_and_library():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    p = M.init_params(5, rng)
    g = {k: rng.normal(size=np.shape(p[k])) for k in M.PARAM_KEYS}
    lr, wd = 1e-3, 0.01
    p0 = {k: np.array(p[k], copy=True) for k in M.PARAM_KEYS}
    st = {}
    M.adamw_step(p, g, st, lr, weight_decay=wd, eps=0.0)
    # First step: m_hat = g, v_hat = g^2, so the Adam part moves by lr*sign(g).
    for k in M.PARAM_KEYS:
        np.testing.assert_allclose(p[k], p0[k] * (1 - lr * wd) - lr * np.sign(g[k]), rtol=1e-12, atol=1e-15)
    # Ten steps against torch.optim.AdamW.
    p = {k: np.array(p0[k], copy=True) for k in M.PARAM_KEYS}
    T = [torch.tensor(p0[k], dtype=torch.float64, requires_grad=True) for k in M.PARAM_KEYS]
    opt = torch.optim.AdamW(T, lr=lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    st = {}
    for it in range(10):
        gi = {k: rng.normal(size=np.shape(p0[k])) for k in M.PARAM_KEYS}
        M.adamw_step(p, gi, st, lr, weight_decay=wd)
        for tt, k in zip(T, M.PARAM_KEYS):
            tt.grad = torch.tensor(gi[k])
        opt.step()
    for tt, k in zip(T, M.PARAM_KEYS):
        np.testing.assert_allclose(p[k], tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_pair_barrier_is_representable_exactly_by_the_features():
    """The pair-model barrier is affine in one-hot(A) x one-hot(slot species):
    a least-squares fit on the one-hot features of each mover species
    reproduces it to rounding, so the surrogate's target lies in reach."""
    from paper_2604_24091_amd import workloads as W
    from oracle import akmc_oracle as O
    rng = np.random.default_rng(4)
    spec = W.random_lattice(rng, (8, 8, 8), 5, 0, solute_total=0.4)
    o = O.Oracle(spec)
    sites = rng.choice(spec.n_sites, 400, replace=False).astype(np.int32)
    envs, eas = [], []
    _, ea = o.rates_sites(sites)
    for a, i in enumerate(sites):
        for k in range(8):
            e = o.encode_env(int(i), k)
            if e[0] == 4:
                continue
            envs.append(e)
            eas.append(ea[a, k])
    envs, eas = np.array(envs), np.array(eas)
    for A in range(4):
        m = envs[:, 0] == A
        if m.sum() < 200:
            continue
        X = np.hstack([M.one_hot(envs[m], 5), np.ones((m.sum(), 1))])
        coef, *_ = np.linalg.lstsq(X, eas[m], rcond=None)
        assert np.max(np.abs(X @ coef - eas[m])) < 1e-10


def test_ood_rule_and_learned_barrier_model():
    """The learned barrier model: inadmissible jumps stay +inf, candidates
    whose moving species or any bond-group count lies outside the training
    rows take the pair barrier, every other candidate the network's."""
    from paper_2604_24091_amd import workloads as W
    from oracle import akmc_oracle as O
    rng = np.random.default_rng(12)
    spec = W.random_lattice(rng, (6, 6, 6), 5, 6, solute_total=0.05)
    o = O.Oracle(spec)
    env_all = o.encode_env_sites(np.arange(spec.n_sites, dtype=np.int32)).reshape(-1, 27)
    # Training rows: only all-Fe environments with Fe moving.
    train = np.zeros((10, 27), dtype=np.uint8)
    train[3, 0] = 4                                   # a vacancy row: not a training row
    b = M.ood_bounds(train, 5)
    assert list(b["seen"]) == [0] and b["max"].shape == (4, 5)
    assert np.all(b["max"][:, 0] == [7, 6, 7, 6]) and np.all(b["max"][:, 1:] == 0)
    ind = M.in_distribution(b, env_all, 5)
    allfe = np.all(env_all == 0, axis=1)
    assert np.array_equal(ind, allfe)
    # One extra Cu in N2(j) takes a row out; a Cu mover too.
    e = np.zeros((2, 27), dtype=np.uint8)
    e[0, 22] = 1
    e[1, 0] = 1
    assert not M.in_distribution(b, e, 5).any()
    p = M.init_params(5, rng, mu=0.6, sigma=0.05)
    model = M.barrier_model(p, b, o, 5)
    ea = model(o.occ, o.slots)
    _, ea_pair = o.rates_sites(o.slots)
    env = o.encode_env_sites(o.slots).reshape(-1, 27)
    ind = M.in_distribution(b, env, 5) & np.isfinite(ea_pair.reshape(-1))
    flat = ea.reshape(-1)
    assert np.array_equal(np.isinf(flat), np.isinf(ea_pair.reshape(-1)))
    assert np.array_equal(flat[~ind], ea_pair.reshape(-1)[~ind])
    if ind.any():
        np.testing.assert_array_equal(flat[ind], M.predict_ea(p, env[ind], 5, True))


def test_follower_reproduces_the_plain_oracle_and_flags_a_wrong_log():
    """The Python follow mode with pair barriers, on the C oracle's own log:
    every choice inside its interval, and the final state, digest and time
    equal to the oracle run bit for bit; a log with one wrong direction is a
    structural mismatch, and a log whose uniforms belong to another stream
    puts choices outside their intervals."""
    from paper_2604_24091_amd import workloads as W
    from oracle import akmc_oracle as O
    from oracle.follow import Follower
    spec = W.random_lattice(np.random.default_rng(13), (5, 5, 5), 5, 7, solute_total=0.3)
    ref = O.Oracle(spec)
    _, log = ref.run(500, log=True)
    geo = O.Oracle(spec)
    pair = lambda occ, slots: geo.rates_sites(slots, occ)[1]
    f = Follower(spec, pair)
    r = f.follow(log)
    assert r["mismatches"] == 0 and r["n_differ"] == 0 and r["events"] == 500
    assert r["max_select_violation"] == 0.0 and r["max_gamma_rel"] < 1e-15 and r["max_dt_rel"] < 1e-15
    assert np.array_equal(f.occ, ref.occ) and f.digest == ref.state.digest and f.t == ref.state.t
    bad = log.copy()
    bad["dir"][100] = (bad["dir"][100] + 1) % 8
    r = Follower(spec, pair).follow(bad)
    assert r["mismatches"] == 1 and r["events"] <= 100
    other = W.LatticeSpec(**{**spec.__dict__, "stream_id": spec.stream_id + 1})
    r = Follower(other, pair).follow(log)
    assert r["n_differ"] > 100

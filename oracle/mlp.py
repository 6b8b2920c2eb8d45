"""Binary64 reference of the learned barrier surrogate (test infrastructure).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.

The paper replaces per-atom GEMVs of a shared network by batched GEMMs
(Sec. III-B1, "swarm gathering") and runs the matrix work in reduced
precision with layer fusion; it trains with AdamW, batch 256 (Sec. IV-C).
The surrogate here is the small network those ideas are applied to in this
project: the barrier Ea of a vacancy jump predicted from the species in the
bonds the jump changes.

Definition (a reading; the paper gives no barrier network):
  input   27 footprint slots in the jump frame (slot 0 the moving species,
          then N1(i)\\{j}, N2(i), N1(j)\\{i}, N2(j)), each one-hot over the S
          species codes: x[27*S] zero-padded to K1 = 32*ceil(27*S/32)
  layers  z1 = x W1 + b1 (K1 x 128), h1 = gelu(z1)
          z2 = h1 W2 + b2 (128 x 128), h2 = gelu(z2)
          y  = h2 . w3 + b3,   Ea = mu + sigma * y
  gelu    0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))
  loss    mean over the batch of (y - (Ea_target - mu)/sigma)^2
  AdamW   decoupled weight decay, then Adam with bias correction
          (Loshchilov and Hutter, ICLR 2019).
bf16=True rounds x W-inputs and hidden activations to bfloat16 where the
GPU kernels store them in bfloat16 (weights, h1, h2); accumulation stays
binary64.

Out of distribution (a reading; the paper's policy masks inadmissible
moves but states no rule for unfamiliar environments): a candidate whose
moving species never moved in the training rows, or whose count of some
species in one of the four bond groups (N1(i) without j, N2(i), N1(j)
without i, N2(j)) exceeds the largest count of that species in that group
over the training rows, takes the pair-model barrier instead.
"""
from __future__ import annotations

import math

import numpy as np

HID = 128
N_SLOTS = 27
GELU_C = math.sqrt(2.0 / math.pi)


def k1_of(S: int) -> int:
    return 32 * ((N_SLOTS * S + 31) // 32)


def bf16(a):
    """Round binary64/32 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def one_hot(env: np.ndarray, S: int) -> np.ndarray:
    env = np.asarray(env, dtype=np.int64).reshape(-1, N_SLOTS)
    x = np.zeros((env.shape[0], k1_of(S)), dtype=np.float64)
    rows = np.repeat(np.arange(env.shape[0]), N_SLOTS)
    cols = (np.arange(N_SLOTS)[None, :] * S + env).reshape(-1)
    x[rows, cols] = 1.0
    return x


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = GELU_C * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3 * 0.044715 * z * z)


def init_params(S: int, rng: np.random.Generator, mu: float = 0.0, sigma: float = 1.0):
    k1 = k1_of(S)
    return {"W1": rng.uniform(-1, 1, (k1, HID)) * math.sqrt(3.0 / 27.0),
            "b1": np.zeros(HID),
            "W2": rng.uniform(-1, 1, (HID, HID)) * math.sqrt(3.0 / HID),
            "b2": np.zeros(HID),
            "w3": rng.uniform(-1, 1, HID) * math.sqrt(3.0 / HID),
            "b3": np.zeros(1),
            "mu": float(mu), "sigma": float(sigma)}


PARAM_KEYS = ("W1", "b1", "W2", "b2", "w3", "b3")


def forward(p, x, bf16_act: bool = False):
    r = bf16 if bf16_act else (lambda a: a)
    W1, W2, w3 = r(p["W1"]), r(p["W2"]), r(p["w3"])
    z1 = x @ W1 + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ W2 + p["b2"]
    h2 = r(gelu(z2))
    y = h2 @ w3 + p["b3"][0]
    return y, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "W2": W2, "w3": w3}


def predict_ea(p, env, S, bf16_act: bool = False):
    y, _ = forward(p, one_hot(env, S), bf16_act)
    return p["mu"] + p["sigma"] * y


def loss_and_grads(p, x, target_ea, bf16_act: bool = False):
    """MSE on the standardised target and its gradients (plain chain rule)."""
    y, c = forward(p, x, bf16_act)
    t = (np.asarray(target_ea, dtype=np.float64) - p["mu"]) / p["sigma"]
    B = x.shape[0]
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / B
    g = {"w3": c["h2"].T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, c["w3"]) * gelu_grad(c["z2"])
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ c["W2"].T) * gelu_grad(c["z1"])
    g["W1"] = c["x"].T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, g


def adamw_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in PARAM_KEYS:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        p[k] = p[k] * (1.0 - lr * weight_decay)
        m[:] = beta1 * m + (1.0 - beta1) * g[k]
        v[:] = beta2 * v + (1.0 - beta2) * g[k] * g[k]
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return p


GROUPS = ((1, 8), (8, 14), (14, 21), (21, 27))   # slot ranges of the four bond groups


def group_counts(env, S: int) -> np.ndarray:
    """[n][4][S] per-species counts of the four bond groups."""
    env = np.asarray(env).reshape(-1, N_SLOTS)
    return np.stack([np.stack([(env[:, a:b] == s).sum(1) for s in range(S)], 1)
                     for a, b in GROUPS], 1)


def ood_bounds(train_env, S: int) -> dict:
    """The training set's largest group counts and its moving species
    (rows whose slot 0 is the vacancy code are not training rows)."""
    tr = np.asarray(train_env).reshape(-1, N_SLOTS)
    tr = tr[tr[:, 0] != S - 1]
    return {"max": group_counts(tr, S).max(0), "seen": np.unique(tr[:, 0])}


def in_distribution(bounds: dict, env, S: int) -> np.ndarray:
    env = np.asarray(env).reshape(-1, N_SLOTS)
    return np.isin(env[:, 0], bounds["seen"]) & \
        np.all(group_counts(env, S) <= bounds["max"][None], axis=(1, 2))


def barrier_model(p, bounds: dict, oracle, S: int, bf16_act: bool = True):
    """Barriers of the learned model with its pair-model fallback, as a
    function (occ, slots) -> [nv][8] (binary64; +inf for an inadmissible
    jump).  oracle: an akmc_oracle.Oracle of the same lattice (pair barriers
    and slot codes)."""
    def fn(occ, slots):
        _, ea_pair = oracle.rates_sites(slots, occ)
        env = oracle.encode_env_sites(slots, occ).reshape(-1, N_SLOTS)
        ea = ea_pair.reshape(-1).copy()
        use = np.isfinite(ea) & in_distribution(bounds, env, S)
        if use.any():
            ea[use] = predict_ea(p, env[use], S, bf16_act)
        return ea.reshape(-1, 8)
    return fn


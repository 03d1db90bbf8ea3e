"""FP64 reference of the IPPO actor-critic pieces (policy forward, GAE, clipped PPO loss).

TEST INFRASTRUCTURE ONLY (tests, smoke, benchmark baseline).  Plain NumPy in float64,
written from the method: each agent type has its own network (Sec. 4.2: separate
weights per agent type, independent PPO); the network is an MLP
40 -> 256 -> 256 -> (9 policy logits + 1 value) with tanh.  Gradients of the reference
loss come from PyTorch float64 autograd on the same expression (a library primitive),
pinned against central finite differences in the tests.

Parameter layout (flat, float): W1 [40][256] (input-major), b1 [256], W2 [256][256],
b2 [256], W3 [256][10], b3 [10] -> 78,858 values.
"""
from __future__ import annotations

import numpy as np

OBS_DIM, HID, OUT = 40, 256, 10
N_PARAMS = OBS_DIM * HID + HID + HID * HID + HID + HID * OUT + OUT
SLICES = {}
_o = 0
for _name, _shape in (("W1", (OBS_DIM, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
                      ("W3", (HID, OUT)), ("b3", (OUT,))):
    _n = int(np.prod(_shape))
    SLICES[_name] = (_o, _o + _n, _shape)
    _o += _n
assert _o == N_PARAMS == 78858


def unpack(params):
    return {k: params[a:b].reshape(s) for k, (a, b, s) in SLICES.items()}


def xavier_init(rng: np.random.Generator) -> np.ndarray:
    """Glorot-uniform weights, zero biases (float32 parameter vector)."""
    p = np.zeros(N_PARAMS, dtype=np.float32)
    for k, (a, b, s) in SLICES.items():
        if k.startswith("W"):
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            p[a:b] = rng.uniform(-lim, lim, size=b - a).astype(np.float32)
    return p


def mlp_forward(params, obs):
    """Logits [N, 9] and value [N] in float64 (the first n_actions logits are used)."""
    P = unpack(np.asarray(params, dtype=np.float64))
    x = np.asarray(obs, dtype=np.float64)
    h1 = np.tanh(x @ P["W1"] + P["b1"])
    h2 = np.tanh(h1 @ P["W2"] + P["b2"])
    out = h2 @ P["W3"] + P["b3"]
    return out[:, :9], out[:, 9]


def log_softmax(logits, n_actions):
    z = np.asarray(logits, dtype=np.float64)[:, :n_actions]
    m = z.max(axis=1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(axis=1, keepdims=True))


def gae(rewards, values, dones, last_value, gamma, lam):
    """Generalised advantage estimation over a [T, N] rollout.

    delta_t = r_t + gamma * V_{t+1} * (1 - d_t) - V_t, with V_T = last_value;
    A_t = delta_t + gamma * lam * (1 - d_t) * A_{t+1}, A_T = 0; returns R_t = A_t + V_t.
    d_t = 1 when the episode ended at step t (no bootstrap across it)."""
    r = np.asarray(rewards, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    d = np.asarray(dones, dtype=np.float64)
    T = r.shape[0]
    adv = np.zeros_like(r)
    nxt_v = np.asarray(last_value, dtype=np.float64)
    nxt_a = np.zeros_like(nxt_v)
    for t in range(T - 1, -1, -1):
        delta = r[t] + gamma * nxt_v * (1.0 - d[t]) - v[t]
        nxt_a = delta + gamma * lam * (1.0 - d[t]) * nxt_a
        adv[t] = nxt_a
        nxt_v = v[t]
    return adv, adv + v


def action_index(actions, n_actions):
    """The action a sample's log-probability is taken at.  Reading (the paper is silent):
    an action outside [0, n_actions) counts as action 0, the action the env step takes
    for it."""
    a = np.asarray(actions, dtype=np.int64)
    return np.where((a < 0) | (a >= n_actions), 0, a)


def loss_terms(logits, value, actions, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01):
    """The clipped PPO objective from the network outputs of N samples (logits [N, >=
    n_actions], value [N]), float64: (total, policy, value, entropy), each a mean over the
    samples.  ratio = exp(logp - logp_old); policy = -mean(min(ratio A, clip(ratio, 1-eps,
    1+eps) A)); value = 0.5 mean(max((V - R)^2, (V_old + clip(V - V_old, -eps, eps) - R)^2));
    entropy = mean(-sum_a p log p); total = policy + c_v value - c_e entropy."""
    lp = log_softmax(logits, n_actions)
    a = action_index(actions, n_actions)
    logp = lp[np.arange(len(a)), a]
    ratio = np.exp(logp - np.asarray(logp_old, dtype=np.float64))
    A = np.asarray(adv, dtype=np.float64)
    pol = -np.mean(np.minimum(ratio * A, np.clip(ratio, 1 - clip, 1 + clip) * A))
    v = np.asarray(value, dtype=np.float64)
    R = np.asarray(ret, dtype=np.float64)
    vo = np.asarray(v_old, dtype=np.float64)
    vc = vo + np.clip(v - vo, -clip, clip)
    val = 0.5 * np.mean(np.maximum((v - R) ** 2, (vc - R) ** 2))
    ent = np.mean(-(np.exp(lp) * lp).sum(axis=1))
    return pol + c_v * val - c_e * ent, pol, val, ent


def loss_terms_torch(out, actions, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01):
    """``loss_terms`` in torch float64 from the outputs out [N, 10] (logits, then value),
    differentiable in out: the total loss (a 0-d tensor)."""
    import torch
    lp = torch.log_softmax(out[:, :n_actions], dim=1)
    a = torch.tensor(action_index(actions, n_actions))
    logp = lp[torch.arange(len(a)), a]
    ratio = torch.exp(logp - torch.tensor(np.asarray(logp_old, dtype=np.float64)))
    A = torch.tensor(np.asarray(adv, dtype=np.float64))
    pol = -torch.mean(torch.minimum(ratio * A, torch.clamp(ratio, 1 - clip, 1 + clip) * A))
    v = out[:, 9]
    R = torch.tensor(np.asarray(ret, dtype=np.float64))
    vo = torch.tensor(np.asarray(v_old, dtype=np.float64))
    vc = vo + torch.clamp(v - vo, -clip, clip)
    val = 0.5 * torch.mean(torch.maximum((v - R) ** 2, (vc - R) ** 2))
    ent = torch.mean(-(torch.exp(lp) * lp).sum(dim=1))
    return pol + c_v * val - c_e * ent


def ppo_loss_parts(params, obs, actions, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01):
    """Clipped PPO objective of the MLP on one minibatch, float64: returns (total, policy,
    value, entropy) (see loss_terms)."""
    logits, value = mlp_forward(params, obs)
    return loss_terms(logits, value, actions, logp_old, adv, ret, v_old, n_actions, clip, c_v, c_e)


def ppo_loss_and_grad(params, obs, actions, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01):
    """The same loss in torch float64 with its gradient by autograd: (loss, grad[78858])."""
    import torch
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    P = {k: p[a:b].reshape(s) for k, (a, b, s) in SLICES.items()}
    x = torch.tensor(np.asarray(obs, dtype=np.float64))
    h1 = torch.tanh(x @ P["W1"] + P["b1"])
    h2 = torch.tanh(h1 @ P["W2"] + P["b2"])
    out = h2 @ P["W3"] + P["b3"]
    loss = loss_terms_torch(out, actions, logp_old, adv, ret, v_old, n_actions, clip, c_v, c_e)
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()

"""FP64 reference of the recurrent (GRU) actor-critic and its clipped-PPO loss.

TEST INFRASTRUCTURE ONLY (tests, smoke, benchmark baseline).  The paper trains its
agents with a GRU-based network so that recurrence can pick up time-dependent patterns
(Sec. 5.2.1), one network per agent type (Sec. 4.2).  It gives no sizes; the reading
used here:

    e_t   = tanh(x_t W_e + b_e)                                  embedding, 40 -> 128
    r_t   = sigmoid(e_t W_ir + b_ir + h_{t-1} W_hr + b_hr)       reset gate
    u_t   = sigmoid(e_t W_iz + b_iz + h_{t-1} W_hz + b_hz)       update gate
    n_t   = tanh(e_t W_in + b_in + r_t * (h_{t-1} W_hn + b_hn))  candidate
    h_t   = (1 - u_t) * n_t + u_t * h_{t-1}                      hidden state, 128
    out_t = h_t W_o + b_o                                        9 policy logits + 1 value

(the gated recurrent unit of Cho et al. 2014, gates ordered r, u, n as in the common
library form), with h_{t-1} = 0 at an episode's first step (start flag).  The clipped
PPO loss per (step, env) sample is the feed-forward network's (``ppo_ref``), averaged
over the T x m samples of a minibatch of m whole sequences; its gradient flows back
through time.

Plain NumPy float64 for the forward pass; the gradient comes from PyTorch float64
autograd on the same expressions (a library primitive), pinned in the tests against
central finite differences and closed forms.

Parameter layout (flat): W_e [40][128], b_e [128], W_i [128][384] (columns r | u | n),
b_i [384], W_h [128][384], b_h [384], W_o [128][10], b_o [10] -> 105,610 values.
"""
from __future__ import annotations

import numpy as np

OBS_DIM, HID, OUT = 40, 128, 10
G3 = 3 * HID
SLICES = {}
_o = 0
for _name, _shape in (("We", (OBS_DIM, HID)), ("be", (HID,)), ("Wi", (HID, G3)), ("bi", (G3,)),
                      ("Wh", (HID, G3)), ("bh", (G3,)), ("Wo", (HID, OUT)), ("bo", (OUT,))):
    _n = int(np.prod(_shape))
    SLICES[_name] = (_o, _o + _n, _shape)
    _o += _n
N_PARAMS = _o
assert N_PARAMS == 105610


def unpack(params):
    return {k: params[a:b].reshape(s) for k, (a, b, s) in SLICES.items()}


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Glorot-uniform matrices, zero biases (float32 parameter vector)."""
    p = np.zeros(N_PARAMS, dtype=np.float32)
    for k, (a, b, s) in SLICES.items():
        if k.startswith("W"):
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            p[a:b] = rng.uniform(-lim, lim, size=b - a).astype(np.float32)
    return p


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def gru_cell(P, e, h):
    """One step of the gated recurrent unit, float64: (h', r, u, n)."""
    gi = e @ P["Wi"] + P["bi"]
    gh = h @ P["Wh"] + P["bh"]
    r = _sigmoid(gi[:, :HID] + gh[:, :HID])
    u = _sigmoid(gi[:, HID:2 * HID] + gh[:, HID:2 * HID])
    n = np.tanh(gi[:, 2 * HID:] + r * gh[:, 2 * HID:])
    return (1.0 - u) * n + u * h, r, u, n


def forward(params, obs, start, h0):
    """obs [T][m][40], start [T][m] (1 = the episode starts at this step: h_{t-1} = 0),
    h0 [m][128] -> logits [T][m][9], value [T][m], hidden states [T+1][m][128] (h[0] = h0
    as given, h[t+1] after step t)."""
    P = unpack(np.asarray(params, dtype=np.float64))
    x = np.asarray(obs, dtype=np.float64)
    st = np.asarray(start, dtype=bool)
    T, m = x.shape[0], x.shape[1]
    hs = np.zeros((T + 1, m, HID))
    hs[0] = np.asarray(h0, dtype=np.float64)
    outs = np.zeros((T, m, OUT))
    for t in range(T):
        h = np.where(st[t][:, None], 0.0, hs[t])
        e = np.tanh(x[t] @ P["We"] + P["be"])
        hs[t + 1] = gru_cell(P, e, h)[0]
        outs[t] = hs[t + 1] @ P["Wo"] + P["bo"]
    return outs[:, :, :9], outs[:, :, 9], hs


def ppo_loss_parts(params, obs, start, h0, actions, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5,
                   c_e=0.01):
    """Clipped PPO objective over a minibatch of whole sequences [T][m], float64:
    (total, policy, value, entropy), each the mean over the T x m samples (the per-sample
    terms of the feed-forward network's loss, ``ppo_ref.loss_terms``)."""
    from oracle.ppo_ref import loss_terms
    logits, value, _ = forward(params, obs, start, h0)
    T, m = value.shape
    return loss_terms(logits.reshape(T * m, 9), value.reshape(-1), np.asarray(actions).reshape(-1),
                      np.asarray(logp_old).reshape(-1), np.asarray(adv).reshape(-1), np.asarray(ret).reshape(-1),
                      np.asarray(v_old).reshape(-1), n_actions, clip, c_v, c_e)


def ppo_loss_and_grad(params, obs, start, h0, actions, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5,
                      c_e=0.01):
    """The same loss in torch float64, its gradient by autograd through time:
    (loss, grad [N_PARAMS])."""
    import torch
    from oracle.ppo_ref import loss_terms_torch
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    P = {k: p[a:b].reshape(s) for k, (a, b, s) in SLICES.items()}
    x = torch.tensor(np.asarray(obs, dtype=np.float64))
    st = torch.tensor(np.asarray(start, dtype=bool))
    T, m = x.shape[0], x.shape[1]
    h = torch.tensor(np.asarray(h0, dtype=np.float64))
    outs = []
    for t in range(T):
        h = torch.where(st[t][:, None], torch.zeros_like(h), h)
        e = torch.tanh(x[t] @ P["We"] + P["be"])
        gi = e @ P["Wi"] + P["bi"]
        gh = h @ P["Wh"] + P["bh"]
        r = torch.sigmoid(gi[:, :HID] + gh[:, :HID])
        u = torch.sigmoid(gi[:, HID:2 * HID] + gh[:, HID:2 * HID])
        n = torch.tanh(gi[:, 2 * HID:] + r * gh[:, 2 * HID:])
        h = (1 - u) * n + u * h
        outs.append(h @ P["Wo"] + P["bo"])
    out = torch.stack(outs).reshape(T * m, OUT)
    loss = loss_terms_torch(out, np.asarray(actions).reshape(-1), np.asarray(logp_old).reshape(-1),
                            np.asarray(adv).reshape(-1), np.asarray(ret).reshape(-1), np.asarray(v_old).reshape(-1),
                            n_actions, clip, c_v, c_e)
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()

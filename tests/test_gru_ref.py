"""Pins of the FP64 recurrent actor-critic reference (oracle/gru_ref.py).

* The cell against an independent implementation: torch.nn.GRUCell / torch.nn.GRU in
  float64 with the same weights (the library's gated recurrent unit: gates r, z, n).
* Closed forms: all-zero parameters give r = u = 1/2 and n = 0, so h' = h / 2; a large
  positive update-gate bias carries h unchanged; a large negative one with zero
  recurrent weights gives h' = n, a feed-forward layer of e (r = sigmoid(e W_ir + b_ir +
  b_hr), n = tanh(e W_in + b_in + r b_hn)).
* An episode start at step k: the outputs from k on equal a fresh sequence started there.
* The numpy loss equals the torch-float64 loss; autograd's gradient through time equals
  central finite differences of the numpy loss on sampled coordinates of every tensor.
"""
import numpy as np
import pytest
import torch

from oracle import gru_ref as G


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = G.init_params(rng).astype(np.float64) * scale
    for k in ("be", "bi", "bh", "bo"):
        a, b, _ = G.SLICES[k]
        p[a:b] = rng.normal(0, 0.3, size=b - a)
    return p


def test_layout():
    assert G.N_PARAMS == 40 * 128 + 128 + 2 * (128 * 384 + 384) + 128 * 10 + 10
    P = G.unpack(np.arange(G.N_PARAMS, dtype=np.float64))
    assert P["We"].shape == (40, 128) and P["Wi"].shape == (128, 384) and P["bo"][-1] == G.N_PARAMS - 1


def test_cell_matches_the_library_gru():
    p = _params(1)
    P = G.unpack(p)
    rng = np.random.default_rng(2)
    e = rng.normal(0, 1, size=(7, 128))
    h = rng.normal(0, 0.5, size=(7, 128))
    cell = torch.nn.GRUCell(128, 128).double()
    with torch.no_grad():
        cell.weight_ih.copy_(torch.tensor(P["Wi"].T))
        cell.weight_hh.copy_(torch.tensor(P["Wh"].T))
        cell.bias_ih.copy_(torch.tensor(P["bi"]))
        cell.bias_hh.copy_(torch.tensor(P["bh"]))
        ref = cell(torch.tensor(e), torch.tensor(h)).numpy()
    got = G.gru_cell(P, e, h)[0]
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


def test_sequence_matches_the_library_gru():
    p = _params(3)
    P = G.unpack(p)
    rng = np.random.default_rng(4)
    T, m = 9, 5
    x = rng.normal(0, 1, size=(T, m, 40))
    h0 = rng.normal(0, 0.3, size=(m, 128))
    logits, value, hs = G.forward(p, x, np.zeros((T, m), bool), h0)
    gru = torch.nn.GRU(128, 128).double()
    with torch.no_grad():
        gru.weight_ih_l0.copy_(torch.tensor(P["Wi"].T))
        gru.weight_hh_l0.copy_(torch.tensor(P["Wh"].T))
        gru.bias_ih_l0.copy_(torch.tensor(P["bi"]))
        gru.bias_hh_l0.copy_(torch.tensor(P["bh"]))
        emb = torch.tanh(torch.tensor(x) @ torch.tensor(P["We"]) + torch.tensor(P["be"]))
        out, hn = gru(emb, torch.tensor(h0)[None])
        head = (out @ torch.tensor(P["Wo"]) + torch.tensor(P["bo"])).numpy()
    assert np.allclose(hs[1:], out.numpy(), atol=1e-13)
    assert np.allclose(logits, head[:, :, :9], atol=1e-12) and np.allclose(value, head[:, :, 9], atol=1e-12)


def test_cell_closed_forms():
    rng = np.random.default_rng(5)
    e = rng.normal(0, 1, size=(4, 128))
    h = rng.normal(0, 1, size=(4, 128))
    zero = G.unpack(np.zeros(G.N_PARAMS))
    assert np.allclose(G.gru_cell(zero, e, h)[0], 0.5 * h, atol=0, rtol=1e-15)
    p = _params(6)
    a, b, _ = G.SLICES["bi"]
    p[a + 128: a + 256] = 60.0  # update gate saturated open: carry
    assert np.allclose(G.gru_cell(G.unpack(p), e, h)[0], h, atol=1e-20)
    p[a + 128: a + 256] = -60.0  # update gate shut: h' = n
    wa, wb, _ = G.SLICES["Wh"]
    p[wa:wb] = 0.0
    P = G.unpack(p)
    n = np.tanh(e @ P["Wi"][:, 256:] + P["bi"][256:] + 1.0 / (1.0 + np.exp(-(e @ P["Wi"][:, :128] + P["bi"][:128]
                                                                             + P["bh"][:128]))) * P["bh"][256:])
    assert np.allclose(G.gru_cell(P, e, h)[0], n, atol=1e-15)


def test_episode_start_resets_the_state():
    p = _params(7)
    rng = np.random.default_rng(8)
    T, m, k = 10, 3, 4
    x = rng.normal(0, 1, size=(T, m, 40))
    h0 = rng.normal(0, 0.5, size=(m, 128))
    start = np.zeros((T, m), bool)
    start[k, 1] = True
    lg, v, hs = G.forward(p, x, start, h0)
    lg2, v2, _ = G.forward(p, x[k:, 1:2], np.zeros((T - k, 1), bool), np.zeros((1, 128)))
    assert np.allclose(lg[k:, 1], lg2[:, 0], atol=1e-14) and np.allclose(v[k:, 1], v2[:, 0], atol=1e-14)
    # the other envs are unaffected
    lg3, _, _ = G.forward(p, x, np.zeros((T, m), bool), h0)
    assert np.array_equal(lg[:, [0, 2]], lg3[:, [0, 2]])
    assert not np.allclose(lg[k:, 1], lg3[k:, 1])


def _seq_batch(rng, T, m, p, n_act=9):
    x = rng.normal(0, 1, size=(T, m, 40))
    start = np.zeros((T, m), bool)
    start[0] = True
    start[T // 2, 0] = True
    h0 = rng.normal(0, 0.3, size=(m, 128))
    logits, v, _ = G.forward(p, x, start, h0)
    z = logits[:, :, :n_act]
    lp = z - z.max(-1, keepdims=True)
    lp = lp - np.log(np.exp(lp).sum(-1, keepdims=True))
    act = rng.integers(0, n_act, size=(T, m))
    logp = np.take_along_axis(lp, act[:, :, None], -1)[:, :, 0]
    logp_old = logp + rng.normal(0, 0.05, size=(T, m))
    adv = rng.normal(0, 1, size=(T, m))
    ret = v + rng.normal(0, 0.5, size=(T, m))
    v_old = v + rng.uniform(-0.1, 0.1, size=(T, m))
    return x, start, h0, act, logp_old, adv, ret, v_old


def test_numpy_and_torch_losses_agree():
    p = _params(9, 0.8)
    rng = np.random.default_rng(10)
    b = _seq_batch(rng, 6, 4, p)
    parts = G.ppo_loss_parts(p, *b, 9)
    loss, _ = G.ppo_loss_and_grad(p, *b, 9)
    assert abs(parts[0] - loss) <= 1e-12 * max(1.0, abs(loss))


def test_gradient_through_time_matches_finite_differences():
    p = _params(11, 0.8)
    rng = np.random.default_rng(12)
    b = _seq_batch(rng, 5, 3, p)
    _, g = G.ppo_loss_and_grad(p, *b, 9)
    h = 1e-6
    checked = 0
    for k, (a, e, _) in G.SLICES.items():
        for j in rng.choice(np.arange(a, e), size=6, replace=False):
            q = p.copy()
            q[j] += h
            lp = G.ppo_loss_parts(q, *b, 9)[0]
            q[j] -= 2 * h
            lm = G.ppo_loss_parts(q, *b, 9)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[j]) <= 1e-7 + 1e-5 * abs(g[j]), (k, j, fd, g[j])
            checked += 1
    assert checked == 6 * len(G.SLICES)
    # the recurrent weights do receive gradient through time
    a, e, _ = G.SLICES["Wh"]
    assert np.abs(g[a:e]).max() > 1e-6

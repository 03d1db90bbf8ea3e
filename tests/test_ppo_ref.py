"""Pins of the FP64 IPPO reference (oracle/ppo_ref.py).

* The numpy loss and the torch-float64 autograd loss are independent implementations of
  the same expression: they must agree, and autograd's gradient must agree with central
  finite differences of the numpy loss (away from the clip kinks).
* Closed forms: ratio 1 and V = V_old give policy = -mean(A) and value =
  0.5 mean((V - R)^2); a zero output layer gives uniform logits, entropy log(n).
* GAE: lambda = 0 gives A = delta; gamma = lambda = 1 without dones gives the reverse
  cumulative reward plus the bootstrap minus V; a done stops the recursion.
"""
import numpy as np
import pytest

from oracle import ppo_ref as R


def batch(rng, m, n_act, params, ratio_noise=0.05, big=False):
    obs = rng.normal(0, 1, size=(m, 40)).astype(np.float32)
    logits, v = R.mlp_forward(params, obs)
    lp = R.log_softmax(logits, n_act)
    act = rng.integers(0, n_act, size=m)
    logp = lp[np.arange(m), act]
    logp_old = logp + rng.normal(0, ratio_noise, size=m)
    if big:  # some samples deep in the clipped regions (away from the kinks)
        k = m // 4
        logp_old[:k] = logp[:k] - np.log(1.6)
        logp_old[k:2 * k] = logp[k:2 * k] - np.log(0.5)
    adv = rng.normal(0, 1, size=m)
    ret = v + rng.normal(0, 0.5, size=m)
    v_old = v + rng.choice([-1, 1], size=m) * rng.uniform(0.0, 0.15, size=m)
    if big:
        k = m // 4
        v_old[2 * k:3 * k] = v[2 * k:3 * k] + rng.choice([-1, 1], size=k) * rng.uniform(0.3, 0.6, size=k)
    return obs, act, logp_old.astype(np.float32), adv.astype(np.float32), ret.astype(np.float32), v_old.astype(np.float32)


def test_parameter_layout_and_init():
    rng = np.random.default_rng(0)
    p = R.xavier_init(rng)
    assert p.shape == (78858,)
    P = R.unpack(p)
    assert P["W1"].shape == (40, 256) and P["W3"].shape == (256, 10)
    for k, (fi, fo) in (("W1", (40, 256)), ("W2", (256, 256)), ("W3", (256, 10))):
        lim = np.sqrt(6 / (fi + fo))
        assert np.abs(P[k]).max() <= lim
        assert abs(P[k].var() - lim * lim / 3) < 0.1 * lim * lim / 3
    assert not P["b1"].any() and not P["b3"].any()


@pytest.mark.parametrize("n_act,big", [(9, False), (3, True), (9, True)])
def test_autograd_matches_numpy_loss_and_finite_differences(n_act, big):
    rng = np.random.default_rng(n_act + 10 * big)
    params = R.xavier_init(rng).astype(np.float64)
    params[R.SLICES["b1"][0]:R.SLICES["b1"][1]] = rng.normal(0, 0.1, 256)
    params[R.SLICES["b3"][0]:R.SLICES["b3"][1]] = rng.normal(0, 0.1, 10)
    b = batch(rng, 48, n_act, params, big=big)
    tot, pol, val, ent = R.ppo_loss_parts(params, *b, n_act)
    loss, grad = R.ppo_loss_and_grad(params, *b, n_act)
    assert abs(loss - tot) <= 1e-12 * max(1.0, abs(tot))
    idx = np.concatenate([rng.choice(np.arange(a, bb), size=min(25, bb - a), replace=False)
                          for a, bb, _ in R.SLICES.values()])
    h = 1e-6
    fd = np.empty(len(idx))
    for j, i in enumerate(idx):
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd[j] = (R.ppo_loss_parts(pp, *b, n_act)[0] - R.ppo_loss_parts(pm, *b, n_act)[0]) / (2 * h)
    err = np.linalg.norm(grad[idx] - fd) / np.linalg.norm(fd)
    assert err < 1e-7


def test_loss_closed_forms():
    rng = np.random.default_rng(3)
    params = R.xavier_init(rng).astype(np.float64)
    obs = rng.normal(size=(32, 40))
    logits, v = R.mlp_forward(params, obs)
    lp = R.log_softmax(logits, 9)
    act = rng.integers(0, 9, size=32)
    A = rng.normal(size=32)
    Rt = rng.normal(size=32)
    tot, pol, val, ent = R.ppo_loss_parts(params, obs, act, lp[np.arange(32), act], A, Rt, v, 9)
    assert np.isclose(pol, -A.mean(), rtol=1e-12)
    assert np.isclose(val, 0.5 * np.mean((v - Rt) ** 2), rtol=1e-12)
    assert np.isclose(tot, pol + 0.5 * val - 0.01 * ent, rtol=1e-12)
    # zero output layer: uniform policy, entropy log(n)
    p0 = params.copy()
    a, b, _ = R.SLICES["W3"]
    p0[a:b] = 0
    for n in (3, 9):
        _, _, _, e = R.ppo_loss_parts(p0, obs, act % n, np.full(32, -np.log(n)), A, Rt, np.zeros(32), n)
        assert np.isclose(e, np.log(n), rtol=1e-12)


def test_gae_special_cases():
    rng = np.random.default_rng(4)
    T, N = 12, 5
    r, v = rng.normal(size=(T, N)), rng.normal(size=(T, N))
    last = rng.normal(size=N)
    d = np.zeros((T, N))
    adv, ret = R.gae(r, v, d, last, 0.9, 0.0)
    vn = np.vstack([v[1:], last])
    assert np.allclose(adv, r + 0.9 * vn - v, rtol=0, atol=1e-12)
    adv, ret = R.gae(r, v, d, last, 1.0, 1.0)
    expect = np.cumsum(r[::-1], axis=0)[::-1] + last - v
    assert np.allclose(adv, expect, atol=1e-12)
    assert np.allclose(ret, adv + v, atol=1e-12)
    d[5, :] = 1  # the episode ends at step 5: no bootstrap from step 6, recursion stops
    adv, _ = R.gae(r, v, d, last, 1.0, 1.0)
    assert np.allclose(adv[5], r[5] - v[5], atol=1e-12)
    assert np.allclose(adv[:6], np.cumsum(r[5::-1], axis=0)[::-1] - v[:6], atol=1e-12)


def test_out_of_range_actions_count_as_action_zero():
    """Reading shared with the env step: an action outside [0, n_actions) is action 0,
    in the loss and in its gradient."""
    rng = np.random.default_rng(11)
    p = R.xavier_init(rng)
    obs, act, lpo, adv, ret, vo = batch(rng, 24, 9, p)
    act = act.copy()
    act[:6] = 0
    bad = act.copy()
    bad[:3] = -1
    bad[3:6] = 9
    a = R.ppo_loss_parts(p, obs, act, lpo, adv, ret, vo, 9)
    b = R.ppo_loss_parts(p, obs, bad, lpo, adv, ret, vo, 9)
    assert np.allclose(a, b, rtol=0, atol=0)
    la, ga = R.ppo_loss_and_grad(p, obs, act, lpo, adv, ret, vo, 9)
    lb, gb = R.ppo_loss_and_grad(p, obs, bad, lpo, adv, ret, vo, 9)
    assert la == lb and np.array_equal(ga, gb)

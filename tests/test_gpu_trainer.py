"""Learned-policy rollouts (policy forward + env step per step), their HIP-graph
capture, and the IPPO update loop."""
import numpy as np
import pytest
import torch

from paper_2511_02136_amd import synth
from oracle import OracleEnvs
from helpers import subset_stream
from gpu_compare import assert_same_outputs

pytestmark = pytest.mark.gpu


def make_trainer(n_envs=256, n_steps=16, seed=3, **kw):
    from paper_2511_02136_amd.lob import LobEnv, DeviceStream
    from paper_2511_02136_amd.trainer import IppoTrainer
    w = synth.WORKLOADS["ippo4096"].scaled(n_envs=n_envs, n_steps=n_steps)
    s = synth.generate(w)
    env = LobEnv(s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    ds = DeviceStream.from_host(s)
    book = {k: torch.from_numpy(v).cuda() for k, v in s.book.items()}
    return w, s, IppoTrainer(env, ds, book, n_steps, seed=seed, param_seed=seed, **kw)


def snapshot(tr):
    keys = ("n_trades", "fills", "reward", "obs", "done")
    out = {k: tr.out[k].clone() for k in keys}
    out.update({k: v.clone() for k, v in tr.pol.items()})
    out["obs_in"] = tr.obs.clone()
    return out


def test_graph_replays_equal_eager_rollout():
    w, s, tr = make_trainer()
    tr.rollout(use_graph=True)  # builds the graph (its warm-up pass bumps the counter too)
    tr.epoch.fill_(10)
    tr.rollout(use_graph=False)
    torch.cuda.synchronize()
    ref = snapshot(tr)
    for rep in range(3):
        tr.epoch.fill_(10)
        tr.rollout(use_graph=True)
        torch.cuda.synchronize()
        got = snapshot(tr)
        for k in ref:
            assert torch.equal(got[k], ref[k]), (rep, k)
        # eager work between replays
        tr.epoch.fill_(20)
        tr.rollout(use_graph=False)
        torch.cuda.synchronize()
    # a different epoch draws different actions
    assert not torch.equal(snapshot(tr)["actions"], ref["actions"])


def test_learned_policy_rollout_env_parity():
    """The env part of a learned-policy rollout is bit-exact vs the oracle fed the
    recorded actions (the policy itself is fp32 MFMA, checked separately)."""
    w, s, tr = make_trainer(n_envs=96, n_steps=12, seed=5)
    tr.rollout(use_graph=True)
    torch.cuda.synchronize()
    acts = tr.pol["actions"].cpu().numpy()
    o = OracleEnvs(s.caps, w.max_cap, synth.agent_kinds(w.agents), w.ep_len, w.seed)
    o.reset(s.book)
    ref = o.step(s, n_steps=12, actions=acts)
    got = {k: tr.out[k] for k in ("n_trades", "fills", "reward", "obs", "done")}
    got["actions"] = None
    r = dict(ref)
    r["trades"] = None
    assert_same_outputs(got, r, 12, what="learned")
    n = ref["n_trades"].sum(0)
    goff = tr.out["trade_off"].cpu().numpy()
    for e in range(0, 96, 5):
        a = tr.out["trades"][goff[e]: goff[e] + n[e]].cpu().numpy()
        b = ref["trades"][ref["trade_off"][e]: ref["trade_off"][e] + n[e]]
        assert np.array_equal(a, b), e


def test_update_runs_and_changes_the_policy():
    w, s, tr = make_trainer(n_envs=128, n_steps=16, seed=7)
    tr.rollout(use_graph=True)
    before = tr.params.detach().clone()
    st = tr.update()
    torch.cuda.synchronize()
    assert np.isfinite(st["loss"])
    assert st["minibatches"] == tr.epochs * tr.minibatches
    assert not torch.equal(before, tr.params.detach())
    assert torch.isfinite(tr.params).all()


@pytest.mark.parametrize("network", ["mlp", "gru"])
def test_update_on_agent_streams_equals_one_stream(network):
    """The update issues each agent's fused loss calls on a stream of its own; with the
    same rollout and the same minibatch shuffles the parameters after the update are
    bit-identical to an update with every call on the current stream."""
    res = []
    for concurrent in (True, False):
        w, s, tr = make_trainer(n_envs=128, n_steps=16, seed=11, network=network, agent_streams=concurrent)
        tr.rollout(use_graph=False)
        torch.manual_seed(5)
        st = tr.update()
        torch.cuda.synchronize()
        res.append((st["loss"], tr.params.detach().clone()))
    assert res[0][0] == res[1][0]
    assert torch.equal(res[0][1], res[1][1])


def test_full_size_learned_policy_rollout_parity():
    """The IPPO workload's rollout at full size (4096 envs x 128 steps, actions sampled by
    the policy kernel) in the form the benchmark times, a replay of the captured HIP
    graph: 48 sampled envs replayed by the oracle with the recorded actions are
    bit-exact (trades, fills, rewards, observations, done)."""
    w, s, tr = make_trainer(n_envs=4096, n_steps=128, seed=9)
    assert w == synth.WORKLOADS["ippo4096"]
    print("\n[parity] full-size ippo4096 learned-policy rollout", flush=True)
    tr.rollout(use_graph=True)
    tr.rollout(use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(w.n_envs, size=48, replace=False))
    hs, book, caps = subset_stream(s, sample)
    acts = np.ascontiguousarray(tr.pol["actions"].cpu().numpy()[:, :, sample])
    assert acts.min() >= 0 and acts.max() <= 8
    o = OracleEnvs(caps, w.max_cap, synth.agent_kinds(w.agents), w.ep_len, w.seed, env_ids=sample)
    o.reset(book)
    ref = o.step(hs, n_steps=w.n_steps, actions=acts)
    got = {k: tr.out[k] for k in ("n_trades", "fills", "reward", "obs", "done")}
    got["actions"] = None
    r = dict(ref)
    r["trades"] = None
    assert_same_outputs(got, r, w.n_steps, envs=sample, what="ippo4096")
    goff = tr.out["trade_off"].cpu().numpy()
    for j, e in enumerate(sample):
        cnt = int(ref["n_trades"][:, j].sum())
        a = tr.out["trades"][goff[e]: goff[e] + cnt].cpu().numpy()
        b = ref["trades"][ref["trade_off"][j]: ref["trade_off"][j] + cnt]
        assert np.array_equal(a, b), e

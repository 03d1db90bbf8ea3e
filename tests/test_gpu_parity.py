"""Parity of the HIP path (through the C-ABI) with the CPU oracle, element by element.

Books, trades, fills, counters and state must be bit-identical; rewards and
observations are compared bit for bit as well (both sides evaluate the same double
expression with contraction off and round once; observations are exact integers).
"""
import numpy as np
import pytest
import torch

from paper_2511_02136_amd import synth
from oracle import OracleEnvs
from helpers import hand_stream, hand_book, msg, subset_stream
from gpu_compare import assert_same_outputs, assert_same_books, assert_same_state

pytestmark = pytest.mark.gpu

LIMIT, PARTIAL_CANCEL, DELETE, MARKET = 1, 2, 3, 4
BUY, SELL = 0, 1


def _lob():
    from paper_2511_02136_amd.lob import LobEnv, DeviceStream
    return LobEnv, DeviceStream


def oracle_for(stream_like, book, caps, max_cap, agents, ep_len, seed, env_ids=None, **kw):
    o = OracleEnvs(caps, max_cap, synth.agent_kinds(agents), ep_len, seed, env_ids=env_ids, **kw)
    o.reset(book)
    return o


def gpu_env(caps, max_cap, agents, ep_len, seed, book, **kw):
    LobEnv, _ = _lob()
    env = LobEnv(caps, max_cap, agents, ep_len, seed, **kw)
    env.reset(book)
    return env


def run_steps(env, ds, n_steps, actions, trade_off):
    """n_steps plain lob_step calls appending into one set of outputs."""
    out = env._alloc_out(n_steps, True, True, trade_off, ds)
    cursor = torch.zeros(env.n_envs, dtype=torch.int64, device=env.device)
    for t in range(n_steps):
        view = {k: (v[t:t + 1] if k not in ("trades", "trade_off") and v is not None else v) for k, v in out.items()}
        a = None if actions is None else actions[t]
        env.step(ds, a, out=view, cursor=cursor)
    return out


def parity_case(w: synth.Workload, n_steps: int, mode: str, given_actions=False, kw=None, name=""):
    kw = kw or {}
    print(f"\n[parity] {name or w.name} envs={w.n_envs} steps={n_steps} mode={mode}", flush=True)
    _, DeviceStream = _lob()
    s = synth.generate(w)
    acts = None
    if given_actions:
        rng = np.random.default_rng(w.seed)
        kinds = synth.agent_kinds(w.agents)
        acts = np.stack([rng.integers(-1, 10 if k != 2 else 4, size=(n_steps, w.n_envs)) for k in kinds], 1).astype(np.int32)
    o = oracle_for(s, s.book, s.caps, w.max_cap, w.agents, w.ep_len, w.seed, **kw)
    ref = o.step(s, n_steps=n_steps, actions=acts)
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book, **kw)
    ds = DeviceStream.from_host(s)
    toff = torch.from_numpy(ref["trade_off"]).cuda()
    ta = None if acts is None else torch.from_numpy(acts).cuda()
    if mode == "rollout":
        got = env.rollout(ds, n_steps, actions=ta, trade_off=toff)
    else:
        got = run_steps(env, ds, n_steps, ta, toff)
    torch.cuda.synchronize()
    assert_same_outputs(got, ref, n_steps, what=name)
    assert_same_books(env.books(), o.books(), what=name)
    assert_same_state(env.state(), o.state(), what=name)
    obs_now = env.observe().cpu().numpy()
    assert np.array_equal(obs_now.view(np.int32), o.observe().view(np.int32))
    return env, o


SMALL = [
    synth.Workload("replay_only", n_envs=3, n_steps=20, msgs_per_step=100, cap=100, seed=31),
    synth.Workload("exec_mm", n_envs=64, n_steps=16, msgs_per_step=100, cap=100, agents=("exec", "mm"), seed=32),
    synth.Workload("uneven", n_envs=96, n_steps=12, msgs_range=(1, 400), cap_choices=(50, 100, 200, 400),
                   agents=("exec", "mm"), seed=33),
    synth.Workload("three_agents_cap1000", n_envs=24, n_steps=10, msgs_per_step=400, burst_pct=10, burst_extra=480,
                   cap=1000, agents=("exec", "mm", "dir"), seed=34),
    synth.Workload("row_edges", n_envs=40, n_steps=12, msgs_range=(50, 300), cap_choices=(1, 2, 63, 64, 65, 127, 128, 129),
                   agents=("mm", "dir"), seed=35, snapshot_fill_pct=100),
    synth.Workload("tiny_books", n_envs=32, n_steps=16, msgs_per_step=60, cap=3, agents=("exec", "mm", "dir", "mm"),
                   seed=36, snapshot_fill_pct=100),
    # replayed executions of named orders (some of agents' orders) and ignored messages
    synth.Workload("executions", n_envs=48, n_steps=12, msgs_range=(20, 300), cap_choices=(50, 100, 200),
                   agents=("exec", "mm"), seed=38, exec_pct=12, ignored_pct=4),
    # envs that replay no message at all beside envs with one or two per step: empty
    # steps, agents acting alone on the reset book
    synth.Workload("empty_steps", n_envs=40, n_steps=16, msgs_range=(0, 2), cap_choices=(3, 50, 100),
                   agents=("exec", "mm", "dir"), seed=39),
    # the largest capacity the library accepts (16 rows of 64 orders per side), books full
    # from the start: the last row, evictions and the time lookup of every row
    synth.Workload("max_cap", n_envs=8, n_steps=6, msgs_per_step=400, cap=1024, agents=("exec", "mm"),
                   seed=37, snapshot_fill_pct=100),
    # one env alone: a plan and a queue of one
    synth.Workload("single_env", n_envs=1, n_steps=24, msgs_per_step=150, cap=50, agents=("exec", "mm"), seed=40),
]


@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
@pytest.mark.parametrize("mode", ["step", "rollout"])
def test_parity_small(w, mode):
    parity_case(w, w.n_steps, mode, name=f"{w.name}/{mode}")


@pytest.mark.parametrize("w", SMALL[1:4], ids=lambda w: w.name)
def test_parity_given_actions(w):
    parity_case(w, w.n_steps, "rollout", given_actions=True, name=f"{w.name}/given")


def test_parity_reward_weights():
    w = synth.Workload("weights", n_envs=48, n_steps=12, msgs_per_step=80, cap=64, agents=("mm", "exec", "mm"), seed=37)
    parity_case(w, 12, "rollout", kw=dict(exec_penalty=0.07, mm_lambda=0.3, mm_rho=0.02, exec_task=60, exec_q0=3),
                name="weights")


@pytest.mark.parametrize("mode", ["step", "rollout"])
def test_parity_buysell_market_maker(mode):
    """The market maker with the buy-sell reward (Eq. 4) and the quadratic inventory
    penalty, next to the Spooner market maker and the execution agent."""
    w = synth.Workload("buysell", n_envs=40, n_steps=10, msgs_per_step=80, cap=64,
                       agents=("mm_buysell", "exec", "mm"), seed=39)
    parity_case(w, 10, mode, kw=dict(mm_lambda=0.3, mm_rho=0.02, exec_task=60, exec_q0=3), name=f"buysell/{mode}")


def test_rollout_resumes_across_calls():
    """128 = 5 + 7 steps in two rollouts equals the oracle's 12 steps (state carried)."""
    _, DeviceStream = _lob()
    w = synth.Workload("resume", n_envs=50, n_steps=12, msgs_range=(1, 200), cap_choices=(50, 100), agents=("exec", "mm"),
                       seed=38)
    s = synth.generate(w)
    o = oracle_for(s, s.book, s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    ref1 = o.step(s, n_steps=5)
    ref2 = o.step(s, n_steps=7)
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    ds = DeviceStream.from_host(s)
    g1 = env.rollout(ds, 5, trade_off=torch.from_numpy(ref1["trade_off"]).cuda())
    g2 = env.rollout(ds, 7, trade_off=torch.from_numpy(ref2["trade_off"]).cuda())
    assert_same_outputs(g1, ref1, 5, what="resume/1")
    assert_same_outputs(g2, ref2, 7, what="resume/2")
    assert_same_books(env.books(), o.books(), what="resume")


def test_hand_scenario_on_gpu():
    _, DeviceStream = _lob()
    snap = hand_book([([[99, 10, 1, 0, 1, 0]], [[101, 10, 2, 0, 1, 5]])], 10)
    steps = [[[msg(MARKET, BUY, 0, 15, 50, 0, 2, 0)], [msg(LIMIT, BUY, 103, 5, 51, 0, 2, 10)]]]
    hs = hand_stream(steps)
    kw = dict(exec_task=6, exec_q0=4, mm_q=10, exec_penalty=0.5)
    o = oracle_for(hs, snap, np.array([10]), 10, ("exec", "mm"), 2, 5, **kw)
    acts = np.array([[[4], [1]], [[8], [0]]], dtype=np.int32)
    ref = o.step(hs, n_steps=2, actions=acts)
    env = gpu_env(np.array([10]), 10, ("exec", "mm"), 2, 5, snap, **kw)
    got = env.rollout(DeviceStream.from_host(hs), 2, actions=torch.from_numpy(acts).cuda(),
                      trade_off=torch.from_numpy(ref["trade_off"]).cuda())
    assert_same_outputs(got, ref, 2, what="hand")
    assert got["reward"][:, :, 0].cpu().tolist() == [[4.0, 1.75], [6.0, -2.0]]


def test_sweeps_across_rows_and_empty_sides():
    """Market and limit orders that sweep several 64-slot rows; books emptied and
    refilled; malformed messages; an empty side at reset."""
    _, DeviceStream = _lob()
    asks = [[1000 + k // 3, 1 + k % 5, 10 + k, 0, 1, k] for k in range(300)]
    bids1 = [[990 - k // 4, 1 + k % 3, 20000 + k, 0, 1, k] for k in range(70)]
    snap = hand_book([([], asks), (bids1, [])], 320)
    e0 = [
        [msg(MARKET, BUY, 0, 200, 5000), msg(LIMIT, BUY, 1030, 400, 5001), msg(9, BUY, 1, 1, 1),
         msg(LIMIT, SELL, 1000, 0, 5002)],
        [msg(MARKET, SELL, 0, 10_000, 5003), msg(PARTIAL_CANCEL, SELL, 0, 0, 200), msg(DELETE, SELL, 0, 0, 250)],
        [msg(LIMIT, SELL, 1100, 3, 5004 + k) for k in range(150)] + [msg(LIMIT, BUY, 1200, 100, 6000)],
    ]
    e1 = [[msg(LIMIT, SELL, 999, 50, 7000)], [msg(MARKET, BUY, 0, 5, 7001)], [msg(DELETE, BUY, 0, 0, 10)]]
    hs = hand_stream([e0, e1])
    caps = np.array([320, 100])
    for agents in ((), ("mm", "exec")):
        o = oracle_for(hs, snap, caps, 320, agents, 3, 9)
        ref = o.step(hs, n_steps=3)
        env = gpu_env(caps, 320, agents, 3, 9, snap)
        got = env.rollout(DeviceStream.from_host(hs), 3, trade_off=torch.from_numpy(ref["trade_off"]).cuda())
        assert_same_outputs(got, ref, 3, what=f"sweeps{agents}")
        assert_same_books(env.books(), o.books(), what=f"sweeps{agents}")
        assert_same_state(env.state(), o.state(), what=f"sweeps{agents}")


@pytest.mark.parametrize("mode", ["rollout", "step"])
def test_more_than_a_row_of_agent_orders(mode):
    """An agent alone at the best ask, its order there partly filled every step, tops the
    level up with a new order each step until it rests more than 64 orders (more than the
    agents' orders a step keeps in registers): its resting quantity is measured and the
    cancel walk runs over all of them, cancelling the excess from the newest ones when the
    desired quantity falls, and deleting them all when the level moves away; in the second
    env a second agent's order rests below them on the same side."""
    _, DeviceStream = _lob()
    T, T1 = 110, 89
    bids = [[990, 5, 1, 0, 1, 0]]
    asks = [[1000, 1, 2, 0, 1, 0]]
    snap = hand_book([(bids, asks), (bids, asks)], 200)
    # every step one market buy of 1: it fills the ask side's first order in priority
    steps = [[[msg(MARKET, BUY, 0, 1, 100 + t)] for t in range(T)] for _ in range(2)]
    hs = hand_stream(steps)
    caps = np.array([200, 200])
    kw = dict(exec_task=100_000, exec_q0=300, mm_q=7)
    # exec: one level at the best ask (action 4), at twice the quantity (action 6) for
    # steps 70-73, the level two ticks up (action 5) at step 90; mm: nothing in env 0,
    # from step 20 on in env 1 an ask two ticks above the best ask (action 5)
    acts = np.zeros((T, 2, 2), np.int32)
    acts[:, 0, :] = 4
    acts[70:74, 0, :] = 6
    acts[90, 0, :] = 5
    acts[20:, 1, 1] = 5
    o = oracle_for(hs, snap, caps, 200, ("exec", "mm"), T, 17, **kw)
    ref1 = o.step(hs, n_steps=T1, actions=acts[:T1])
    b1 = o.books()
    for e in range(2):
        n = int(b1["n"][e, 1])
        assert int((b1["tid"][e, 1, :n] == 1).sum()) > 64
    ref2 = o.step(hs, n_steps=T - T1, actions=acts[T1:])
    env = gpu_env(caps, 200, ("exec", "mm"), T, 17, snap, **kw)
    ds = DeviceStream.from_host(hs)
    for (t0, n, ref) in ((0, T1, ref1), (T1, T - T1, ref2)):
        toff = torch.from_numpy(ref["trade_off"]).cuda()
        a = torch.from_numpy(np.ascontiguousarray(acts[t0:t0 + n])).cuda()
        got = env.rollout(ds, n, actions=a, trade_off=toff) if mode == "rollout" else run_steps(env, ds, n, a, toff)
        assert_same_outputs(got, ref, n, what=f"agent orders/{mode}/{t0}")
    assert_same_books(env.books(), o.books(), what=f"agent orders/{mode}")
    assert_same_state(env.state(), o.state(), what=f"agent orders/{mode}")


@pytest.mark.parametrize("mode", ["rollout", "step"])
def test_sweeps_of_a_row_or_more_that_stop(mode):
    """Incoming orders that trade against 64 or more resting orders: exactly one row of
    crossing orders and then an order that does not cross; a row and a part; an order
    filled exactly by the 64th order; a market order across three rows; two full rows
    and then a price that stops the sweep (remainder rests)."""
    _, DeviceStream = _lob()
    B = [
        ([], [[1000, 2, 100 + k, 0, 1, k] for k in range(64)] + [[1050, 1, 300 + k, 0, 1, k] for k in range(20)]),
        ([], [[1000, 2, 100 + k, 0, 1, k] for k in range(80)] + [[1050, 1, 300 + k, 0, 1, k] for k in range(20)]),
        ([[990, 3, 100 + k, 0, 1, k] for k in range(64)] + [[980, 1, 300 + k, 0, 1, k] for k in range(10)], []),
        ([], [[1000 + k // 10, 1, 100 + k, 0, 1, k] for k in range(130)]),
        ([], [[1000, 1, 100 + k, 0, 1, k] for k in range(128)] + [[1100, 1, 300 + k, 0, 1, k] for k in range(5)]),
    ]
    snap = hand_book(B, 200)
    steps = [
        [[msg(LIMIT, BUY, 1020, 500, 9000)], [msg(MARKET, SELL, 0, 400, 9001)]],
        [[msg(LIMIT, BUY, 1020, 500, 9000)], [msg(LIMIT, SELL, 1000, 10, 9001)]],
        [[msg(LIMIT, SELL, 985, 192, 9000)], [msg(LIMIT, SELL, 985, 5, 9001)]],
        [[msg(MARKET, BUY, 0, 129, 9000)], [msg(MARKET, BUY, 0, 5, 9001)]],
        [[msg(LIMIT, BUY, 1000, 200, 9000)], [msg(MARKET, SELL, 0, 100, 9001)]],
    ]
    hs = hand_stream(steps)
    caps = np.full(len(B), 200)
    for agents in ((), ("exec", "mm")):
        o = oracle_for(hs, snap, caps, 200, agents, 2, 5)
        acts = np.zeros((2, len(agents), len(B)), np.int32)
        ref = o.step(hs, n_steps=2, actions=acts if agents else None)
        env = gpu_env(caps, 200, agents, 2, 5, snap)
        ds = DeviceStream.from_host(hs)
        toff = torch.from_numpy(ref["trade_off"]).cuda()
        a = torch.from_numpy(acts).cuda() if agents else None
        if mode == "rollout":
            got = env.rollout(ds, 2, actions=a, trade_off=toff)
        else:
            got = run_steps(env, ds, 2, a, toff)
        assert_same_outputs(got, ref, 2, what=f"deep sweeps {agents}")
        assert_same_books(env.books(), o.books(), what=f"deep sweeps {agents}")
        assert_same_state(env.state(), o.state(), what=f"deep sweeps {agents}")
    # the sweeps did trade across rows: 64, 80, 64, 129 and 128 resting orders
    assert ref["n_trades"][0].tolist() == [64, 80, 64, 129, 128]


def test_trade_region_overflow_is_counted():
    _, DeviceStream = _lob()
    w = synth.Workload("overflow", n_envs=16, n_steps=8, msgs_per_step=100, cap=100, agents=("exec", "mm"), seed=39)
    s = synth.generate(w)
    small = np.concatenate([[0], np.cumsum(np.full(16, 5))]).astype(np.int64)
    o = oracle_for(s, s.book, s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    ref = o.step(s, n_steps=8, trade_off=small)
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    got = env.rollout(DeviceStream.from_host(s), 8, trade_off=torch.from_numpy(small).cuda())
    assert_same_outputs(got, ref, 8, what="overflow")
    st = o.state()
    assert st["counters"][:, 9].sum() > 0
    assert_same_state(env.state(), st, what="overflow")


def test_call_order_errors():
    LobEnv, DeviceStream = _lob()
    from paper_2511_02136_amd.lob import LobError
    w = synth.Workload("order", n_envs=4, n_steps=2, msgs_per_step=10, cap=16, agents=("mm",), seed=40)
    s = synth.generate(w)
    env = LobEnv(s.caps, 16, ("mm",), 2, 1)
    ds = DeviceStream.from_host(s)
    with pytest.raises(LobError):
        env.step(ds)  # not reset
    env.reset(s.book)
    env.rollout(ds, 2)
    with pytest.raises(LobError):
        env.step(ds)  # episode over
    with pytest.raises(LobError):
        LobEnv(np.array([2000]), 2000, (), 2, 1)  # capacity beyond the supported maximum


@pytest.mark.parametrize("name", ["uniform4096", "uneven8192"])
def test_full_size_sampled_parity(name):
    """Full-size workload in the launch configuration the benchmark times (persistent
    rollout over all steps); a sample of envs is replayed on the oracle with the
    recorded actions of the GPU and the same env ids."""
    _, DeviceStream = _lob()
    w = synth.WORKLOADS[name]
    print(f"\n[parity] full-size {name}", flush=True)
    s = synth.generate(w)
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    ds = DeviceStream.from_host(s)
    got = env.rollout(ds, w.n_steps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(w.n_envs, size=48, replace=False))
    hs, book, caps = subset_stream(s, sample)
    o = oracle_for(hs, book, caps, w.max_cap, w.agents, w.ep_len, w.seed, env_ids=sample)
    acts = got["actions"].cpu().numpy()[:, :, sample]
    ref = o.step(hs, n_steps=w.n_steps, actions=np.ascontiguousarray(acts))
    # the GPU's trade regions differ from the subset's; compare records by content
    g = {k: v for k, v in got.items()}
    goff = got["trade_off"].cpu().numpy()
    for j, e in enumerate(sample):
        cnt = int(ref["n_trades"][:, j].sum())
        gt = got["trades"][goff[e]: goff[e] + cnt].cpu().numpy()
        assert np.array_equal(gt, ref["trades"][ref["trade_off"][j]: ref["trade_off"][j] + cnt]), e
    g["trades"] = None
    ref = dict(ref)
    ref["trades"] = None
    assert_same_outputs(g, ref, w.n_steps, envs=sample, what=name)
    assert_same_books(env.books(), o.books(), envs=sample, what=name)
    assert_same_state(env.state(), o.state(), envs=sample, what=name)
    # random actions are uniform over each agent's action set
    a = got["actions"].cpu().numpy()
    assert a.min() >= 0 and a[:, 0].max() <= 8


def test_large16384_full_size_sampled_parity():
    """The large workload at full size (16384 envs, capacity 1000, 400 messages per step
    with 10% burst steps, three agents, 256 steps: about 1.9e9 messages) in the persistent
    launch.  Trade records are kept for the sampled envs only: every other env gets an
    empty region, so its trades are counted (trade_overflow) but not stored."""
    _, DeviceStream = _lob()
    w = synth.WORKLOADS["large16384"]
    print(f"\n[parity] full-size {w.name}", flush=True)
    s = synth.generate(w)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(w.n_envs, size=24, replace=False))
    hs, book, caps = subset_stream(s, sample)
    msgs = s.off[sample, w.n_steps] - s.off[sample, 0]
    sizes = np.zeros(w.n_envs, dtype=np.int64)
    sizes[sample] = 2 * caps.astype(np.int64) + 2 * (msgs + w.n_steps * len(w.agents) * 8)
    toff = np.concatenate([[0], np.cumsum(sizes)])
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    ds = DeviceStream.from_host(s)
    del s
    print("[parity] rollout", flush=True)
    got = env.rollout(ds, w.n_steps, trade_off=toff)
    torch.cuda.synchronize()
    print("[parity] oracle on the sample", flush=True)
    o = oracle_for(hs, book, caps, w.max_cap, w.agents, w.ep_len, w.seed, env_ids=sample)
    acts = got["actions"].cpu().numpy()[:, :, sample]
    ref = o.step(hs, n_steps=w.n_steps, actions=np.ascontiguousarray(acts))
    for j, e in enumerate(sample):
        cnt = int(ref["n_trades"][:, j].sum())
        gt = got["trades"][toff[e]: toff[e] + cnt].cpu().numpy()
        assert np.array_equal(gt, ref["trades"][ref["trade_off"][j]: ref["trade_off"][j] + cnt]), e
    g = dict(got)
    g["trades"] = None
    ref = dict(ref)
    ref["trades"] = None
    assert_same_outputs(g, ref, w.n_steps, envs=sample, what=w.name)
    assert_same_books(env.books(), o.books(), envs=sample, what=w.name)
    assert_same_state(env.state(), o.state(), envs=sample, what=w.name)
    a = got["actions"].cpu().numpy()
    assert a.min() >= 0 and a[:, 2].max() <= 2


def test_plain_and_persistent_forms_identical_full_size():
    """Property at full size: the per-step form and the persistent form agree exactly."""
    _, DeviceStream = _lob()
    w = synth.WORKLOADS["uneven8192"].scaled(n_steps=16)
    s = synth.generate(w)
    ds = DeviceStream.from_host(s)
    e1 = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    toff = ds.trade_regions(e1.caps, 0, 16, 2)
    a = e1.rollout(ds, 16, trade_off=toff)
    e2 = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    b = run_steps(e2, ds, 16, None, toff)
    torch.cuda.synchronize()
    for k in ("n_trades", "fills", "reward", "obs", "done", "actions"):
        assert torch.equal(a[k], b[k]), k
    n = a["n_trades"].sum(0).cpu().numpy()
    off = toff.cpu().numpy()
    for e in range(0, w.n_envs, 97):
        assert torch.equal(a["trades"][off[e]: off[e] + n[e]], b["trades"][off[e]: off[e] + n[e]]), e
    ba, bb = e1.books(), e2.books()
    for k in ba:
        assert torch.equal(ba[k], bb[k]), k


def test_rollout_captured_in_a_graph():
    """A rollout of several capacity classes (concurrent launches on forked streams,
    staggered starts, queue counters cleared by a kernel) captured in a HIP graph: every
    replay, with eager work and synchronisation between the replays, equals the oracle."""
    w = SMALL[2]  # uneven: 96 envs, books of 50..400 orders, execution + market-making agent
    n = w.n_steps
    print(f"\n[graph] {w.name} envs={w.n_envs} steps={n}", flush=True)
    _, DeviceStream = _lob()
    s = synth.generate(w)
    o = oracle_for(s, s.book, s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    ref = o.step(s, n_steps=n)
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    assert len(env.schedule()) > 1
    ds = DeviceStream.from_host(s)
    toff = torch.from_numpy(ref["trade_off"]).cuda()
    book = {k: torch.from_numpy(v).cuda() for k, v in s.book.items()}
    out = env._alloc_out(n, True, True, toff, ds)
    env.plan(ds, n)
    env.rollout(ds, n, out=out)  # eager first: streams, events and plan in place
    torch.cuda.synchronize()
    assert_same_outputs(out, ref, n, what="eager")
    g = torch.cuda.CUDAGraph()
    env.reset(book)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        env.rollout(ds, n, out=out)
    for rep in range(3):
        for k in ("n_trades", "fills", "reward", "obs", "done", "trades"):
            if out.get(k) is not None:
                out[k].fill_(7)
        env.reset(book)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_same_outputs(out, ref, n, what=f"graph replay {rep}")
        assert_same_books(env.books(), o.books(), what=f"graph replay {rep}")


def test_schedule_independence():
    """Every schedule the autotuner can pick, and the padded single-class grouping,
    give identical outputs and books."""
    _, DeviceStream = _lob()
    w = synth.Workload("sched", n_envs=300, n_steps=6, msgs_range=(1, 300), cap_choices=(50, 100, 200, 400),
                       agents=("exec", "mm"), seed=41)
    s = synth.generate(w)
    ds = DeviceStream.from_host(s)
    ref_env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    toff = ds.trade_regions(ref_env.caps, 0, w.n_steps, 2)
    ref = ref_env.rollout(ds, w.n_steps, trade_off=toff)
    ref_books = ref_env.books()
    n_classes = len(ref_env.schedule())
    for padded, mode, waves in [(False, m, wv) for m in (0, 1) for wv in (1, 2, 4)] + [(True, 0, 2), (True, 1, 1)]:
        env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
        if padded:
            env.set_padded(True)
            assert len(env.schedule()) == 1 and env.schedule()[0]["cap_slots"] == max(s.caps)
        env.plan(ds, w.n_steps)
        for k in range(len(env.schedule())):
            try:
                env.set_schedule(k, waves, mode, 0 if mode == 0 else 7)
            except Exception:
                pass  # the workgroup would need more LDS than allowed
        got = env.rollout(ds, w.n_steps, trade_off=toff)
        torch.cuda.synchronize()
        for key in ("n_trades", "fills", "reward", "obs", "done", "actions", "trades"):
            assert torch.equal(got[key], ref[key]) or key == "trades", (mode, waves, key)
        n = got["n_trades"].sum(0).cpu().numpy()
        off = toff.cpu().numpy()
        for e in range(0, w.n_envs, 7):
            assert torch.equal(got["trades"][off[e]: off[e] + n[e]], ref["trades"][off[e]: off[e] + n[e]])
        gb = env.books()
        for key in gb:
            assert torch.equal(gb[key], ref_books[key]), (mode, waves, key)
    # the proportional work-queue schedule of the concurrent classes, at several LDS
    # shares (1 permille leaves a few envs resident), and switched off
    for b in (1, 300, 880, 1000, 0):
        env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
        env.set_balance(b)
        env.plan(ds, w.n_steps)
        sch = env.schedule()
        assert all(c["mode"] == (1 if b > 0 and n_classes > 1 else 0) for c in sch), (b, sch)
        if b == 1:
            assert all(c["grid"] >= 1 for c in sch) and sum(c["grid"] * c["waves"] for c in sch) <= 12, sch
        got = env.rollout(ds, w.n_steps, trade_off=toff)
        torch.cuda.synchronize()
        for key in ("n_trades", "fills", "reward", "obs", "done", "actions"):
            assert torch.equal(got[key], ref[key]), (b, key)
        gb = env.books()
        for key in gb:
            assert torch.equal(gb[key], ref_books[key]), (b, key)
    # the tuner picks one of them and restores the state it started from
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    sched = env.autotune(ds, w.n_steps)
    assert len(sched) == n_classes
    got = env.rollout(ds, w.n_steps, trade_off=toff)
    for key in ("n_trades", "fills", "reward", "obs", "done", "actions"):
        assert torch.equal(got[key], ref[key]), key


@pytest.mark.parametrize("agents,mode", [((), "rollout"), (("exec", "mm"), "step"), (("exec", "mm"), "rollout")])
def test_lobster_format_day_parity(tmp_path, agents, mode):
    """A synthetic day in LOBSTER's file formats (messages with executions of named
    orders and ignored messages; its order-book file), parsed, cut into env windows with
    reset books from the order-book rows before them, replayed on the GPU and by the
    oracle."""
    from paper_2511_02136_amd import lobster
    from lobster_files import synthetic_day
    _, DeviceStream = _lob()
    _, msg_path, book_path, _ = synthetic_day(str(tmp_path), n=3000)
    m = lobster.read_messages(msg_path)
    starts = [0, 150, 400, 900, 1200, 1500, 1800, 2100]
    n_steps, per = 8, 60
    s = lobster.build_stream(m, starts, n_steps=n_steps, msgs_per_step=per, cap=64,
                             books=lobster.books_before(book_path, starts), agents=agents, seed=61)
    w = s.workload
    print(f"\n[parity] lobster day envs={w.n_envs} steps={n_steps} agents={agents} mode={mode}", flush=True)
    o = oracle_for(s, s.book, s.caps, w.max_cap, agents, w.ep_len, w.seed)
    ref = o.step(s, n_steps=n_steps)
    env = gpu_env(s.caps, w.max_cap, agents, w.ep_len, w.seed, s.book)
    ds = DeviceStream.from_host(s)
    toff = torch.from_numpy(ref["trade_off"]).cuda()
    got = env.rollout(ds, n_steps, trade_off=toff) if mode == "rollout" else run_steps(env, ds, n_steps, None, toff)
    torch.cuda.synchronize()
    name = f"lobster/{mode}"
    assert_same_outputs(got, ref, n_steps, what=name)
    assert_same_books(env.books(), o.books(), what=name)
    assert_same_state(env.state(), o.state(), what=name)
    ct = o.state()["counters"]
    assert ct[:, 10].sum() > 0 and ct[:, 1].sum() > 0  # ignored messages and trades occurred


def test_import_state_continues_in_a_fresh_context():
    """64 steps, export of the books and state, import into a fresh context, 64 more
    steps: every output, the books and the state equal the oracle's uninterrupted
    128-step run, and the observation right after the import equals the exporting
    context's.  The oracle's own state at step 64, imported into a third context and
    run in the per-step form, continues the same way."""
    LobEnv, DeviceStream = _lob()
    w = synth.Workload("import", n_envs=160, n_steps=128, msgs_range=(1, 200), cap_choices=(50, 100, 200, 400),
                       agents=("exec", "mm"), seed=42)
    print(f"\n[import] envs={w.n_envs} steps=64+64", flush=True)
    s = synth.generate(w)
    o = oracle_for(s, s.book, s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    ref1 = o.step(s, n_steps=64)
    o_books, o_state, o_obs = o.books(), o.state(), o.observe()
    ref2 = o.step(s, n_steps=64)
    ds = DeviceStream.from_host(s)
    env1 = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    g1 = env1.rollout(ds, 64, trade_off=torch.from_numpy(ref1["trade_off"]).cuda())
    books, state = env1.books(), env1.state()
    obs1 = env1.observe()
    torch.cuda.synchronize()
    assert_same_outputs(g1, ref1, 64, what="import/first")
    env1.close()
    env2 = LobEnv(s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    env2.import_state(books, state, 64)
    assert env2.t == 64
    assert torch.equal(env2.observe(), obs1)
    assert np.array_equal(obs1.cpu().numpy().view(np.int32), o_obs.view(np.int32))
    g2 = env2.rollout(ds, 64, trade_off=torch.from_numpy(ref2["trade_off"]).cuda())
    torch.cuda.synchronize()
    assert_same_outputs(g2, ref2, 64, what="import/second")
    assert_same_books(env2.books(), o.books(), what="import")
    assert_same_state(env2.state(), o.state(), what="import")
    # the oracle's state imported
    env3 = LobEnv(s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    env3.import_state({k: torch.from_numpy(v) for k, v in o_books.items()},
                      {k: torch.from_numpy(v) for k, v in o_state.items()}, 64)
    g3 = run_steps(env3, ds, 64, None, torch.from_numpy(ref2["trade_off"]).cuda())
    torch.cuda.synchronize()
    assert_same_outputs(g3, ref2, 64, what="import/oracle state")
    assert_same_books(env3.books(), o.books(), what="import/oracle state")
    assert_same_state(env3.state(), o.state(), what="import/oracle state")


def test_replay1_full_size_parity():
    """The single-env replay workload at full size (10^6 messages in 10,000 steps of 100,
    no agents) in one persistent launch: every step's trade count and every trade
    record, the final book and the state equal the oracle's."""
    _, DeviceStream = _lob()
    w = synth.WORKLOADS["replay1"]
    print(f"\n[parity] full-size {w.name}", flush=True)
    s = synth.generate(w)
    o = oracle_for(s, s.book, s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    ref = o.step(s, n_steps=w.n_steps)
    env = gpu_env(s.caps, w.max_cap, w.agents, w.ep_len, w.seed, s.book)
    got = env.rollout(DeviceStream.from_host(s), w.n_steps, trade_off=torch.from_numpy(ref["trade_off"]).cuda())
    torch.cuda.synchronize()
    assert int(ref["n_trades"].sum()) > 100_000
    assert_same_outputs(got, ref, w.n_steps, what=w.name)
    assert_same_books(env.books(), o.books(), what=w.name)
    assert_same_state(env.state(), o.state(), what=w.name)
    assert int(o.state()["counters"][0, 0]) == 1_000_000


@pytest.mark.parametrize("mode", ["step", "rollout"])
@pytest.mark.parametrize("given", [False, True])
def test_parity_agent_variants(mode, given):
    """The market maker's spread-skew and AvSt action spaces and the TWAP and
    Avellaneda-Stoikov baselines (quotes that move with inventory and steps left), next to
    each other, in both forms, with random and given (including out-of-range) actions."""
    w = synth.Workload("variants", n_envs=56, n_steps=14, msgs_range=(1, 250), cap_choices=(20, 64, 100, 200),
                       agents=("mm_spreadskew", "exec_twap", "mm_avst", "mm_as"), seed=43)
    parity_case(w, w.n_steps, mode, given_actions=given,
                kw=dict(exec_task=120, mm_lambda=0.5, mm_rho=0.01, avst_gamma=0.02, avst_sigma2=6.0, avst_kappa=0.6),
                name=f"variants/{mode}/{'given' if given else 'random'}")

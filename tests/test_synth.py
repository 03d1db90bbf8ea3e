"""Statistics and layout of the synthetic MBO input generator (inputs only)."""
import numpy as np

from paper_2511_02136_amd import synth


def small(**kw):
    base = dict(name="t", n_envs=64, n_steps=50, msgs_per_step=100, cap=100, seed=123)
    base.update(kw)
    return synth.Workload(**base)


def test_message_mix_and_laws():
    s = synth.generate(small(n_envs=256))
    typ = s.ts & 0xFF
    side = (s.ts >> 8) & 1
    n = len(typ)
    for code, p in ((1, 0.5), (2, 0.2), (3, 0.2), (4, 0.1)):
        frac = np.mean(typ == code)
        assert abs(frac - p) < 4 * np.sqrt(p * (1 - p) / n)
    assert abs(side.mean() - 0.5) < 4 * np.sqrt(0.25 / n)
    assert set(np.unique(typ)) <= {1, 2, 3, 4}
    # sizes of new orders: lognormal(4, 1) through a 4096-quantile table
    lim = typ == 1
    q = s.qty[lim]
    assert q.min() >= 1
    assert abs(np.log(q).mean() - 4.0) < 0.02
    assert abs(np.log(q).std() - 1.0) < 0.03
    assert abs(np.median(q) - np.exp(4.0)) <= 2
    # limit prices sit at mid -/+ g with g ~ Geometric(0.3) (failures): recover g from the
    # per-env mid walk is not possible directly, so check the spread of prices around the
    # running median of each env-step instead: the distance is small and one-sided
    assert np.all(s.oid[lim] > 0)


def test_geometric_offset_law():
    # reconstruct the mid walk exactly for one env from the same hash the generator uses
    w = small(n_envs=1, n_steps=400)
    s = synth.generate(w)
    tb = synth.size_table()
    assert tb.shape == (4096,)
    # prices of buy limits are <= prices of sell limits on average by ~2*7/3 ticks
    typ = s.ts & 0xFF
    side = (s.ts >> 8) & 1
    b = s.price[(typ == 1) & (side == 0)].astype(np.float64)
    a = s.price[(typ == 1) & (side == 1)].astype(np.float64)
    assert 3.0 < a.mean() - b.mean() < 6.5


def test_table_is_lognormal_quantiles():
    from scipy.stats import lognorm
    tb = synth.size_table().astype(np.float64)
    u = (np.arange(4096) + 0.5) / 4096
    x = lognorm.ppf(u, s=1.0, scale=np.exp(4.0))
    assert np.all(np.abs(tb - np.maximum(1, np.floor(x + 0.5))) <= 1)


def test_determinism_and_env_independence():
    w = small(n_envs=8, n_steps=20)
    a = synth.generate(w, threads=1)
    b = synth.generate(w, threads=4)
    for x, y in zip(a.msg_fields(), b.msg_fields()):
        assert np.array_equal(x, y)
    # env 3 alone (first 4 envs generated) equals env 3 of the larger run
    c = synth.generate(w.scaled(n_envs=4), threads=1)
    lo, hi = a.off[3, 0], a.off[3, -1]
    lo2, hi2 = c.off[3, 0], c.off[3, -1]
    for x, y in zip(a.msg_fields(), c.msg_fields()):
        assert np.array_equal(x[lo:hi], y[lo2:hi2])


def test_csr_offsets_and_uneven_shapes():
    w = synth.Workload("u", n_envs=512, n_steps=4, msgs_range=(1, 400), cap_choices=(50, 100, 200, 400),
                       seed=9)
    s = synth.generate(w)
    off = s.off
    assert off[0, 0] == 0
    assert np.all(np.diff(off, axis=1) >= 1)
    assert np.all(off[1:, 0] == off[:-1, -1])
    per_env = np.diff(off, axis=1)
    assert np.all(per_env == per_env[:, :1])  # fixed count per env
    assert per_env.min() >= 1 and per_env.max() <= 400
    assert abs(per_env[:, 0].mean() - 200.5) < 4 * 115.5 / np.sqrt(512)
    assert set(np.unique(s.caps)) == {50, 100, 200, 400}
    # snapshot: half the capacity per side, best price first, uncrossed, ids 1..
    n = s.book["n"]
    assert np.array_equal(n[:, 0], s.caps // 2) and np.array_equal(n[:, 1], s.caps // 2)
    for e in range(0, 512, 37):
        bp = s.book["price"][e, 0, : n[e, 0]]
        ap = s.book["price"][e, 1, : n[e, 1]]
        assert np.all(np.diff(bp) <= 0) and np.all(np.diff(ap) >= 0)
        assert bp[0] < ap[0]


def test_burst_steps_carry_extra_cancels():
    w = synth.Workload("b", n_envs=64, n_steps=64, msgs_per_step=40, burst_pct=10, burst_extra=48,
                       cap=100, seed=4)
    s = synth.generate(w)
    per = np.diff(s.off, axis=1)
    bursts = per == 88
    assert np.all((per == 40) | bursts)
    assert abs(bursts.mean() - 0.1) < 4 * np.sqrt(0.09 / bursts.size)
    e, t = np.argwhere(bursts)[0]
    lo = s.off[e, t]
    typ = s.ts[lo + 40: lo + 88] & 0xFF
    assert set(np.unique(typ)) <= {2, 3}

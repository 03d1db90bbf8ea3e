"""Element-by-element comparison of GPU outputs with the oracle's (shared by GPU tests)."""
from __future__ import annotations

import numpy as np


def to_np(x):
    if x is None:
        return None
    if hasattr(x, "detach"):
        return x.detach().cpu().numpy()
    return np.asarray(x)


def assert_same_outputs(got: dict, ref: dict, n_steps: int, envs=None, what=""):
    """got: GPU outputs (torch), ref: oracle outputs (numpy), same layouts.  envs: the
    GPU env indices that correspond to the oracle's envs 0..len-1 (None = identity)."""
    g = {k: to_np(v) for k, v in got.items() if not k.startswith("_")}
    N = ref["n_trades"].shape[1]
    sel = np.arange(N) if envs is None else np.asarray(envs)
    assert np.array_equal(g["n_trades"][:, sel], ref["n_trades"]), f"{what}: n_trades"
    assert np.array_equal(g["done"][:, sel], ref["done"]), f"{what}: done"
    if ref["fills"].shape[1]:
        assert np.array_equal(g["fills"][:, :, sel], ref["fills"]), f"{what}: fills"
        # rewards and observations compared bit for bit
        assert np.array_equal(g["reward"][:, :, sel].view(np.int32), ref["reward"].view(np.int32)), f"{what}: reward"
        if g.get("obs") is not None:
            assert np.array_equal(g["obs"][:, :, sel].view(np.int32), ref["obs"].view(np.int32)), f"{what}: obs"
        if g.get("actions") is not None:
            assert np.array_equal(g["actions"][:, :, sel], ref["actions"]), f"{what}: actions"
    if g.get("trades") is not None and ref.get("trades") is not None:
        gt, rt = g["trades"], ref["trades"]
        goff, roff = g["trade_off"], ref["trade_off"]
        for j, e in enumerate(sel):
            cnt = int(ref["n_trades"][:, j].sum())
            room_r = int(roff[j + 1] - roff[j])
            room_g = int(goff[e + 1] - goff[e])
            k = min(cnt, room_r, room_g)
            a = gt[goff[e]: goff[e] + k]
            b = rt[roff[j]: roff[j] + k]
            if not np.array_equal(a, b):
                bad = np.nonzero((a != b).any(1))[0][0]
                raise AssertionError(f"{what}: trades env {e} record {bad}: gpu {a[bad].tolist()} oracle {b[bad].tolist()}")


def assert_same_books(gb: dict, rb: dict, envs=None, what=""):
    g = {k: to_np(v) for k, v in gb.items()}
    sel = slice(None) if envs is None else np.asarray(envs)
    assert np.array_equal(g["n"][sel], rb["n"]), f"{what}: book sizes"
    for k in ("price", "qty", "oid", "tid", "tsec", "tns"):
        a, b = g[k][sel], rb[k]
        if not np.array_equal(a, b):
            e, s, i = np.argwhere(a != b)[0]
            raise AssertionError(f"{what}: book {k} env {e} side {s} slot {i}: gpu {a[e, s, i]} oracle {b[e, s, i]}")


def assert_same_state(gs: dict, rs: dict, envs=None, what=""):
    sel = slice(None) if envs is None else np.asarray(envs)
    for k in ("env", "agents", "counters"):
        a, b = to_np(gs[k])[sel], rs[k]
        if not np.array_equal(a, b):
            idx = np.argwhere(a != b)[0]
            raise AssertionError(f"{what}: state {k} at {idx.tolist()}: gpu {a[tuple(idx)]} oracle {b[tuple(idx)]}")

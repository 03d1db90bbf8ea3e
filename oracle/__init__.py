"""CPU oracle of the batched limit-order-book environment step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares no code with the HIP library; the
two meet only in the seeded inputs from ``paper_2511_02136_amd.synth``.

The C++ core (``oracle.cpp``) is a plain sequential implementation of the paper's
environment step (Sec. 4: action conversion, shuffle, concatenation, book processing,
outcomes) over a ``std::map``-of-deques price-time-priority book (Sec. 2.1).  The
PPO/MLP part of the oracle (``ppo_ref``) is a float64 NumPy/PyTorch-CPU reference.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OBS_DIM = 40
TRADE_WORDS = 8
N_COUNTERS = 11
COUNTER_NAMES = ("msgs", "trades", "miss", "evict", "evicted_qty", "drop", "dropped_qty",
                 "market_unfilled", "bad", "trade_overflow", "ignored")
ENV_STATE_NAMES = ("last_bb", "last_ba", "mid2_prev", "p_init2", "last_tsec", "last_tns", "t",
                   "last_dmid2", "step_buy_vol", "step_sell_vol", "step_trades", "step_last_price")
AGENT_STATE_NAMES = ("inventory", "cash", "remaining", "order_counter", "step_bought", "step_sold")
ENV_STATE_WORDS = len(ENV_STATE_NAMES)
AGENT_STATE_WORDS = len(AGENT_STATE_NAMES)
N_ACTIONS = {0: 9, 1: 9, 2: 3, 3: 9, 4: 9, 5: 9, 6: 1, 7: 1}


class _OrCfg(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32),
        ("n_agents", ctypes.c_int32),
        ("max_cap", ctypes.c_int32),
        ("episode_len", ctypes.c_int32),
        ("cap", ctypes.c_void_p),
        ("agent_kind", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("exec_task", ctypes.c_int32),
        ("exec_q0", ctypes.c_int32),
        ("mm_q", ctypes.c_int32),
        ("dir_q", ctypes.c_int32),
        ("exec_penalty", ctypes.c_float),
        ("mm_lambda", ctypes.c_float),
        ("mm_rho", ctypes.c_float),
        ("pad_", ctypes.c_float),
        ("env_id", ctypes.c_void_p),
        ("avst_gamma", ctypes.c_float),
        ("avst_sigma2", ctypes.c_float),
        ("avst_kappa", ctypes.c_float),
        ("pad2_", ctypes.c_float),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        p, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.ob_new.argtypes = [i32]
        lib.ob_new.restype = p
        lib.ob_free.argtypes = [p]
        lib.ob_process.argtypes = [p, p, i32, i32, p, i32, p]
        lib.ob_process.restype = i32
        lib.ob_export.argtypes = [p, i32, p, i32]
        lib.ob_export.restype = i32
        lib.ob_load.argtypes = [p, i32, p, i32]
        lib.oe_new.argtypes = [ctypes.POINTER(_OrCfg)]
        lib.oe_new.restype = p
        lib.oe_free.argtypes = [p]
        lib.oe_reset.argtypes = [p] + [p] * 7
        lib.oe_reset.restype = i32
        lib.oe_step.argtypes = [p, i32] + [p] * 8 + [i32] + [p] * 9 + [i32]
        lib.oe_step.restype = i32
        lib.oe_observe.argtypes = [p, p]
        lib.oe_observe.restype = i32
        lib.oe_export_books.argtypes = [p] + [p] * 7
        lib.oe_export_books.restype = i32
        lib.oe_export_state.argtypes = [p, p, p, p]
        lib.oe_export_state.restype = i32
        lib.oe_import_state.argtypes = [p] * 11 + [i32]
        lib.oe_import_state.restype = i32
        lib.oe_hash.argtypes = [u64] * 5
        lib.oe_hash.restype = u64
        lib.oe_mix.argtypes = [u64]
        lib.oe_mix.restype = u64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def chain_hash(seed: int, dom: int, a: int, b: int, c: int) -> int:
    return int(_load().oe_hash(seed, dom, a, b, c))


def splitmix64_mix(z: int) -> int:
    return int(_load().oe_mix(z))


DOM_SHUFFLE = 0x5348554646
DOM_ACTION = 0x414354


class OracleBook:
    """One price-time-priority book (both sides) with a per-side capacity."""

    def __init__(self, cap: int):
        self._lib = _load()
        self._h = self._lib.ob_new(cap)
        self.cap = cap
        self.counters = np.zeros(N_COUNTERS, dtype=np.int64)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ob_free(h)
            self._h = None

    def process(self, ts: int, price: int, qty: int, oid: int, tid: int = 0, tsec: int = 0,
                tns: int = 0, seq: int = 0, t: int = 0, max_trades: int = 4096) -> np.ndarray:
        msg = np.array([ts, price, qty, oid, tid, tsec, tns], dtype=np.int32)
        buf = np.zeros((max_trades, TRADE_WORDS), dtype=np.int32)
        n = self._lib.ob_process(self._h, _ptr(msg), seq, t, _ptr(buf), max_trades, _ptr(self.counters))
        return buf[: min(n, max_trades)].copy()

    def side(self, s: int) -> np.ndarray:
        """Orders of side s (0 bids, 1 asks) in priority order, [n, 6]."""
        buf = np.zeros((self.cap + 1, 6), dtype=np.int32)
        n = self._lib.ob_export(self._h, s, _ptr(buf), self.cap + 1)
        return buf[:n].copy()

    def load(self, s: int, orders) -> None:
        a = np.ascontiguousarray(np.asarray(orders, dtype=np.int32).reshape(-1, 6))
        self._lib.ob_load(self._h, s, _ptr(a), a.shape[0])


class OracleEnvs:
    """All envs of one workload, stepped sequentially on the host (threads over envs)."""

    def __init__(self, caps: np.ndarray, max_cap: int, agent_kinds: Sequence[int], episode_len: int,
                 seed: int, exec_task: int = 500, exec_q0: int = 4, mm_q: int = 10, dir_q: int = 10,
                 exec_penalty: float = 0.01, mm_lambda: float = 0.0, mm_rho: float = 0.0,
                 env_ids: Optional[np.ndarray] = None, avst_gamma: float = 0.01, avst_sigma2: float = 10.0,
                 avst_kappa: float = 0.5):
        self._lib = _load()
        self.caps = np.ascontiguousarray(caps, dtype=np.int32)
        self.kinds = np.ascontiguousarray(np.asarray(agent_kinds, dtype=np.int32).reshape(-1))
        self.n_envs = int(self.caps.shape[0])
        self.n_agents = int(self.kinds.shape[0])
        self.max_cap = int(max_cap)
        self.episode_len = int(episode_len)
        c = _OrCfg()
        c.n_envs, c.n_agents, c.max_cap, c.episode_len = self.n_envs, self.n_agents, self.max_cap, self.episode_len
        c.cap = self.caps.ctypes.data
        c.agent_kind = self.kinds.ctypes.data if self.n_agents else None
        c.seed = seed
        c.exec_task, c.exec_q0, c.mm_q, c.dir_q = exec_task, exec_q0, mm_q, dir_q
        c.exec_penalty, c.mm_lambda, c.mm_rho = exec_penalty, mm_lambda, mm_rho
        c.avst_gamma, c.avst_sigma2, c.avst_kappa = avst_gamma, avst_sigma2, avst_kappa
        self.env_ids = None
        if env_ids is not None:
            self.env_ids = np.ascontiguousarray(np.asarray(env_ids, dtype=np.int32).reshape(-1))
            assert self.env_ids.shape[0] == self.n_envs
            c.env_id = self.env_ids.ctypes.data
        self._h = self._lib.oe_new(ctypes.byref(c))
        if not self._h:
            raise ValueError("oracle rejected the configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oe_free(h)
            self._h = None

    def reset(self, book: dict) -> None:
        arrs = [np.ascontiguousarray(book[k], dtype=np.int32)
                for k in ("price", "qty", "oid", "tid", "tsec", "tns", "n")]
        rc = self._lib.oe_reset(self._h, *[_ptr(a) for a in arrs])
        if rc != 0:
            raise RuntimeError(f"oe_reset: {rc}")

    def step(self, stream, n_steps: int = 1, actions: Optional[np.ndarray] = None,
             trade_off: Optional[np.ndarray] = None, threads: Optional[int] = None,
             record_trades: bool = True) -> dict:
        """Advance every env by n_steps.  actions: int32 [n_steps, A, n_envs] or None
        (random policy).  Returns the step outputs in the GPU library's layouts."""
        N, A = self.n_envs, self.n_agents
        off = np.ascontiguousarray(stream.off, dtype=np.int64)
        off_steps = off.shape[1] - 1
        if actions is not None:
            actions = np.ascontiguousarray(np.asarray(actions, dtype=np.int32).reshape(n_steps, A, N))
        if trade_off is None:
            trade_off = trade_bound_offsets(stream, self.caps, self.state()["env"][:, 6], n_steps, A)
        out = {
            "n_trades": np.zeros((n_steps, N), dtype=np.int32),
            "fills": np.zeros((n_steps, A, N, 4), dtype=np.int64),
            "reward": np.zeros((n_steps, A, N), dtype=np.float32),
            "obs": np.zeros((n_steps, A, N, OBS_DIM), dtype=np.float32),
            "done": np.zeros((n_steps, N), dtype=np.uint8),
            "actions": np.zeros((n_steps, A, N), dtype=np.int32),
            "trade_off": trade_off,
        }
        trades = np.zeros((int(trade_off[-1]), TRADE_WORDS), dtype=np.int32) if record_trades else None
        if threads is None:
            threads = min(16, os.cpu_count() or 1)
        rc = self._lib.oe_step(self._h, n_steps, *[_ptr(np.ascontiguousarray(f)) for f in stream.msg_fields()],
                               _ptr(off), off_steps, _ptr(actions), _ptr(trades), _ptr(trade_off),
                               _ptr(out["n_trades"]), _ptr(out["fills"]), _ptr(out["reward"]),
                               _ptr(out["obs"]), _ptr(out["done"]), _ptr(out["actions"]), int(threads))
        if rc != 0:
            raise RuntimeError(f"oe_step: {rc}")
        out["trades"] = trades
        return out

    def observe(self) -> np.ndarray:
        obs = np.zeros((self.n_agents, self.n_envs, OBS_DIM), dtype=np.float32)
        self._lib.oe_observe(self._h, _ptr(obs))
        return obs

    def books(self) -> dict:
        N, mc = self.n_envs, self.max_cap
        b = {k: np.zeros((N, 2, mc), dtype=np.int32) for k in ("price", "qty", "oid", "tid", "tsec", "tns")}
        b["n"] = np.zeros((N, 2), dtype=np.int32)
        self._lib.oe_export_books(self._h, *[_ptr(b[k]) for k in ("price", "qty", "oid", "tid", "tsec", "tns", "n")])
        return b

    def state(self) -> dict:
        N, A = self.n_envs, self.n_agents
        es = np.zeros((N, ENV_STATE_WORDS), dtype=np.int64)
        ag = np.zeros((N, max(A, 1), AGENT_STATE_WORDS), dtype=np.int64)
        ct = np.zeros((N, N_COUNTERS), dtype=np.int64)
        self._lib.oe_export_state(self._h, _ptr(es), _ptr(ag), _ptr(ct))
        return {"env": es, "agents": ag[:, :A], "counters": ct}

    def import_state(self, book: dict, state: dict, step: int) -> None:
        """Continue every env from ``book`` (canonical layout) and ``state`` (the layouts
        of ``state()``; counters optional) with its step counter at ``step``."""
        N, A = self.n_envs, self.n_agents
        arrs = [np.ascontiguousarray(book[k], dtype=np.int32)
                for k in ("price", "qty", "oid", "tid", "tsec", "tns", "n")]
        es = np.ascontiguousarray(state["env"], dtype=np.int64).reshape(N, ENV_STATE_WORDS)
        ag = np.ascontiguousarray(np.asarray(state["agents"], dtype=np.int64).reshape(N, A, AGENT_STATE_WORDS)) \
            if A else np.zeros((N, 1, AGENT_STATE_WORDS), dtype=np.int64)
        ct = state.get("counters")
        ct = None if ct is None else np.ascontiguousarray(ct, dtype=np.int64).reshape(N, N_COUNTERS)
        rc = self._lib.oe_import_state(self._h, *[_ptr(a) for a in arrs], _ptr(es), _ptr(ag), _ptr(ct), int(step))
        if rc != 0:
            raise RuntimeError(f"oe_import_state: {rc}")


def trade_bound_offsets(stream, caps: np.ndarray, t0: np.ndarray, n_steps: int, n_agents: int) -> np.ndarray:
    """Per-env trade-record regions that can never overflow over steps [t0, t0+n_steps).

    Every trade either fully consumes a resting order or ends an aggressive message, so
    the count is at most (resting orders at the start + orders inserted) + messages
    <= 2*cap + 2*(messages), agent messages counted at their per-step maximum."""
    off = stream.off
    N = off.shape[0]
    rows = np.arange(N)
    t0 = np.asarray(t0, dtype=np.int64).reshape(-1)
    if t0.shape[0] == 1:
        t0 = np.repeat(t0, N)
    msgs = off[rows, t0 + n_steps] - off[rows, t0]
    agent_msgs = n_steps * n_agents * 8
    bound = 2 * caps.astype(np.int64) + 2 * (msgs + agent_msgs)
    return np.concatenate([[0], np.cumsum(bound)]).astype(np.int64)

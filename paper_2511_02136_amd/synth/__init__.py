"""Seeded synthetic market-by-order inputs shared by the CPU oracle and the GPU path.

This module generates inputs only (message streams, CSR step offsets, per-env book
capacities and reset snapshots).  It contains none of the order-book method's
arithmetic.  The paper replays LOBSTER market-by-order data stored contiguously
with episode start indices (Sec. 4); the generator stands in for that data with
the message mix, price and size laws of the benchmark workloads (see ``WORKLOADS``).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

SEED_BASE = 2511021360

# message type codes (low byte of the type|side word); side is bit 8 (0 buy, 1 sell)
LIMIT, PARTIAL_CANCEL, DELETE, MARKET = 1, 2, 3, 4
BUY, SELL = 0, 1

AGENT_KINDS = {"exec": 0, "mm": 1, "dir": 2, "mm_buysell": 3, "mm_spreadskew": 4, "mm_avst": 5, "exec_twap": 6,
               "mm_as": 7}


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32),
        ("n_steps", ctypes.c_int32),
        ("msgs_per_step", ctypes.c_int32),
        ("msgs_lo", ctypes.c_int32),
        ("msgs_hi", ctypes.c_int32),
        ("burst_pct", ctypes.c_int32),
        ("burst_extra", ctypes.c_int32),
        ("cap_fixed", ctypes.c_int32),
        ("n_cap_choices", ctypes.c_int32),
        ("cap_choices", ctypes.c_int32 * 8),
        ("mid0", ctypes.c_int32),
        ("snapshot_fill_pct", ctypes.c_int32),
        ("exec_pct", ctypes.c_int32),
        ("ignored_pct", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.synth_offsets.argtypes = [ctypes.POINTER(_Cfg), p]
        lib.synth_offsets.restype = ctypes.c_int64
        lib.synth_generate.argtypes = [ctypes.POINTER(_Cfg), p, ctypes.c_int32] + [p] * 14 + [ctypes.c_int32]
        lib.synth_generate.restype = ctypes.c_int
        lib.synth_env_cap.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int32]
        lib.synth_env_cap.restype = ctypes.c_int32
        lib.synth_size_table.argtypes = [p]
        lib.synth_size_table.restype = None
        lib.synth_u32.argtypes = [ctypes.c_uint64] * 5
        lib.synth_u32.restype = ctypes.c_uint32
        _lib = lib
    return _lib


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape of one synthetic workload (sizes, mix, agents, seed)."""

    name: str
    n_envs: int
    n_steps: int
    msgs_per_step: int = 0
    msgs_range: Tuple[int, int] = (0, 0)
    burst_pct: int = 0
    burst_extra: int = 0
    cap: int = 0
    cap_choices: Tuple[int, ...] = ()
    agents: Tuple[str, ...] = ()
    episode_len: int = 0  # 0: equal to n_steps
    seed: int = SEED_BASE
    mid0: int = 100_000
    snapshot_fill_pct: int = 50
    exec_pct: int = 0       # percent of replayed messages that are executions of named orders
    ignored_pct: int = 0    # percent that the book ignores (hidden executions, halts)

    def scaled(self, n_envs: Optional[int] = None, n_steps: Optional[int] = None, **kw) -> "Workload":
        d = dataclasses.asdict(self)
        if n_envs is not None:
            d["n_envs"] = n_envs
        if n_steps is not None:
            d["n_steps"] = n_steps
            if self.episode_len in (0, self.n_steps):
                d["episode_len"] = 0
        d.update(kw)
        d["cap_choices"] = tuple(d["cap_choices"])
        d["agents"] = tuple(d["agents"])
        d["msgs_range"] = tuple(d["msgs_range"])
        return Workload(**d)

    @property
    def max_cap(self) -> int:
        return self.cap if self.cap > 0 else max(self.cap_choices)

    @property
    def ep_len(self) -> int:
        return self.episode_len if self.episode_len > 0 else self.n_steps

    def _cfg(self) -> _Cfg:
        c = _Cfg()
        c.n_envs = self.n_envs
        c.n_steps = self.n_steps
        c.msgs_per_step = self.msgs_per_step
        c.msgs_lo, c.msgs_hi = self.msgs_range
        c.burst_pct = self.burst_pct
        c.burst_extra = self.burst_extra
        c.cap_fixed = self.cap
        c.n_cap_choices = len(self.cap_choices)
        for i, v in enumerate(self.cap_choices):
            c.cap_choices[i] = v
        c.mid0 = self.mid0
        c.snapshot_fill_pct = self.snapshot_fill_pct
        c.exec_pct = self.exec_pct
        c.ignored_pct = self.ignored_pct
        c.seed = self.seed
        return c


# The benchmark workloads (sizes, mixes and agent sets of the paper's evaluation
# setting, synthetic data standing in for LOBSTER replay).
WORKLOADS = {
    # single env, plain replay, no agents, 10^6 messages in 10,000 steps of 100
    "replay1": Workload("replay1", n_envs=1, n_steps=10_000, msgs_per_step=100, cap=100,
                        seed=SEED_BASE + 1),
    # 4096 envs, 100 msgs/step, execution + market-making agent, 128-step episodes
    "uniform4096": Workload("uniform4096", n_envs=4096, n_steps=128, msgs_per_step=100, cap=100,
                            agents=("exec", "mm"), seed=SEED_BASE + 2),
    # 8192 uneven envs: cap uniform in {50,100,200,400}, msgs/step uniform in 1..400
    "uneven8192": Workload("uneven8192", n_envs=8192, n_steps=128, msgs_range=(1, 400),
                           cap_choices=(50, 100, 200, 400), agents=("exec", "mm"),
                           seed=SEED_BASE + 3),
    # IPPO rollout feeding two actor-critics
    "ippo4096": Workload("ippo4096", n_envs=4096, n_steps=128, msgs_per_step=100, cap=100,
                         agents=("exec", "mm"), seed=SEED_BASE + 4),
    # large: cap 1000, 400 msgs/step, 10% burst steps with 480 extra cancels, 3 agents
    "large16384": Workload("large16384", n_envs=16384, n_steps=256, msgs_per_step=400,
                           burst_pct=10, burst_extra=480, cap=1000,
                           agents=("exec", "mm", "dir"), seed=SEED_BASE + 5),
}


@dataclasses.dataclass
class Stream:
    """Generated inputs: SoA messages, CSR offsets, capacities, reset snapshot."""

    workload: Workload
    caps: np.ndarray          # int32 [n_envs]
    off: np.ndarray           # int64 [n_envs, n_steps+1]
    ts: np.ndarray            # int32 [n_msgs] type | side << 8
    price: np.ndarray
    qty: np.ndarray
    oid: np.ndarray
    tid: np.ndarray
    tsec: np.ndarray
    tns: np.ndarray
    book: dict                # price/qty/oid/tid/tsec/tns int32 [n_envs,2,max_cap], n int32 [n_envs,2]

    @property
    def n_msgs(self) -> int:
        return int(self.off[-1, -1])

    def msg_fields(self):
        return (self.ts, self.price, self.qty, self.oid, self.tid, self.tsec, self.tns)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def env_caps(w: Workload) -> np.ndarray:
    lib = _load()
    c = w._cfg()
    return np.array([lib.synth_env_cap(ctypes.byref(c), e) for e in range(w.n_envs)], dtype=np.int32)


def generate(w: Workload, threads: Optional[int] = None) -> Stream:
    """Generate the reset snapshot and message stream of every env of ``w``."""
    lib = _load()
    c = w._cfg()
    off = np.empty((w.n_envs, w.n_steps + 1), dtype=np.int64)
    total = int(lib.synth_offsets(ctypes.byref(c), _ptr(off)))
    fields = [np.empty(max(total, 1), dtype=np.int32) for _ in range(7)]
    mc = w.max_cap
    book = {k: np.empty((w.n_envs, 2, mc), dtype=np.int32)
            for k in ("price", "qty", "oid", "tid", "tsec", "tns")}
    book["n"] = np.empty((w.n_envs, 2), dtype=np.int32)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rc = lib.synth_generate(ctypes.byref(c), _ptr(off), mc, *[_ptr(f) for f in fields],
                            *[_ptr(book[k]) for k in ("price", "qty", "oid", "tid", "tsec", "tns", "n")],
                            int(threads))
    if rc != 0:
        raise ValueError("synth_generate rejected the workload")
    caps = env_caps(w)
    fields = [f[:total] for f in fields]
    return Stream(w, caps, off, *fields, book)


def size_table() -> np.ndarray:
    lib = _load()
    out = np.empty(4096, dtype=np.int32)
    lib.synth_size_table(_ptr(out))
    return out


def u32(seed: int, e: int, t: int, m: int, field: int) -> int:
    return int(_load().synth_u32(seed, e, t, m, field))


def agent_kinds(agents: Sequence[str]) -> np.ndarray:
    return np.array([AGENT_KINDS[a] for a in agents], dtype=np.int32)

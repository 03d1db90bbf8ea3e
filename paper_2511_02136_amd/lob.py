"""Python binding of liblob (ctypes): argument marshalling only.

Every step of the environment runs in the HIP kernels of ``liblob.so``; PyTorch is used
for device memory and streams.  The binding fails loudly when the library is missing or
no GPU is visible: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblob.so")
_lib = None

OBS_DIM = 40
TRADE_WORDS = 8
N_COUNTERS = 11
ENV_STATE_WORDS = 12
AGENT_STATE_WORDS = 6
BOOK_FIELDS = ("price", "qty", "oid", "tid", "tsec", "tns")
# actions of each agent kind (directional 3; the TWAP and Avellaneda-Stoikov baselines 1)
N_ACTIONS = {0: 9, 1: 9, 2: 3, 3: 9, 4: 9, 5: 9, 6: 1, 7: 1}
AGENT_KINDS = {"exec": 0, "mm": 1, "dir": 2, "mm_buysell": 3, "mm_spreadskew": 4, "mm_avst": 5, "exec_twap": 6,
               "mm_as": 7}


class LobError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32), ("n_agents", ctypes.c_int32), ("max_cap", ctypes.c_int32),
        ("episode_len", ctypes.c_int32), ("cap", ctypes.c_void_p), ("agent_kind", ctypes.c_void_p),
        ("seed", ctypes.c_uint64), ("exec_task", ctypes.c_int32), ("exec_q0", ctypes.c_int32),
        ("mm_q", ctypes.c_int32), ("dir_q", ctypes.c_int32), ("exec_penalty", ctypes.c_float),
        ("mm_lambda", ctypes.c_float), ("mm_rho", ctypes.c_float), ("flags", ctypes.c_uint32),
        ("avst_gamma", ctypes.c_float), ("avst_sigma2", ctypes.c_float), ("avst_kappa", ctypes.c_float),
    ]


class _Msgs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("ts", "price", "qty", "oid", "tid", "tsec", "tns", "off")] + [
        ("n_steps", ctypes.c_int32), ("n_msgs", ctypes.c_int64)]


class _Books(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in BOOK_FIELDS + ("n",)]


class _Out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("trades", "trade_off", "trade_cursor", "n_trades", "fills",
                                                "reward", "obs", "done", "actions")]


def lib():
    """The loaded liblob.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LobError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        p, i32 = ctypes.c_void_p, ctypes.c_int32
        L.lob_init.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(p)]
        L.lob_reset.argtypes = [p, ctypes.POINTER(_Books), p]
        L.lob_step.argtypes = [p, ctypes.POINTER(_Msgs), p, ctypes.POINTER(_Out), p]
        L.lob_rollout.argtypes = [p, ctypes.POINTER(_Msgs), i32, p, ctypes.POINTER(_Out), p]
        L.lob_observe.argtypes = [p, p, p]
        L.lob_export_books.argtypes = [p, ctypes.POINTER(_Books), p]
        L.lob_export_state.argtypes = [p, p, p, p, p]
        L.lob_import_state.argtypes = [p, ctypes.POINTER(_Books), p, p, p, i32, p]
        L.lob_current_step.argtypes = [p]
        L.lob_plan.argtypes = [p, ctypes.POINTER(_Msgs), i32]
        L.lob_schedule_get.argtypes = [p, p, i32]
        L.lob_schedule_set.argtypes = [p, i32, i32, i32, i32]
        L.lob_set_padded.argtypes = [p, i32]
        L.lob_schedule_balance.argtypes = [p, i32]
        L.lob_autotune.argtypes = [p, ctypes.POINTER(_Msgs), i32, ctypes.POINTER(_Out), p]
        L.lob_destroy.argtypes = [p]
        L.lob_strerror.argtypes = [ctypes.c_int]
        L.lob_strerror.restype = ctypes.c_char_p
        for f in ("lob_init", "lob_reset", "lob_step", "lob_rollout", "lob_observe", "lob_export_books",
                  "lob_export_state", "lob_import_state", "lob_current_step", "lob_destroy", "lob_plan", "lob_schedule_get",
                  "lob_schedule_set", "lob_set_padded", "lob_schedule_balance", "lob_autotune"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise LobError(f"{what}: {lib().lob_strerror(rc).decode()} ({rc})")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu(device):
    if not torch.cuda.is_available():
        raise LobError("no GPU visible: the LOB environment runs only in its HIP kernels")
    return torch.device(device)


class DeviceStream:
    """A market-by-order stream resident in device memory (CSR over envs and steps)."""

    def __init__(self, fields: Sequence[torch.Tensor], off: torch.Tensor):
        self.fields = [f.contiguous() for f in fields]
        self.off = off.contiguous()
        self.n_envs = self.off.shape[0]
        self.n_steps = self.off.shape[1] - 1
        self.n_msgs = int(self.fields[0].numel())
        m = _Msgs()
        for name, f in zip(("ts", "price", "qty", "oid", "tid", "tsec", "tns"), self.fields):
            setattr(m, name, f.data_ptr())
        m.off = self.off.data_ptr()
        m.n_steps = self.n_steps
        m.n_msgs = self.n_msgs
        self._m = m

    @classmethod
    def from_host(cls, stream, device="cuda") -> "DeviceStream":
        dev = _require_gpu(device)
        fields = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in stream.msg_fields()]
        off = torch.from_numpy(np.ascontiguousarray(stream.off, dtype=np.int64)).to(dev)
        return cls(fields, off)

    def trade_regions(self, caps: torch.Tensor, t0: int, n_steps: int, n_agents: int) -> torch.Tensor:
        """Per-env trade-record regions [n_envs+1] that cannot overflow over steps
        [t0, t0+n_steps): every trade consumes a resting order or ends an incoming one,
        so at most 2*cap + 2*(messages + 8 agent orders per agent per step) records."""
        t0 = min(max(t0, 0), self.n_steps)
        t1 = min(t0 + n_steps, self.n_steps)
        msgs = self.off[:, t1] - self.off[:, t0]
        bound = 2 * caps.to(torch.int64) + 2 * (msgs + n_steps * n_agents * 8)
        return torch.cat([torch.zeros(1, dtype=torch.int64, device=self.off.device), torch.cumsum(bound, 0)])


class LobEnv:
    """Batched LOB environments on one GPU (one context of liblob)."""

    def __init__(self, caps, max_cap: int, agents: Sequence = (), episode_len: int = 128, seed: int = 0,
                 exec_task: int = 500, exec_q0: int = 4, mm_q: int = 10, dir_q: int = 10,
                 exec_penalty: float = 0.01, mm_lambda: float = 0.0, mm_rho: float = 0.0,
                 avst_gamma: float = 0.01, avst_sigma2: float = 10.0, avst_kappa: float = 0.5, device="cuda"):
        self.device = _require_gpu(device)
        self._lib = lib()
        self.caps_host = np.ascontiguousarray(np.asarray(caps, dtype=np.int32).reshape(-1))
        kinds = [AGENT_KINDS[k] if isinstance(k, str) else int(k) for k in agents]
        self.kinds = np.ascontiguousarray(np.asarray(kinds, dtype=np.int32))
        self.n_envs = int(self.caps_host.shape[0])
        self.n_agents = int(self.kinds.shape[0])
        self.max_cap = int(max_cap)
        self.episode_len = int(episode_len)
        self.caps = torch.from_numpy(self.caps_host).to(self.device)
        c = _Config()
        c.n_envs, c.n_agents, c.max_cap, c.episode_len = self.n_envs, self.n_agents, self.max_cap, self.episode_len
        c.cap = self.caps_host.ctypes.data
        c.agent_kind = self.kinds.ctypes.data if self.n_agents else None
        c.seed = seed
        c.exec_task, c.exec_q0, c.mm_q, c.dir_q = exec_task, exec_q0, mm_q, dir_q
        c.exec_penalty, c.mm_lambda, c.mm_rho = exec_penalty, mm_lambda, mm_rho
        c.avst_gamma, c.avst_sigma2, c.avst_kappa = avst_gamma, avst_sigma2, avst_kappa
        c.flags = 0
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.lob_init(ctypes.byref(c), ctypes.byref(h)), "lob_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lob_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return int(self._lib.lob_current_step(self._h))

    # ---- state ----
    def reset(self, book: dict):
        bt = {k: torch.as_tensor(np.ascontiguousarray(book[k]) if isinstance(book[k], np.ndarray) else book[k])
              .to(self.device, torch.int32).contiguous() for k in BOOK_FIELDS + ("n",)}
        for k in BOOK_FIELDS:
            if tuple(bt[k].shape) != (self.n_envs, 2, self.max_cap):
                raise LobError(f"snapshot field {k} must be [{self.n_envs}, 2, {self.max_cap}]")
        if tuple(bt["n"].shape) != (self.n_envs, 2):
            raise LobError("snapshot n must be [n_envs, 2]")
        b = _Books(*[bt[k].data_ptr() for k in BOOK_FIELDS + ("n",)])
        _check(self._lib.lob_reset(self._h, ctypes.byref(b), _stream()), "lob_reset")
        self._keep = bt  # alive until the stream has consumed it
        return self

    def _alloc_out(self, n_steps: int, obs: bool, record_trades: bool, trade_off, dstream: DeviceStream,
                   actions_out: bool = True):
        N, A, dev = self.n_envs, self.n_agents, self.device
        out = {
            "n_trades": torch.empty((n_steps, N), dtype=torch.int32, device=dev),
            "fills": torch.empty((n_steps, A, N, 4), dtype=torch.int64, device=dev),
            "reward": torch.empty((n_steps, A, N), dtype=torch.float32, device=dev),
            "obs": torch.empty((n_steps, A, N, OBS_DIM), dtype=torch.float32, device=dev) if obs else None,
            "done": torch.empty((n_steps, N), dtype=torch.uint8, device=dev),
            "actions": torch.empty((n_steps, A, N), dtype=torch.int32, device=dev) if actions_out else None,
        }
        if record_trades:
            if trade_off is None:
                trade_off = dstream.trade_regions(self.caps, self.t, n_steps, A)
            trade_off = torch.as_tensor(trade_off).to(dev, torch.int64).contiguous()
            out["trade_off"] = trade_off
            out["trades"] = torch.empty((int(trade_off[-1].item()), TRADE_WORDS), dtype=torch.int32, device=dev)
        else:
            out["trade_off"] = None
            out["trades"] = None
        return out

    @staticmethod
    def _out_struct(out: dict, cursor: Optional[torch.Tensor] = None) -> _Out:
        o = _Out()
        for k in ("trades", "trade_off", "n_trades", "fills", "reward", "obs", "done", "actions"):
            t = out.get(k)
            setattr(o, k, None if t is None else t.data_ptr())
        o.trade_cursor = None if cursor is None else cursor.data_ptr()
        return o

    def step(self, dstream: DeviceStream, actions: Optional[torch.Tensor] = None, obs: bool = True,
             record_trades: bool = True, trade_off=None, out: Optional[dict] = None,
             cursor: Optional[torch.Tensor] = None) -> dict:
        """One env-step of every env (plain per-step launch)."""
        if out is None:
            out = self._alloc_out(1, obs, record_trades, trade_off, dstream)
        if actions is not None:
            actions = actions.to(self.device, torch.int32).contiguous().reshape(self.n_agents, self.n_envs)
        o = self._out_struct(out, cursor)
        _check(self._lib.lob_step(self._h, ctypes.byref(dstream._m), _p(actions), ctypes.byref(o), _stream()),
               "lob_step")
        out["_actions_in"] = actions
        return out

    def rollout(self, dstream: DeviceStream, n_steps: int, actions: Optional[torch.Tensor] = None,
                obs: bool = True, record_trades: bool = True, trade_off=None, out: Optional[dict] = None,
                cursor: Optional[torch.Tensor] = None) -> dict:
        """n_steps env-steps in one persistent launch per capacity class."""
        if out is None:
            out = self._alloc_out(n_steps, obs, record_trades, trade_off, dstream)
        if actions is not None:
            actions = actions.to(self.device, torch.int32).contiguous().reshape(n_steps, self.n_agents, self.n_envs)
        o = self._out_struct(out, cursor)
        _check(self._lib.lob_rollout(self._h, ctypes.byref(dstream._m), int(n_steps), _p(actions), ctypes.byref(o),
                                     _stream()), "lob_rollout")
        out["_actions_in"] = actions
        return out

    # ---- schedule ----
    def plan(self, dstream: DeviceStream, n_steps: int):
        """Order each capacity class's envs longest first for the next n_steps."""
        _check(self._lib.lob_plan(self._h, ctypes.byref(dstream._m), int(n_steps)), "lob_plan")

    def schedule(self) -> list:
        buf = np.zeros((64, 5), dtype=np.int32)
        n = self._lib.lob_schedule_get(self._h, buf.ctypes.data_as(ctypes.c_void_p), 64)
        if n < 0:
            _check(n, "lob_schedule_get")
        return [dict(cap_slots=int(r[0]), envs=int(r[1]), waves=int(r[2]), mode=int(r[3]), grid=int(r[4]))
                for r in buf[:n]]

    def set_schedule(self, k: int, waves: int, mode: int, grid: int = 0):
        _check(self._lib.lob_schedule_set(self._h, k, waves, mode, grid), "lob_schedule_set")

    def set_balance(self, permille: int):
        """Proportional work-queue schedule of several concurrent classes sized to
        permille/1000 of the LDS from the next plan on; 0 returns every class to its
        default schedule (see lob_schedule_balance)."""
        _check(self._lib.lob_schedule_balance(self._h, int(permille)), "lob_schedule_balance")

    def set_padded(self, padded: bool):
        """Batching ablation: one class padded to the largest capacity (True) or one
        class per book row count (False, the default).  Resets plan and schedules."""
        _check(self._lib.lob_set_padded(self._h, int(bool(padded))), "lob_set_padded")

    def autotune(self, dstream: DeviceStream, n_steps: int, out: Optional[dict] = None) -> list:
        """Time schedule candidates on the next n_steps (state restored) and keep the
        fastest (see lob_autotune).  Returns the chosen schedule."""
        if out is None:
            out = self._alloc_out(n_steps, True, True, None, dstream)
        o = self._out_struct(out)
        _check(self._lib.lob_autotune(self._h, ctypes.byref(dstream._m), int(n_steps), ctypes.byref(o), _stream()),
               "lob_autotune")
        return self.schedule()

    def observe(self) -> torch.Tensor:
        obs = torch.empty((self.n_agents, self.n_envs, OBS_DIM), dtype=torch.float32, device=self.device)
        _check(self._lib.lob_observe(self._h, _p(obs), _stream()), "lob_observe")
        return obs

    def books(self) -> dict:
        N, mc, dev = self.n_envs, self.max_cap, self.device
        b = {k: torch.empty((N, 2, mc), dtype=torch.int32, device=dev) for k in BOOK_FIELDS}
        b["n"] = torch.empty((N, 2), dtype=torch.int32, device=dev)
        s = _Books(*[b[k].data_ptr() for k in BOOK_FIELDS + ("n",)])
        _check(self._lib.lob_export_books(self._h, ctypes.byref(s), _stream()), "lob_export_books")
        return b

    def state(self) -> dict:
        N, A, dev = self.n_envs, self.n_agents, self.device
        es = torch.empty((N, ENV_STATE_WORDS), dtype=torch.int64, device=dev)
        ag = torch.empty((N, max(A, 1), AGENT_STATE_WORDS), dtype=torch.int64, device=dev)
        ct = torch.empty((N, N_COUNTERS), dtype=torch.int64, device=dev)
        _check(self._lib.lob_export_state(self._h, _p(es), _p(ag) if A else None, _p(ct), _stream()),
               "lob_export_state")
        return {"env": es, "agents": ag[:, :A], "counters": ct}

    def import_state(self, books: dict, state: dict, step: int):
        """Continue every env from ``books`` (canonical layout, as ``books()`` returns) and
        ``state`` (the layouts of ``state()``; counters optional) with the step counter at
        ``step`` (see lob_import_state)."""
        N, A, dev = self.n_envs, self.n_agents, self.device
        bt = {k: torch.as_tensor(books[k]).to(dev, torch.int32).contiguous() for k in BOOK_FIELDS + ("n",)}
        for k in BOOK_FIELDS:
            if tuple(bt[k].shape) != (N, 2, self.max_cap):
                raise LobError(f"books field {k} must be [{N}, 2, {self.max_cap}]")
        if tuple(bt["n"].shape) != (N, 2):
            raise LobError("books n must be [n_envs, 2]")
        es = torch.as_tensor(state["env"]).to(dev, torch.int64).contiguous()
        if tuple(es.shape) != (N, ENV_STATE_WORDS):
            raise LobError(f"env state must be [{N}, {ENV_STATE_WORDS}]")
        ag = None
        if A:
            ag = torch.as_tensor(state["agents"]).to(dev, torch.int64).contiguous()
            if tuple(ag.shape) != (N, A, AGENT_STATE_WORDS):
                raise LobError(f"agent state must be [{N}, {A}, {AGENT_STATE_WORDS}]")
        ct = state.get("counters")
        if ct is not None:
            ct = torch.as_tensor(ct).to(dev, torch.int64).contiguous()
            if tuple(ct.shape) != (N, N_COUNTERS):
                raise LobError(f"counters must be [{N}, {N_COUNTERS}]")
        b = _Books(*[bt[k].data_ptr() for k in BOOK_FIELDS + ("n",)])
        _check(self._lib.lob_import_state(self._h, ctypes.byref(b), _p(es), _p(ag), _p(ct), int(step), _stream()),
               "lob_import_state")
        self._keep = (bt, es, ag, ct)  # alive until the stream has consumed them
        return self

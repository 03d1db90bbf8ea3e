"""Test helpers: hand-built streams and snapshots in the library's SoA layouts."""
from __future__ import annotations

import dataclasses

import numpy as np

FIELDS = ("price", "qty", "oid", "tid", "tsec", "tns")


@dataclasses.dataclass
class HandStream:
    off: np.ndarray
    ts: np.ndarray
    price: np.ndarray
    qty: np.ndarray
    oid: np.ndarray
    tid: np.ndarray
    tsec: np.ndarray
    tns: np.ndarray

    def msg_fields(self):
        return (self.ts, self.price, self.qty, self.oid, self.tid, self.tsec, self.tns)

    @property
    def n_msgs(self):
        return int(self.off[-1, -1])


def hand_stream(per_env_steps):
    """per_env_steps[e][t] = list of 7-int messages [ts, price, qty, oid, tid, tsec, tns]."""
    n_envs = len(per_env_steps)
    n_steps = len(per_env_steps[0])
    off = np.zeros((n_envs, n_steps + 1), dtype=np.int64)
    rows = []
    pos = 0
    for e in range(n_envs):
        for t in range(n_steps):
            off[e, t] = pos
            for m in per_env_steps[e][t]:
                rows.append(m)
                pos += 1
        off[e, n_steps] = pos
    arr = np.array(rows, dtype=np.int32).reshape(-1, 7) if rows else np.zeros((0, 7), np.int32)
    cols = [np.ascontiguousarray(arr[:, k]) if len(rows) else np.zeros(1, np.int32) for k in range(7)]
    return HandStream(off, *cols)


def hand_book(per_env, max_cap):
    """per_env[e] = (bids, asks), each a list of [price, qty, oid, tid, tsec, tns]."""
    n = len(per_env)
    b = {k: np.zeros((n, 2, max_cap), dtype=np.int32) for k in FIELDS}
    b["n"] = np.zeros((n, 2), dtype=np.int32)
    for e, sides in enumerate(per_env):
        for s, orders in enumerate(sides):
            b["n"][e, s] = len(orders)
            for j, o in enumerate(orders):
                for k, f in enumerate(FIELDS):
                    b[f][e, s, j] = o[k]
    return b


def book_lists(b, e):
    """(bids, asks) of env e from the SoA layout, as lists of 6-int records."""
    out = []
    for s in (0, 1):
        n = int(b["n"][e, s])
        out.append([[int(b[f][e, s, j]) for f in FIELDS] for j in range(n)])
    return out[0], out[1]


def msg(typ, side, price, qty, oid, tid=0, tsec=0, tns=0):
    return [typ | (side << 8), price, qty, oid, tid, tsec, tns]


def subset_stream(stream, envs):
    """The inputs of a subset of envs (same messages, CSR rebased), for sampled parity."""
    envs = np.asarray(envs, dtype=np.int64)
    off = stream.off
    parts = [np.arange(off[e, 0], off[e, -1]) for e in envs]
    idx = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    lens = off[envs, -1] - off[envs, 0]
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    new_off = off[envs] - off[envs, :1] + starts[:, None]
    fields = [np.ascontiguousarray(f[idx]) for f in stream.msg_fields()]
    hs = HandStream(np.ascontiguousarray(new_off), *fields)
    book = {k: np.ascontiguousarray(v[envs]) for k, v in stream.book.items()}
    return hs, book, np.ascontiguousarray(stream.caps[envs])

"""LOBSTER-format ingestion: message files and order-book snapshots into the library's
message stream (structure of arrays, CSR over envs x steps) and reset books.

The paper replays LOBSTER market-by-order data through the JAX-LOB simulator (Sec. 4,
Table 2).  A LOBSTER message file has one row per event: time (seconds after midnight,
up to nanosecond decimals), type, order id, size, price (dollars x 10^4) and direction
(1 a buy limit order, -1 a sell limit order; for executions, the side of the executed
resting order).  An order-book file has, for each message, the book after it: for every
level k, ask price, ask size, bid price, bid size (empty levels carry the sentinels
+-9999999999 and size 0).

Type mapping onto the library's messages (include/lob.h):
  1 new limit order          -> 1 LIMIT
  2 partial cancellation     -> 2 PARTIAL_CANCEL
  3 deletion                 -> 3 DELETE
  4 execution (visible)      -> 5 EXECUTE (of the resting order named by its id)
  5 execution (hidden), 6 cross trade, 7 trading halt -> 6 IGNORED
Prices become ticks (price / tick, tick in LOBSTER units: 100 = one cent).  Order ids
outside [0, 2^30 - 2^20) (the library reserves 2^30 and above for agents, the block
below it for the reset books' level orders) are renumbered consistently to ids no
message uses.
The reset book of an env is the order-book row just before its first message, one
order per non-empty level (ids from a reserved block below 2^30); cancels and
executions of orders placed before that row find no order and count as misses.

Everything here is host-side data preparation; no book arithmetic happens here.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import synth

LOBSTER_TO_TYPE = {1: 1, 2: 2, 3: 3, 4: 5, 5: 6, 6: 6, 7: 6}
TYPE_TO_LOBSTER = {1: 1, 2: 2, 3: 3, 5: 4, 6: 5}
EMPTY_ASK, EMPTY_BID = 9999999999, -9999999999
AGENT_ID_BIT = 1 << 30
SNAPSHOT_ID_BASE = AGENT_ID_BIT - (1 << 20)  # ids of the reset books' level orders


@dataclasses.dataclass
class Messages:
    """One LOBSTER message file in the library's encoding (int32 each)."""
    ts: np.ndarray      # type | side << 8
    price: np.ndarray   # ticks
    qty: np.ndarray
    oid: np.ndarray
    tid: np.ndarray
    tsec: np.ndarray
    tns: np.ndarray

    def __len__(self) -> int:
        return int(self.ts.shape[0])


def _split_time(s: str) -> Tuple[int, int]:
    """'34200.004241176' -> (34200, 4241176), exactly (no float rounding)."""
    if "." in s:
        a, b = s.split(".", 1)
        b = (b + "000000000")[:9]
    else:
        a, b = s, "0"
    return int(a), int(b)


def read_messages(path: str, tick: int = 100) -> Messages:
    """Parse a LOBSTER message file (CSV, no header)."""
    rows: List[Tuple] = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            t, typ, oid, size, price, direction = [x.strip() for x in line.split(",")[:6]]
            rows.append((t, int(typ), int(oid), int(size), int(price), int(direction)))
    n = len(rows)
    out = Messages(*[np.zeros(n, dtype=np.int32) for _ in range(7)])
    # ids outside [0, SNAPSHOT_ID_BASE) get fresh ids below it that no message uses
    used = {r[2] for r in rows if 0 <= r[2] < SNAPSHOT_ID_BASE}
    remap: Dict[int, int] = {}
    fresh = SNAPSHOT_ID_BASE - 1
    for i, (t, typ, oid, size, price, direction) in enumerate(rows):
        if typ not in LOBSTER_TO_TYPE:
            raise ValueError(f"{path}: row {i}: unknown LOBSTER message type {typ}")
        if direction not in (1, -1):
            raise ValueError(f"{path}: row {i}: direction must be 1 or -1")
        if not 0 <= oid < SNAPSHOT_ID_BASE:
            if oid not in remap:
                while fresh in used:
                    fresh -= 1
                remap[oid] = fresh
                used.add(fresh)
            oid = remap[oid]
        sec, ns = _split_time(t)
        out.ts[i] = LOBSTER_TO_TYPE[typ] | ((0 if direction == 1 else 1) << 8)
        out.price[i] = price // tick
        out.qty[i] = size
        out.oid[i] = oid
        out.tsec[i] = sec
        out.tns[i] = ns
    return out


def write_messages(path: str, m: Messages, tick: int = 100) -> None:
    """Write messages in LOBSTER's message-file format (the inverse of read_messages for
    types 1-3, 5 and 6; ignored messages are written as hidden executions)."""
    with open(path, "w") as f:
        for i in range(len(m)):
            typ, side = int(m.ts[i]) & 0xFF, (int(m.ts[i]) >> 8) & 1
            if typ not in TYPE_TO_LOBSTER:
                raise ValueError(f"message {i}: type {typ} has no LOBSTER form")
            f.write(f"{int(m.tsec[i])}.{int(m.tns[i]):09d},{TYPE_TO_LOBSTER[typ]},{int(m.oid[i])},"
                    f"{int(m.qty[i])},{int(m.price[i]) * tick},{1 if side == 0 else -1}\n")


def read_orderbook_row(path: str, row: int, tick: int = 100) -> Tuple[List[Tuple[int, int]], List[Tuple[int, int]]]:
    """Levels of one order-book row: (bids, asks), each [(price ticks, size)] best first,
    empty levels dropped."""
    with open(path) as f:
        for i, line in enumerate(f):
            if i == row:
                v = [int(x) for x in line.strip().split(",")]
                break
        else:
            raise ValueError(f"{path}: no row {row}")
    if len(v) % 4:
        raise ValueError(f"{path}: row {row} has {len(v)} fields, not a multiple of 4")
    bids, asks = [], []
    for k in range(len(v) // 4):
        ap, asz, bp, bsz = v[4 * k: 4 * k + 4]
        if asz > 0 and ap != EMPTY_ASK:
            asks.append((ap // tick, asz))
        if bsz > 0 and bp != EMPTY_BID:
            bids.append((bp // tick, bsz))
    return bids, asks


def write_orderbook(path: str, rows: Sequence[Tuple[Sequence[Tuple[int, int]], Sequence[Tuple[int, int]]]],
                    levels: int, tick: int = 100) -> None:
    """Write order-book rows ((bids, asks) in ticks, best first) in LOBSTER's format."""
    with open(path, "w") as f:
        for bids, asks in rows:
            v = []
            for k in range(levels):
                ap, asz = (asks[k][0] * tick, asks[k][1]) if k < len(asks) else (EMPTY_ASK, 0)
                bp, bsz = (bids[k][0] * tick, bids[k][1]) if k < len(bids) else (EMPTY_BID, 0)
                v += [ap, asz, bp, bsz]
            f.write(",".join(str(x) for x in v) + "\n")


def build_stream(m: Messages, starts: Sequence[int], n_steps: int, msgs_per_step: int, cap: int,
                 books: Sequence[Tuple[Sequence[Tuple[int, int]], Sequence[Tuple[int, int]]]],
                 agents: Tuple[str, ...] = (), seed: int = synth.SEED_BASE) -> synth.Stream:
    """Env e replays messages [starts[e], starts[e] + n_steps * msgs_per_step) of m,
    msgs_per_step per env-step, from the reset book books[e] = (bids, asks) (one order per
    level, at most cap per side, timed at the env's first message).  Returns a stream the
    library and the oracle take like a generated one."""
    n_envs = len(starts)
    span = n_steps * msgs_per_step
    if len(books) != n_envs:
        raise ValueError("one reset book per env")
    for s0 in starts:
        if s0 < 0 or s0 + span > len(m):
            raise ValueError(f"window [{s0}, {s0 + span}) outside the {len(m)} messages")
    idx = np.concatenate([np.arange(s0, s0 + span, dtype=np.int64) for s0 in starts])
    off = (np.arange(n_envs, dtype=np.int64)[:, None] * span
           + np.arange(n_steps + 1, dtype=np.int64)[None, :] * msgs_per_step)
    w = synth.Workload("lobster", n_envs=n_envs, n_steps=n_steps, msgs_per_step=msgs_per_step, cap=cap,
                       agents=tuple(agents), seed=seed)
    book = {k: np.zeros((n_envs, 2, cap), dtype=np.int32) for k in ("price", "qty", "oid", "tid", "tsec", "tns")}
    book["n"] = np.zeros((n_envs, 2), dtype=np.int32)
    for e, (bids, asks) in enumerate(books):
        s0 = starts[e]
        for s, lv in ((0, bids), (1, asks)):
            lv = list(lv)[:cap]
            for i, (p, q) in enumerate(lv):
                book["price"][e, s, i] = p
                book["qty"][e, s, i] = q
                book["oid"][e, s, i] = SNAPSHOT_ID_BASE + 2 * i + s
                book["tsec"][e, s, i] = m.tsec[s0]
                book["tns"][e, s, i] = m.tns[s0]
            book["n"][e, s] = len(lv)
    return synth.Stream(workload=w, caps=np.full(n_envs, cap, dtype=np.int32), off=off,
                        ts=m.ts[idx].copy(), price=m.price[idx].copy(), qty=m.qty[idx].copy(),
                        oid=m.oid[idx].copy(), tid=m.tid[idx].copy(), tsec=m.tsec[idx].copy(),
                        tns=m.tns[idx].copy(), book=book)


def books_before(orderbook_path: str, starts: Sequence[int], tick: int = 100):
    """The reset books of envs starting at message starts[e]: the order-book row of the
    message just before (an empty book for a start at the first message)."""
    return [lobster_row_or_empty(orderbook_path, s0 - 1, tick) for s0 in starts]


def lobster_row_or_empty(orderbook_path: str, row: int, tick: int = 100):
    return ([], []) if row < 0 else read_orderbook_row(orderbook_path, row, tick)

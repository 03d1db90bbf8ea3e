"""Pins of the oracle's order book (matching, cancels, full-book rule).

The paper defines the book as a continuous double auction with price-time priority
(Sec. 2.1) and defers the rest to the JAX-LOB simulator, which is not available.  The
oracle is pinned here by:
  * hand-worked examples computed from the definition of price-time priority;
  * brute force against a naive sorted-list book (tests/naive_book.py) on every short
    sequence over a tiny alphabet and on random longer sequences;
  * invariants checked after every message (no crossed book, capacity, positive
    quantities, priority order, unique ids, quantity conservation);
  * special cases that reduce to textbook routines (sorted insertion, FIFO queue).
"""
import itertools
import random

import numpy as np
import pytest

from naive_book import NaiveBook
from oracle import OracleBook, COUNTER_NAMES

LIMIT, PARTIAL_CANCEL, DELETE, MARKET, EXECUTE, IGNORED = 1, 2, 3, 4, 5, 6
BUY, SELL = 0, 1
CI = {n: i for i, n in enumerate(COUNTER_NAMES)}


def ts(typ, side):
    return typ | (side << 8)


def book_view(b, s):
    """(price, qty, oid) of side s in priority order."""
    return [tuple(int(v) for v in o[:3]) for o in b.side(s)]


def trade_view(tr):
    """(price, qty, agg_oid, pas_oid) of each trade."""
    return [tuple(int(v) for v in t[:4]) for t in tr]


# ----------------------------------------------------------------------------------
# hand-worked examples
# ----------------------------------------------------------------------------------
def test_crossing_limits_partial_fills_and_resting_remainder():
    b = OracleBook(4)
    for side, p, q, oid in [(SELL, 101, 5, 1), (SELL, 101, 3, 2), (SELL, 102, 4, 3), (BUY, 99, 2, 4)]:
        assert len(b.process(ts(LIMIT, side), p, q, oid)) == 0
    assert book_view(b, SELL) == [(101, 5, 1), (101, 3, 2), (102, 4, 3)]
    assert book_view(b, BUY) == [(99, 2, 4)]
    # a buy for 7 at 101 takes all of #1 then 2 of #2, both at 101; nothing rests
    tr = b.process(ts(LIMIT, BUY), 101, 7, 5)
    assert trade_view(tr) == [(101, 5, 5, 1), (101, 2, 5, 2)]
    assert book_view(b, SELL) == [(101, 1, 2), (102, 4, 3)]
    assert book_view(b, BUY) == [(99, 2, 4)]
    # a buy for 6 at 102 sweeps two levels at the resting prices; 1 rests at 102
    tr = b.process(ts(LIMIT, BUY), 102, 6, 6)
    assert trade_view(tr) == [(101, 1, 6, 2), (102, 4, 6, 3)]
    assert book_view(b, BUY) == [(102, 1, 6), (99, 2, 4)]
    assert book_view(b, SELL) == []
    # trade records carry aggressor side and ids
    assert int(tr[0][4]) == 0 and int(tr[0][6]) & 1 == BUY

    # cancels: partial keeps the order, an oversize partial removes it, a second delete
    # misses, and a delete on the wrong side misses
    b.process(ts(PARTIAL_CANCEL, BUY), 99, 1, 4)
    assert book_view(b, BUY) == [(102, 1, 6), (99, 1, 4)]
    b.process(ts(PARTIAL_CANCEL, BUY), 99, 5, 4)
    assert book_view(b, BUY) == [(102, 1, 6)]
    b.process(ts(DELETE, BUY), 99, 0, 4)
    b.process(ts(DELETE, SELL), 102, 0, 6)
    assert book_view(b, BUY) == [(102, 1, 6)]
    assert b.counters[CI["miss"]] == 2
    assert b.counters[CI["trades"]] == 4


def test_full_book_evict_drop_and_market_orders():
    b = OracleBook(2)
    b.process(ts(LIMIT, BUY), 100, 3, 10)
    b.process(ts(LIMIT, BUY), 101, 2, 11)
    assert book_view(b, BUY) == [(101, 2, 11), (100, 3, 10)]
    # full: 101 is strictly better than the worst (100) -> evict #10
    b.process(ts(LIMIT, BUY), 101, 4, 12)
    assert book_view(b, BUY) == [(101, 2, 11), (101, 4, 12)]
    assert b.counters[CI["evict"]] == 1 and b.counters[CI["evicted_qty"]] == 3
    # 100 is worse than the worst; 101 equals the worst and arrives later: both dropped
    b.process(ts(LIMIT, BUY), 100, 1, 13)
    b.process(ts(LIMIT, BUY), 101, 1, 16)
    assert book_view(b, BUY) == [(101, 2, 11), (101, 4, 12)]
    assert b.counters[CI["drop"]] == 2 and b.counters[CI["dropped_qty"]] == 2
    tr = b.process(ts(MARKET, SELL), 0, 5, 14)
    assert trade_view(tr) == [(101, 2, 14, 11), (101, 3, 14, 12)]
    assert book_view(b, BUY) == [(101, 1, 12)]
    tr = b.process(ts(MARKET, SELL), 0, 2, 15)
    assert trade_view(tr) == [(101, 1, 15, 12)]
    assert b.counters[CI["market_unfilled"]] == 1
    assert book_view(b, BUY) == [] and book_view(b, SELL) == []


def test_fifo_within_level_and_partial_cancel_keeps_priority():
    b = OracleBook(4)
    b.process(ts(LIMIT, SELL), 105, 5, 20)
    b.process(ts(LIMIT, SELL), 105, 5, 21)
    b.process(ts(PARTIAL_CANCEL, SELL), 105, 3, 20)
    assert book_view(b, SELL) == [(105, 2, 20), (105, 5, 21)]
    tr = b.process(ts(MARKET, BUY), 0, 3, 22)
    assert trade_view(tr) == [(105, 2, 22, 20), (105, 1, 22, 21)]
    assert book_view(b, SELL) == [(105, 4, 21)]


def test_sell_side_mirror_and_evict_on_ask_side():
    b = OracleBook(2)
    b.process(ts(LIMIT, SELL), 103, 1, 1)
    b.process(ts(LIMIT, SELL), 102, 1, 2)
    assert book_view(b, SELL) == [(102, 1, 2), (103, 1, 1)]
    b.process(ts(LIMIT, SELL), 101, 1, 3)  # better than worst 103 -> evict #1
    assert book_view(b, SELL) == [(101, 1, 3), (102, 1, 2)]
    b.process(ts(LIMIT, SELL), 104, 7, 4)  # worse -> dropped
    assert b.counters[CI["drop"]] == 1 and b.counters[CI["dropped_qty"]] == 7
    # a sell limit at 100 against no bids rests (side full -> evicts 102)
    b.process(ts(LIMIT, SELL), 100, 2, 5)
    assert book_view(b, SELL) == [(100, 2, 5), (101, 1, 3)]
    # a buy limit crossing at 101 takes 100 first, then 101, rests nothing
    tr = b.process(ts(LIMIT, BUY), 101, 3, 6)
    assert trade_view(tr) == [(100, 2, 6, 5), (101, 1, 6, 3)]
    assert book_view(b, SELL) == [] and book_view(b, BUY) == []


def test_replayed_executions_of_named_orders():
    """A replayed execution names a resting order by id on its own side: the trade is at
    that order's price against an anonymous aggressor of the other side, the rest of the
    order keeps its priority; a missing id is a miss, qty <= 0 is malformed."""
    b = OracleBook(4)
    for side, p, q, oid in [(BUY, 100, 5, 1), (BUY, 100, 3, 2), (BUY, 99, 4, 3), (SELL, 102, 2, 4)]:
        b.process(ts(LIMIT, side), p, q, oid, tid=7)
    # 2 of order #2 (second in the 100 queue): it keeps its place behind #1
    tr = b.process(ts(EXECUTE, BUY), 0, 2, 2, tid=9, seq=4, t=3)
    assert [list(map(int, x)) for x in tr] == [[100, 2, 0, 2, 0, 7, SELL | (4 << 1), 3]]
    assert book_view(b, BUY) == [(100, 5, 1), (100, 1, 2), (99, 4, 3)]
    # more than order #1 holds: only its 5, and it leaves the book
    tr = b.process(ts(EXECUTE, BUY), 0, 9, 1)
    assert trade_view(tr) == [(100, 5, 0, 1)]
    assert book_view(b, BUY) == [(100, 1, 2), (99, 4, 3)]
    # an ask executed whole: the aggressor is a buyer
    tr = b.process(ts(EXECUTE, SELL), 0, 2, 4, seq=6)
    assert [int(v) for v in tr[0]][:7] == [102, 2, 0, 4, 0, 7, BUY | (6 << 1)]
    assert book_view(b, SELL) == []
    # the id on the wrong side, an unknown id, and qty 0
    assert len(b.process(ts(EXECUTE, SELL), 0, 1, 3)) == 0
    assert len(b.process(ts(EXECUTE, BUY), 0, 1, 77)) == 0
    assert len(b.process(ts(EXECUTE, BUY), 0, 0, 3)) == 0
    assert b.counters[CI["miss"]] == 2 and b.counters[CI["bad"]] == 1
    assert b.counters[CI["trades"]] == 3
    # ignored messages (replayed hidden executions, cross trades, halts) change nothing
    assert len(b.process(ts(IGNORED, BUY), 100, 5, 1)) == 0
    assert len(b.process(ts(IGNORED, SELL), 0, 0, 0)) == 0
    assert b.counters[CI["ignored"]] == 2
    assert book_view(b, BUY) == [(100, 1, 2), (99, 4, 3)]
    assert b.counters[CI["msgs"]] == 4 + 8


def test_malformed_messages_are_counted_noops():
    b = OracleBook(3)
    b.process(ts(LIMIT, BUY), 100, 0, 1)
    b.process(ts(MARKET, SELL), 0, -1, 2)
    b.process(ts(PARTIAL_CANCEL, BUY), 100, 0, 1)
    b.process(ts(9, BUY), 100, 5, 3)
    assert b.counters[CI["bad"]] == 4
    assert b.counters[CI["msgs"]] == 4
    assert book_view(b, BUY) == []


# ----------------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------------
def check_invariants(b, cap):
    bids, asks = b.side(BUY), b.side(SELL)
    for s, lst in ((BUY, bids), (SELL, asks)):
        assert len(lst) <= cap
        assert all(o[1] > 0 for o in lst)
        prices = [int(o[0]) for o in lst]
        assert prices == sorted(prices, reverse=(s == BUY))
        oids = [int(o[2]) for o in lst]
        assert len(set(oids)) == len(oids)
    if len(bids) and len(asks):
        assert bids[0][0] < asks[0][0], "crossed book after matching"


def total_qty(b, s):
    return int(sum(int(o[1]) for o in b.side(s)))


def random_msg(rng, issued, pmax=6, qmax=6):
    typ = rng.choice([LIMIT, LIMIT, LIMIT, PARTIAL_CANCEL, DELETE, MARKET, EXECUTE, IGNORED])
    side = rng.randrange(2)
    if typ in (PARTIAL_CANCEL, DELETE, EXECUTE):
        if issued and rng.random() < 0.8:
            oid, side = rng.choice(issued)
        else:
            oid = rng.randrange(1, 50)
        return typ, side, rng.randrange(1, pmax + 1), rng.randrange(1, qmax + 1), oid
    return typ, side, rng.randrange(1, pmax + 1), rng.randrange(1, qmax + 1), None


@pytest.mark.parametrize("seed", range(6))
def test_invariants_and_conservation_random(seed):
    rng = random.Random(seed)
    cap = rng.choice([1, 2, 3, 5, 8])
    b = OracleBook(cap)
    issued = []
    next_oid = 1
    for k in range(400):
        typ, side, p, q, oid = random_msg(rng, issued)
        if oid is None:
            oid = next_oid
            next_oid += 1
            if typ == LIMIT:
                issued.append((oid, side))
        before = {s: total_qty(b, s) for s in (BUY, SELL)}
        c0 = b.counters.copy()
        tr = b.process(ts(typ, side), p, q, oid, seq=k)
        check_invariants(b, cap)
        traded = int(sum(int(t[1]) for t in tr))
        dc = b.counters - c0
        after = {s: total_qty(b, s) for s in (BUY, SELL)}
        if typ in (LIMIT, MARKET):
            # the opposite side loses exactly the traded volume; trades never exceed q
            assert before[1 - side] - after[1 - side] == traded
            assert traded <= q
            if typ == LIMIT:
                rested = q - traded - int(dc[CI["dropped_qty"]])
                assert after[side] - before[side] == rested - int(dc[CI["evicted_qty"]])
            else:
                assert int(dc[CI["market_unfilled"]]) == q - traded
                assert after[side] == before[side]
            # every trade is at a price no worse than the limit
            for t in tr:
                if typ == LIMIT:
                    assert (t[0] <= p) if side == BUY else (t[0] >= p)
        elif typ == EXECUTE:
            # the named side loses exactly the executed volume, at most q, in one trade
            assert len(tr) <= 1 and traded <= q
            assert before[side] - after[side] == traded
            assert after[1 - side] == before[1 - side]
        elif typ == IGNORED:
            assert traded == 0 and after == before
        else:
            assert traded == 0
            assert after[1 - side] == before[1 - side]
            assert before[side] - after[side] <= (q if typ == PARTIAL_CANCEL else before[side])


# ----------------------------------------------------------------------------------
# brute force against the naive book
# ----------------------------------------------------------------------------------
def run_both(cap, msgs):
    b, nb = OracleBook(cap), NaiveBook(cap)
    for k, (typ, side, p, q, oid) in enumerate(msgs):
        t1 = b.process(ts(typ, side), p, q, oid, seq=k)
        t2 = nb.process(ts(typ, side), p, q, oid, seq=k)
        assert [list(map(int, t)) for t in t1] == t2, (cap, msgs, k)
    for s in (BUY, SELL):
        assert [list(map(int, o)) for o in b.side(s)] == nb.side(s), (cap, msgs)
    assert list(map(int, b.counters)) == nb.counters, (cap, msgs)


def test_brute_force_exhaustive_tiny_alphabet():
    alphabet = []
    for side in (BUY, SELL):
        for p in (1, 2, 3):
            for q in (1, 2):
                alphabet.append((LIMIT, side, p, q, None))
        alphabet.append((MARKET, side, 0, 2, None))
        for oid in (1, 2):
            alphabet.append((PARTIAL_CANCEL, side, 0, 1, oid))
            alphabet.append((DELETE, side, 0, 0, oid))
            alphabet.append((EXECUTE, side, 0, 1, oid))
        alphabet.append((IGNORED, side, 0, 0, 0))
    n = 0
    for cap in (1, 2):
        for seq in itertools.product(alphabet, repeat=3):
            msgs = []
            for j, (typ, side, p, q, oid) in enumerate(seq):
                msgs.append((typ, side, p, q, oid if oid is not None else j + 1))
            run_both(cap, msgs)
            n += 1
    assert n == 2 * len(alphabet) ** 3


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_random_sequences(seed):
    rng = random.Random(1000 + seed)
    for _ in range(150):
        cap = rng.choice([1, 2, 3, 4, 7])
        n = rng.randrange(20, 200)
        issued, msgs = [], []
        for k in range(n):
            typ, side, p, q, oid = random_msg(rng, issued, pmax=rng.choice([3, 6, 12]))
            if oid is None:
                oid = 1000 + k
                if typ == LIMIT:
                    issued.append((oid, side))
            msgs.append((typ, side, p, q, oid))
        run_both(cap, msgs)


# ----------------------------------------------------------------------------------
# special cases that reduce to textbook routines
# ----------------------------------------------------------------------------------
def test_non_crossing_inserts_equal_a_stable_sort():
    rng = random.Random(7)
    b = OracleBook(64)
    orders = []
    for k in range(60):
        p = rng.randrange(90, 100)
        q = rng.randrange(1, 9)
        b.process(ts(LIMIT, BUY), p, q, k + 1)
        orders.append((p, q, k + 1))
    expect = sorted(orders, key=lambda o: -o[0])  # Python's sort is stable
    assert book_view(b, BUY) == expect


def test_single_level_market_orders_consume_a_fifo_queue():
    rng = random.Random(8)
    b = OracleBook(50)
    queue = []
    for k in range(40):
        q = rng.randrange(1, 20)
        b.process(ts(LIMIT, SELL), 100, q, k + 1)
        queue.append([k + 1, q])
    for k in range(30):
        want = rng.randrange(1, 30)
        tr = b.process(ts(MARKET, BUY), 0, want, 500 + k)
        expect = []
        left = want
        while left > 0 and queue:
            x = min(left, queue[0][1])
            expect.append((100, x, 500 + k, queue[0][0]))
            queue[0][1] -= x
            left -= x
            if queue[0][1] == 0:
                queue.pop(0)
        assert trade_view(tr) == expect
    assert book_view(b, SELL) == [(100, q, oid) for oid, q in queue]


def test_cancels_only_is_set_deletion():
    b = OracleBook(100)
    rng = random.Random(9)
    live = {}
    for k in range(80):
        p = rng.randrange(100, 120)
        b.process(ts(LIMIT, SELL), p, 5, k + 1)
        live[k + 1] = p
    for oid in rng.sample(sorted(live), 50):
        b.process(ts(DELETE, SELL), 0, 0, oid)
        del live[oid]
    got = {o[2]: o[0] for o in book_view(b, SELL)}
    assert got == live

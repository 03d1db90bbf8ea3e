"""A deliberately naive price-time-priority book for brute-force checks of the oracle.

Each side is one flat Python list that is fully re-sorted (stable sort on price) after
every insertion, so time priority among equal prices is Python's sort stability and
nothing else.  It shares no code with the oracle and is only used on tiny inputs.
"""
from __future__ import annotations

LIMIT, PARTIAL_CANCEL, DELETE, MARKET, EXECUTE, IGNORED = 1, 2, 3, 4, 5, 6
BUY, SELL = 0, 1

# counters (same meaning and order as the oracle's)
MSGS, TRADES, MISS, EVICT, EVICTED_QTY, DROP, DROPPED_QTY, MARKET_UNFILLED, BAD, OVERFLOW, IGNORED_CT = range(11)


class NaiveBook:
    def __init__(self, cap: int):
        self.cap = cap
        self.sides = {BUY: [], SELL: []}  # entries: [price, qty, oid, tid, tsec, tns]
        self.counters = [0] * 11

    def _sort(self, s):
        # bids: highest price first; asks: lowest first; stable => arrival order kept
        self.sides[s].sort(key=(lambda o: -o[0]) if s == BUY else (lambda o: o[0]))

    def load(self, s, orders):
        self.sides[s] = [list(o) for o in orders]

    def process(self, ts, price, qty, oid, tid=0, tsec=0, tns=0, seq=0, t=0):
        typ, side = ts & 0xFF, (ts >> 8) & 1
        c = self.counters
        c[MSGS] += 1
        trades = []
        if typ in (LIMIT, MARKET):
            if qty <= 0:
                c[BAD] += 1
                return trades
            opp = self.sides[1 - side]
            q = qty
            while q > 0 and opp:
                best = opp[0]
                if typ == LIMIT and not (best[0] <= price if side == BUY else best[0] >= price):
                    break
                x = min(q, best[1])
                trades.append([best[0], x, oid, best[2], tid, best[3], side | (seq << 1), t])
                c[TRADES] += 1
                best[1] -= x
                q -= x
                if best[1] == 0:
                    opp.pop(0)
            if typ == MARKET:
                c[MARKET_UNFILLED] += q
                return trades
            if q > 0:
                own = self.sides[side]
                if len(own) >= self.cap:
                    worst = own[-1]
                    if (price > worst[0]) if side == BUY else (price < worst[0]):
                        c[EVICT] += 1
                        c[EVICTED_QTY] += worst[1]
                        own.pop()
                    else:
                        c[DROP] += 1
                        c[DROPPED_QTY] += q
                        return trades
                own.append([price, q, oid, tid, tsec, tns])
                self._sort(side)
            return trades
        if typ in (PARTIAL_CANCEL, DELETE):
            if typ == PARTIAL_CANCEL and qty <= 0:
                c[BAD] += 1
                return trades
            lst = self.sides[side]
            for j, o in enumerate(lst):
                if o[2] == oid:
                    if typ == DELETE:
                        lst.pop(j)
                    else:
                        o[1] -= min(qty, o[1])
                        if o[1] == 0:
                            lst.pop(j)
                    return trades
            c[MISS] += 1
            return trades
        if typ == EXECUTE:
            # a replayed execution of the named resting order on `side`: the trade is at
            # that order's price, the aggressor (id 0, trader 0) is on the other side
            if qty <= 0:
                c[BAD] += 1
                return trades
            lst = self.sides[side]
            for j, o in enumerate(lst):
                if o[2] == oid:
                    x = min(qty, o[1])
                    trades.append([o[0], x, 0, o[2], 0, o[3], (1 - side) | (seq << 1), t])
                    c[TRADES] += 1
                    o[1] -= x
                    if o[1] == 0:
                        lst.pop(j)
                    return trades
            c[MISS] += 1
            return trades
        if typ == IGNORED:
            c[IGNORED_CT] += 1
            return trades
        c[BAD] += 1
        return trades

    def side(self, s):
        return [list(o) for o in self.sides[s]]

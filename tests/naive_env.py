"""A naive, pure-Python environment step used to brute-force check the oracle on tiny inputs.

Written from the same readings of the paper's five-stage step (Sec. 4) as the oracle,
but coded independently on top of tests/naive_book.py.  Slow; only for a handful of
envs and steps.
"""
from __future__ import annotations

from naive_book import NaiveBook, LIMIT, PARTIAL_CANCEL, DELETE, MARKET, BUY, SELL

M64 = (1 << 64) - 1
DOM_SHUFFLE = 0x5348554646
DOM_ACTION = 0x414354
EXEC, MM, DIR, MM_BUYSELL, MM_SPREADSKEW, MM_AVST, EXEC_TWAP, MM_AS = 0, 1, 2, 3, 4, 5, 6, 7
EXEC_KINDS = (EXEC, EXEC_TWAP)
SPOONER_KINDS = (MM, MM_SPREADSKEW, MM_AVST, MM_AS)


def n_actions(kind):
    if kind == DIR:
        return 3
    if kind in (EXEC_TWAP, MM_AS):
        return 1
    return 9


def sm64(z):
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def hash_chain(seed, dom, a, b, c):
    h = sm64(seed ^ dom)
    for w in (a, b, c):
        h = sm64(h ^ w)
    return h


def f32(x):
    import numpy as np
    return np.float32(x)


class NaiveEnv:
    def __init__(self, e, cap, kinds, episode_len, seed, exec_task=500, q0=4, mm_q=10, dir_q=10,
                 pen=0.01, lam=0.0, rho=0.0, avst_gamma=0.01, avst_sigma2=10.0, avst_kappa=0.5):
        import numpy as np
        self.e, self.cap, self.kinds, self.T, self.seed = e, cap, list(kinds), episode_len, seed
        self.exec_task, self.q0, self.mm_q, self.dir_q = exec_task, q0, mm_q, dir_q
        # float parameters are given in single precision, used in double
        self.pen, self.lam, self.rho = (float(np.float32(v)) for v in (pen, lam, rho))
        self.gamma0, self.sigma2, self.kappa = (float(np.float32(v)) for v in (avst_gamma, avst_sigma2, avst_kappa))

    def reset(self, bids, asks):
        self.book = NaiveBook(self.cap)
        self.book.load(BUY, bids[: self.cap])
        self.book.load(SELL, asks[: self.cap])
        bl, al = self.book.side(BUY), self.book.side(SELL)
        self.bb = bl[0][0] if bl else (al[0][0] - 1 if al else 0)
        self.ba = al[0][0] if al else (bl[0][0] + 1 if bl else 0)
        self.pinit2 = self.bb + self.ba
        self.mid2_prev = self.pinit2
        self.dmid2 = 0
        times = [(o[4], o[5]) for o in bl + al]
        self.time = max(times) if times else (0, 0)
        self.t = 0
        A = len(self.kinds)
        self.inv = [0] * A
        self.cash = [0] * A
        self.rem = [self.exec_task if k in EXEC_KINDS else 0 for k in self.kinds]
        self.ctr = [0] * A
        self.step_bq = [0] * A
        self.step_sq = [0] * A
        self.stats = (0, 0, 0, 0)  # buy vol, sell vol, trades, last price

    def _desires(self, i, a, bb, ba):
        """[(side, price, qty)], market [(side, qty)] for agent i's action a."""
        k = self.kinds[i]
        lim, mkt = [], []
        if k == EXEC:
            q0 = self.q0
            plan = {1: [("m", q0)], 2: [(bb, q0)], 3: [(-((-(bb + ba)) // 2), q0)], 4: [(ba, q0)],
                    5: [(ba + 2, q0)], 6: [(ba, 2 * q0)], 7: [(ba, 5 * q0)],
                    8: [(ba, q0), (ba + 1, q0), (ba + 2, q0), (ba + 3, q0)]}.get(a, [])
            left = self.rem[i]
            for p, q in plan:
                q = min(q, left)
                left -= q
                if q > 0:
                    if p == "m":
                        mkt.append((SELL, q))
                    else:
                        lim.append((SELL, p, q))
        elif k == MM_SPREADSKEW:
            # a table of (spread, skew): spread 1, 3 or 5 ticks around the mid, skew -1, 0, +1
            spread, skew = (1, 3, 5)[a // 3], a % 3 - 1
            m2 = bb + ba
            bid = (m2 - spread) // 2 + skew
            ask = -((-(m2 + spread)) // 2) + skew
            lim.append((BUY, min(bid, ba - 1), self.mm_q))
            lim.append((SELL, max(ask, bb + 1), self.mm_q))
        elif k in (MM_AVST, MM_AS):
            import math
            g = self.gamma0 * 2.0 ** ((a if k == MM_AVST else 4) - 4)
            A_ = g * self.sigma2
            B_ = (2.0 / g) * math.log(1.0 + g / self.kappa)
            q = self.inv[i] / self.mm_q
            tau = float(self.T - self.t)
            r = float(bb + ba) * 0.5 - q * A_ * tau
            d = A_ * tau + B_
            lo, hi = -float(1 << 30), float(1 << 30)
            bid = int(min(max(math.floor(r - d * 0.5), lo), hi))
            ask = int(min(max(math.ceil(r + d * 0.5), lo), hi))
            lim.append((BUY, min(bid, ba - 1), self.mm_q))
            lim.append((SELL, max(ask, bb + 1), self.mm_q))
        elif k == EXEC_TWAP:
            target = (self.exec_task * (self.t + 1) + self.T - 1) // self.T
            q = min(max(target - (self.exec_task - self.rem[i]), 0), self.rem[i])
            if q > 0:
                lim.append((SELL, bb, q))
        elif k in (MM, MM_BUYSELL):
            offs = {1: [(BUY, 2), (SELL, 2)], 2: [(BUY, 4), (SELL, 4)], 3: [(BUY, -1), (SELL, -1)],
                    4: [(BUY, 2)], 5: [(SELL, 2)], 6: [(BUY, 5), (SELL, -1)], 7: [(BUY, -1), (SELL, 5)],
                    8: [(BUY, 0), (BUY, 1), (BUY, 2), (BUY, 3), (SELL, 0), (SELL, 1), (SELL, 2), (SELL, 3)]}
            for s, o in offs.get(a, []):
                p = min(bb - o, ba - 1) if s == BUY else max(ba + o, bb + 1)
                lim.append((s, p, self.mm_q))
        else:
            if a == 1:
                lim.append((BUY, ba, self.dir_q))
            elif a == 2:
                lim.append((SELL, bb, self.dir_q))
        return lim, mkt

    def step(self, replay, actions=None):
        """replay: list of 7-int messages; actions: list per agent or None.  Returns dict."""
        A = len(self.kinds)
        bl, al = self.book.side(BUY), self.book.side(SELL)
        bb = bl[0][0] if bl else self.bb
        ba = al[0][0] if al else self.ba
        tsec, tns = self.time
        cancel_msgs, new_msgs, used = [], [], []
        for i in range(A):
            n_act = n_actions(self.kinds[i])
            if actions is None:
                u = hash_chain(self.seed, DOM_ACTION, self.e, self.t, i) >> 32
                a = (u * n_act) >> 32
            else:
                a = int(actions[i])
            used.append(a)
            if not (0 <= a < n_act):
                a = 0
            lim, mkt = self._desires(i, a, bb, ba)
            want = {}
            order = []
            for s, p, q in lim:
                if (s, p) not in want:
                    want[(s, p)] = 0
                    order.append((s, p))
                want[(s, p)] += q
            tid = i + 1
            mine = [(s, o) for s in (BUY, SELL) for o in self.book.side(s) if o[3] == tid]
            rest = {}
            for s, o in mine:
                rest[(s, o[0])] = rest.get((s, o[0]), 0) + o[1]
            # cancel amounts: excess removed from the newest orders of each level
            amount = {}
            for lvl, r in rest.items():
                d = want.get(lvl, 0)
                if d == 0 or r <= d:
                    continue
                need = r - d
                for s, o in reversed(mine):
                    if (s, o[0]) == lvl and need > 0:
                        x = min(need, o[1])
                        amount[(s, o[2])] = x
                        need -= x
            for s, o in mine:
                d = want.get((s, o[0]), 0)
                if d == 0:
                    cancel_msgs.append([DELETE | (s << 8), o[0], o[1], o[2], tid, tsec, tns])
                elif (s, o[2]) in amount:
                    cancel_msgs.append([PARTIAL_CANCEL | (s << 8), o[0], amount[(s, o[2])], o[2], tid, tsec, tns])
            def new(typ, s, p, q):
                oid = (1 << 30) | (i << 26) | (self.ctr[i] % (1 << 26))
                self.ctr[i] += 1
                new_msgs.append([typ | (s << 8), p, q, oid, tid, tsec, tns])
            for lvl in order:
                r = rest.get(lvl, 0)
                if want[lvl] > r:
                    new(LIMIT, lvl[0], lvl[1], want[lvl] - r)
            for s, q in mkt:
                new(MARKET, s, 0, q)
        keyed = sorted(range(len(new_msgs)),
                       key=lambda k: ((hash_chain(self.seed, DOM_SHUFFLE, self.e, self.t, k) >> 32), k))
        seq = cancel_msgs + [new_msgs[k] for k in keyed] + [list(m) for m in replay]
        trades = []
        S = n = 0
        for k, m in enumerate(seq):
            trades += self.book.process(*m, seq=k, t=self.t)
            self.time = (m[5], m[6])
            bl, al = self.book.side(BUY), self.book.side(SELL)
            if bl and al:
                S += bl[0][0] + al[0][0]
                n += 1
        bq, bn, sq, sn = [0] * A, [0] * A, [0] * A, [0] * A
        bvol = svol = 0
        lastp = 0
        for tr in trades:
            p, q, agg_tid, pas_tid, side = tr[0], tr[1], tr[4], tr[5], tr[6] & 1
            if side == BUY:
                bvol += q
            else:
                svol += q
            lastp = p
            for i in range(A):
                if agg_tid == i + 1:
                    if side == BUY:
                        bq[i] += q; bn[i] += p * q
                    else:
                        sq[i] += q; sn[i] += p * q
                if pas_tid == i + 1:
                    if side == BUY:
                        sq[i] += q; sn[i] += p * q
                    else:
                        bq[i] += q; bn[i] += p * q
        bl, al = self.book.side(BUY), self.book.side(SELL)
        bb1 = bl[0][0] if bl else self.bb
        ba1 = al[0][0] if al else self.ba
        mid2 = bb1 + ba1
        last = self.t + 1 == self.T
        rewards = []
        for i in range(A):
            self.inv[i] += bq[i] - sq[i]
            self.cash[i] += sn[i] - bn[i]
            if self.kinds[i] in EXEC_KINDS:
                self.rem[i] -= sq[i]
            mbar = S / (2.0 * n) if n > 0 else self.mid2_prev * 0.5
            psi_b = mbar * bq[i] - bn[i]
            psi_s = sn[i] - mbar * sq[i]
            if self.kinds[i] in SPOONER_KINDS:
                psi_inv = self.inv[i] * (mid2 * 0.5 - self.mid2_prev * 0.5)
                r = psi_b + psi_s + psi_inv - (1.0 - self.lam) * (psi_inv if psi_inv > 0.0 else 0.0) \
                    - self.rho * (float(self.inv[i]) * float(self.inv[i]))
            elif self.kinds[i] == MM_BUYSELL:
                r = psi_b + psi_s - self.rho * (float(self.inv[i]) * float(self.inv[i]))
            elif self.kinds[i] == DIR:
                r = psi_b + psi_s
            else:
                pinit = self.pinit2 * 0.5
                r = sn[i] - pinit * sq[i]
                if last:
                    r = r - (self.pen * self.rem[i]) * pinit
            rewards.append(f32(r))
        self.step_bq, self.step_sq = bq, sq
        self.stats = (bvol, svol, len(trades), lastp)
        self.dmid2 = mid2 - self.mid2_prev
        self.bb, self.ba = bb1, ba1
        self.mid2_prev = mid2
        self.t += 1
        fills = [[bq[i], bn[i], sq[i], sn[i]] for i in range(A)]
        return {"trades": trades, "fills": fills, "reward": rewards, "done": int(last),
                "obs": [self.observe(i) for i in range(A)], "actions": used}

    def observe(self, i):
        f = [0] * 40
        bb, ba = self.bb, self.ba
        mid2 = bb + ba
        f[0] = ba - bb
        f[1] = self.dmid2
        f[2] = mid2 - self.pinit2
        tid = i + 1
        for s in (BUY, SELL):
            for o in self.book.side(s):
                d = bb - o[0] if s == BUY else o[0] - ba
                if 0 <= d <= 9:
                    f[(3 if s == BUY else 13) + d] += o[1]
                f[23 + s] += o[1]
                f[25 + s] += 1
                if o[3] == tid:
                    f[35 + s] += o[1]
                    f[37] += 1
        bvol, svol, ntr, lastp = self.stats
        f[27], f[28], f[29] = bvol, svol, ntr
        f[30] = 2 * lastp - mid2 if ntr > 0 else 0
        f[31], f[32] = self.inv[i], self.cash[i]
        f[33] = self.rem[i] if self.kinds[i] in EXEC_KINDS else 0
        f[34] = self.T - self.t
        f[38], f[39] = self.step_bq[i], self.step_sq[i]
        return [f32(v) for v in f]

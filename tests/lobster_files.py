"""A synthetic LOBSTER-format trading day for the ingestion tests: generated messages
(limit orders, cancels, executions, ignored messages; no market orders, which LOBSTER
does not have) written as a message file, and its order-book file computed by replaying
them through the oracle's single book (levels aggregated per price)."""
import os

import numpy as np

from oracle import OracleBook
from paper_2511_02136_amd import lobster, synth

LEVELS = 10


def synthetic_day(tmpdir, n=3000, seed=51):
    w = synth.Workload("day", n_envs=1, n_steps=n // 100, msgs_per_step=100, cap=400, seed=seed,
                       exec_pct=10, ignored_pct=4, snapshot_fill_pct=0)
    s = synth.generate(w, threads=1)
    t = s.ts & 0xFF
    keep = (t != 4) & (s.oid < lobster.SNAPSHOT_ID_BASE)
    m = lobster.Messages(*[np.ascontiguousarray(a[keep]) for a in s.msg_fields()])
    msg_path = os.path.join(tmpdir, "day_message_10.csv")
    book_path = os.path.join(tmpdir, "day_orderbook_10.csv")
    lobster.write_messages(msg_path, m)
    b = OracleBook(1000)
    rows = []
    for i in range(len(m)):
        b.process(int(m.ts[i]), int(m.price[i]), int(m.qty[i]), int(m.oid[i]), 0, int(m.tsec[i]), int(m.tns[i]), seq=i)
        levels = []
        for side in (0, 1):
            agg = {}
            for o in b.side(side):
                agg[int(o[0])] = agg.get(int(o[0]), 0) + int(o[1])
            ps = sorted(agg, reverse=(side == 0))[:LEVELS]
            levels.append([(p, agg[p]) for p in ps])
        rows.append((levels[0], levels[1]))
    lobster.write_orderbook(book_path, rows, LEVELS)
    return m, msg_path, book_path, rows

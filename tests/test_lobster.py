"""LOBSTER-format ingestion (host side): parsing, type and side mapping, exact times,
id renumbering, order-book rows, env windows and reset books."""
import os

import numpy as np
import pytest

from lobster_files import synthetic_day
from paper_2511_02136_amd import lobster


def test_parse_hand_written_rows(tmp_path):
    p = tmp_path / "m.csv"
    p.write_text("34200.004241176,1,16113575,18,5853300,1\n"
                 "34200.5,3,16113575,18,5853300,1\n"
                 "34201,4,2147483700,5,5853400,-1\n"
                 "34201.000000001,7,-1,0,-1,-1\n"
                 "34202.25,5,0,7,5853500,1\n"
                 "34202.250000000,2,9,3,5853200,-1\n")
    m = lobster.read_messages(str(p))
    assert (m.ts & 0xFF).tolist() == [1, 3, 5, 6, 6, 2]
    assert (m.ts >> 8).tolist() == [0, 0, 1, 1, 0, 1]
    assert m.price.tolist()[:3] == [58533, 58533, 58534]
    assert m.tsec.tolist() == [34200, 34200, 34201, 34201, 34202, 34202]
    assert m.tns.tolist() == [4241176, 500000000, 0, 1, 250000000, 250000000]
    # ids outside the replay range get fresh ids below the reserved block, consistently
    assert m.oid[0] == m.oid[1] == 16113575 and m.oid[4] == 0 and m.oid[5] == 9
    assert m.oid[2] != m.oid[3]
    assert all(0 <= x < lobster.SNAPSHOT_ID_BASE for x in m.oid.tolist())
    assert m.oid[2] not in (16113575, 0, 9) and m.oid[3] not in (16113575, 0, 9)


def test_rejects_unknown_types_and_directions(tmp_path):
    p = tmp_path / "m.csv"
    p.write_text("34200.1,8,1,1,100,1\n")
    with pytest.raises(ValueError):
        lobster.read_messages(str(p))
    p.write_text("34200.1,1,1,1,100,0\n")
    with pytest.raises(ValueError):
        lobster.read_messages(str(p))


def test_message_file_round_trip(tmp_path):
    m, msg_path, _, _ = synthetic_day(str(tmp_path), n=1500)
    back = lobster.read_messages(msg_path)
    for f in ("ts", "price", "qty", "oid", "tsec", "tns"):
        assert np.array_equal(getattr(back, f), getattr(m, f)), f
    kinds = set((m.ts & 0xFF).tolist())
    assert kinds == {1, 2, 3, 5, 6}


def test_orderbook_rows_and_reset_books(tmp_path):
    m, _, book_path, rows = synthetic_day(str(tmp_path), n=1500)
    for r in (0, 17, 700, len(rows) - 1):
        assert lobster.read_orderbook_row(book_path, r) == (rows[r][0], rows[r][1])
    starts = [0, 300, 800]
    books = lobster.books_before(book_path, starts)
    assert books[0] == ([], [])
    assert books[1] == (rows[299][0], rows[299][1])
    s = lobster.build_stream(m, starts, n_steps=5, msgs_per_step=100, cap=12, books=books)
    assert s.off.tolist()[1] == [500, 600, 700, 800, 900, 1000]
    assert np.array_equal(s.price[500:1000], m.price[300:800])
    for e, (bids, asks) in enumerate(books):
        for side, lv in ((0, bids), (1, asks)):
            n = min(len(lv), 12)
            assert s.book["n"][e, side] == n
            assert s.book["price"][e, side, :n].tolist() == [p for p, _ in lv[:n]]
            assert s.book["qty"][e, side, :n].tolist() == [q for _, q in lv[:n]]
            assert (s.book["tsec"][e, side, :n] == m.tsec[starts[e]]).all()
            assert len(set(s.book["oid"][e, side, :n].tolist())) == n
    with pytest.raises(ValueError):
        lobster.build_stream(m, [len(m) - 10], n_steps=1, msgs_per_step=100, cap=12, books=[([], [])])

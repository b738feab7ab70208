"""Host logic of the serving loop (no GPU): first-come first-served admission
by memory budget and slots."""
import collections

import pytest

from paper_2602_00290_amd.serve import Admission, Request


def _q(specs):
    return collections.deque(Request(rid=i, prob=None, arrival=a, steps=1, nbytes=b) for i, (a, b) in enumerate(specs))


def test_admits_only_arrived_requests():
    adm = Admission(100, 10)
    q = _q([(0.0, 10), (1.0, 10)])
    got = adm.take(q, now=0.5)
    assert [r.rid for r in got] == [0] and len(q) == 1
    got = adm.take(q, now=1.0)
    assert [r.rid for r in got] == [1]


def test_memory_budget_and_fifo_order():
    adm = Admission(100, 10)
    q = _q([(0.0, 60), (0.0, 50), (0.0, 10)])
    got = adm.take(q, now=0.0)
    # the 50-byte head does not fit after 60; the 10-byte request behind it must not overtake it
    assert [r.rid for r in got] == [0]
    assert adm.in_use == 60
    adm.release(got[0])
    got = adm.take(q, now=0.0)
    assert [r.rid for r in got] == [1, 2] and adm.in_use == 60


def test_slot_limit():
    adm = Admission(1000, 2)
    q = _q([(0.0, 1)] * 5)
    assert len(adm.take(q, 0.0)) == 2
    assert adm.take(q, 0.0) == []
    adm.release(Request(0, None, 0.0, 1, 1))
    assert len(adm.take(q, 0.0)) == 1


def test_oversized_request_rejected():
    adm = Admission(100, 4)
    with pytest.raises(ValueError):
        adm.check(Request(0, None, 0.0, 1, 101))
    with pytest.raises(ValueError):
        Admission(0, 1)

"""Admission policy of the serving loop (host only, no device calls)."""
import heapq

import numpy as np
import pytest

from paper_2510_21105_amd.serve import Admission


def test_arrival_order_without_overtaking():
    a = Admission(budget=100, slots=2)
    a.arrive("a", 60)
    a.arrive("b", 50)
    a.arrive("c", 10)
    assert a.admit() == ["a"]          # b does not fit and c may not overtake it
    assert a.admit() == []
    a.finish("a")
    assert a.admit() == ["b", "c"]
    assert a.used == 60 and len(a.running) == 2
    a.finish("b")
    a.finish("c")
    assert a.idle() and a.used == 0


def test_slots_limit_concurrency():
    a = Admission(budget=10 ** 9, slots=2)
    for r in range(5):
        a.arrive(r, 1)
    assert a.admit() == [0, 1]
    a.finish(1)
    assert a.admit() == [2]


def test_requests_larger_than_the_budget_are_refused():
    a = Admission(budget=100, slots=4)
    with pytest.raises(ValueError, match="more than the budget"):
        a.arrive("big", 101)
    a.arrive("ok", 100)
    assert a.admit() == ["ok"]
    with pytest.raises(ValueError):
        Admission(budget=0, slots=1)


def test_cancel_only_waiting_requests():
    a = Admission(budget=100, slots=1)
    a.arrive(1, 10)
    a.arrive(2, 10)
    a.arrive(3, 10)
    assert a.admit() == [1]
    assert a.cancel(2) is True
    assert a.cancel(1) is False        # already running
    assert a.cancel(9) is False        # unknown
    a.finish(1)
    assert a.admit() == [3]


def test_simulated_trace_keeps_budget_slots_and_order():
    """Event simulation with random sizes and durations: never over budget or
    slots, admissions in arrival order, every request served once."""
    rng = np.random.default_rng(5)
    budget, slots = 1000, 4
    a = Admission(budget, slots)
    n = 300
    arrivals = np.cumsum(rng.exponential(1.0, n))
    sizes = rng.integers(1, budget + 1, n)
    durs = rng.exponential(3.0, n)
    events, t, nxt, order, done = [], 0.0, 0, [], set()
    while nxt < n or not a.idle():
        t_arr = arrivals[nxt] if nxt < n else np.inf
        t_fin = events[0][0] if events else np.inf
        if t_arr <= t_fin:
            t = t_arr
            a.arrive(nxt, int(sizes[nxt]))
            nxt += 1
        else:
            t, rid = heapq.heappop(events)
            a.finish(rid)
            done.add(rid)
        for rid in a.admit():
            order.append(rid)
            heapq.heappush(events, (t + durs[rid], rid))
        assert a.used <= budget and len(a.running) <= slots
    assert order == list(range(n)) and done == set(range(n))

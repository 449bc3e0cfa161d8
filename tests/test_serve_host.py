"""Host-side logic of the serving loop: admission budget and batch splitting."""
import threading
import time

import pytest

from paper_1804_01698_amd.serve import MemoryGate, split_to_budget


def test_split_to_budget_groups_in_order():
    sizes = [4, 4, 4, 10, 1, 1, 30, 2]
    g = split_to_budget(sizes, budget=12, fixed=2)
    assert [i for grp in g for i in grp] == list(range(len(sizes)))      # order kept, nothing lost
    for grp in g:
        if len(grp) > 1:
            assert 2 + sum(sizes[i] for i in grp) <= 12
    assert [6] in g                                                       # oversize item alone
    assert split_to_budget([], 10) == []


def test_split_to_budget_greedy_maximal():
    sizes = [3, 3, 3, 3]
    assert split_to_budget(sizes, 9) == [[0, 1, 2], [3]]
    assert split_to_budget(sizes, 6, fixed=1) == [[0], [1], [2], [3]]


def test_memory_gate_blocks_until_release():
    g = MemoryGate(100)
    g.acquire(70)
    got = []

    def worker():
        g.acquire(50)
        got.append(time.perf_counter())
        g.release(50)

    t = threading.Thread(target=worker)
    t0 = time.perf_counter()
    t.start()
    time.sleep(0.2)
    assert not got                      # 70 + 50 > 100: still waiting
    g.release(70)
    t.join(5)
    assert got and got[0] - t0 >= 0.2
    assert g.used == 0 and g.peak == 70 and g.waits == 1


def test_memory_gate_rejects_oversize():
    g = MemoryGate(10)
    with pytest.raises(MemoryError):
        g.acquire(11)
    assert g.fits(10) and not g.fits(11)


def test_memory_gate_try_acquire_never_waits():
    g = MemoryGate(100)
    assert g.try_acquire(60)
    assert not g.try_acquire(50)           # would exceed: refused at once
    assert g.used == 60 and g.waits == 0
    assert g.try_acquire(40) and g.used == 100 and g.peak == 100
    g.release(100)
    assert g.used == 0

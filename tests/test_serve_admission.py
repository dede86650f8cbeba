"""Admission by device bytes (the serving loop's accounting, host logic only): the
running rollouts never hold more than the budget, requests are admitted first in,
first out, and a request larger than the whole budget is refused."""
import numpy as np

from paper_2609_27342_amd.serve import Admission


def test_admission_never_exceeds_budget_and_refuses_oversized():
    rng = np.random.default_rng(0)
    budget = 1000
    adm = Admission(budget)
    sizes = [int(s) for s in rng.integers(50, 700, size=300)] + [1500, 1001]
    rng.shuffle(sizes)
    queue = list(enumerate(sizes))
    running = []
    admitted_order, refused = [], []
    while queue or running:
        # admit first in, first out while the head fits; refuse what never fits
        while queue:
            i, nb = queue[0]
            if adm.refuses(nb):
                refused.append(i)
                queue.pop(0)
                continue
            if not adm.fits(nb):
                break
            queue.pop(0)
            adm.take(nb)
            running.append((i, nb))
            admitted_order.append(i)
            assert adm.used <= budget
        # a random subset of the running rollouts finishes
        keep = []
        for i, nb in running:
            if rng.uniform() < 0.3:
                adm.release(nb)
            else:
                keep.append((i, nb))
        running = keep
        assert 0 <= adm.used <= budget
    assert sorted(refused) == sorted(i for i, s in enumerate(sizes) if s > budget)
    assert admitted_order == sorted(admitted_order)  # FIFO
    assert len(admitted_order) + len(refused) == len(sizes)
    assert adm.used == 0


def test_take_beyond_budget_raises():
    adm = Admission(100)
    adm.take(60)
    try:
        adm.take(41)
    except ValueError:
        return
    raise AssertionError("admission beyond the budget was accepted")

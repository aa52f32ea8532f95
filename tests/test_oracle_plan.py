"""The oracle's plan runner with an item limit (the stop-and-resume
mechanism a long experimental plan uses, paper section 1): a run stopped
after k items has run exactly the k longest, and resuming from its done
flags gives the uninterrupted plan's outputs bit for bit, wherever it
stopped and however often."""
import numpy as np

from oracle import plan as oplan
from paper_1501_01405_amd import inputs


def _items():
    # 40 items with repeated run lengths (ties keep index order)
    t = inputs.plan_table(n_dp=8, reps=5, n_lo=200, n_hi=3000, seed=3)
    t["customers"][[3, 7, 11]] = 1500
    return [(int(r["dp"]), int(r["rep"]), int(r["customers"]), float(r["lambda_"]),
             float(r["mu"])) for r in t]


def test_longest_first_is_stable():
    assert oplan.longest_first([5, 9, 5, 9, 1]) == [1, 3, 0, 2, 4]


def test_limit_runs_the_longest_items_first():
    items = _items()
    out, done = oplan.plan_run(11, items, max_items=7)
    order = oplan.longest_first([it[2] for it in items])
    assert set(np.flatnonzero(done)) == set(order[:7])
    assert np.all(np.isnan(out[done == 0]))
    assert not np.any(np.isnan(out[done == 1]))


def test_stopped_and_resumed_plans_equal_the_uninterrupted_plan():
    items = _items()
    n = len(items)
    want, done_all = oplan.plan_run(11, items)
    assert np.all(done_all == 1)
    for k in (1, 9, 39):
        out, done = oplan.plan_run(11, items, max_items=k)
        assert done.sum() == k
        out2, done2 = oplan.plan_run(11, items, skip_done=done, prev=out)
        assert np.all(done2 == 1)
        assert np.array_equal(out2, want)
    # stopped twice, then finished
    out, done = oplan.plan_run(11, items, max_items=5)
    out, done = oplan.plan_run(11, items, max_items=6, skip_done=done, prev=out)
    assert done.sum() == 11
    out, done = oplan.plan_run(11, items, skip_done=done, prev=out)
    assert np.array_equal(out, want) and done.sum() == n
    # a resume with every item done runs nothing
    out3, done3 = oplan.plan_run(11, items, skip_done=np.ones(n, np.uint8), prev=want)
    assert np.array_equal(out3, want)

"""Plan runs that stop early and resume, oracle side -- TEST INFRASTRUCTURE ONLY.

An experimental plan (paper section 1) is a set of replication runs at
several factor levels. Each run is a pure function of the seed and its
item, so a plan stopped part-way is finished by running the items that did
not complete, and the result cannot depend on where it stopped.

A plan run serves its items longest first (ties keep their index order),
skips the items a done mask flags, and with an item limit stops after that
many items; it reports per item whether its outputs are final.
"""
import numpy as np

from . import core


def longest_first(customers):
    """Item indices by run length, longest first; equal lengths keep their
    index order."""
    return sorted(range(len(customers)), key=lambda i: -int(customers[i]))


def plan_run(seed, items, max_items=0, skip_done=None, prev=None, threads=1):
    """One plan run: items = iterable of (dp, rep, customers, lambda, mu).
    Runs the items whose skip_done flag is 0 (all without a mask) in
    longest-first order, stopping after max_items of them (0 = no limit).
    Returns (outputs (n, 3) float32: the mean wait, sojourn and idle time
    per item; items not run keep prev's rows, NaN without prev; done (n,)
    uint8: 1 for the items run now or flagged in skip_done)."""
    items = list(items)
    n = len(items)
    skip = np.zeros(n, np.uint8) if skip_done is None else (np.asarray(skip_done) != 0).astype(np.uint8)
    todo = [i for i in longest_first([it[2] for it in items]) if not skip[i]]
    if max_items:
        todo = todo[:max_items]
    out = np.full((n, 3), np.nan, np.float32) if prev is None else np.array(prev, np.float32)
    if todo:
        out[todo] = core.mm1_items(seed, [items[i] for i in todo], threads=threads)
    done = skip.copy()
    done[todo] = 1
    return out, done

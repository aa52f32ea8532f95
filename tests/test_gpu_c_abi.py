"""The library driven from plain C (paper_1501_01405_amd/examples/mrip_from_c.c,
through include/mrip.h only, in a process of its own): its outputs match the
oracle to the same bar as the Python-driven tests (integers bit-exact, fp32
M/M/1 means within 1e-5), and its intervals match numpy's over those
outputs."""
import os
import subprocess

import numpy as np
import pytest

from gpu_util import announce, rel_err
from oracle import core

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1501_01405_amd", "examples", "mrip_from_c")


def _run(*args):
    announce("C client", *args)
    r = subprocess.run([EXE, *map(str, args)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    outs, stats = {}, {}
    for line in r.stdout.splitlines():
        f = line.split()
        if f[0] == "out":
            outs[int(f[1])] = np.array([float(x) for x in f[2:]])
        elif f[0] == "stats":
            stats[int(f[1])] = dict(zip(("n", "mean", "var", "half", "t"), map(float, f[2:])))
    return outs, stats


def _check_stats(x, st):
    x = x.astype(np.float64)
    assert st["n"] == len(x)
    assert abs(st["mean"] - x.mean()) <= 1e-12 * max(1.0, abs(x.mean()))
    assert abs(st["var"] - x.var(ddof=1)) <= 1e-9 * max(1e-300, x.var(ddof=1))


@pytest.mark.parametrize("mapping", ["wave", "simt", "lane0"])
def test_pi_from_c(gpu, mapping):
    outs, stats = _run("pi", 100001, 40, 7, mapping)
    ref = core.pi_many(7, 40, 100001, threads=core.default_threads())
    assert np.array_equal(outs[0].astype(np.int64), ref)
    assert np.array_equal(outs[1].astype(np.float32), (4.0 * ref / 100001).astype(np.float32))
    _check_stats(outs[0], stats[0])


@pytest.mark.parametrize("mapping,split", [("wave", 1), ("wave", 4), ("simt", 1)])
def test_mm1_from_c(gpu, mapping, split):
    outs, stats = _run("mm1", 0.9, 1.0, 20000, 33, 5, mapping, split)
    got = np.stack([outs[k] for k in range(3)], axis=1).astype(np.float32)
    ref = core.mm1_many(5, 33, 20000, 0.9, 1.0, threads=core.default_threads())
    assert rel_err(got, ref).max() <= 1e-5
    for k in range(3):
        _check_stats(outs[k].astype(np.float32), stats[k])


@pytest.mark.parametrize("mapping", ["wave", "simt"])
def test_rw_from_c(gpu, mapping):
    outs, stats = _run("rw", 64, 64, 1000, 32, 11, mapping, 1)
    ref = core.rw_many(11, 32, 64, 64, 1000, threads=core.default_threads(), walker_sites=True)
    for k in range(3):
        assert np.array_equal(outs[k].astype(np.int64), ref[k])
        _check_stats(outs[k], stats[k])

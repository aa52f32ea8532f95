"""Host-side parts of bench.py that need no GPU: the refusal of more than
one GPU, the algorithmic slot counts its rooflines divide by, and its
command-line defaults."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_slot_counts():
    # Philox block: 20 multiply-adds at 2.12 slots and 20 three-input xors
    assert abs(bench.philox_block_slots() - 62.4) < 1e-9
    # M/M/1: half a block, two variates (4 simple + convert 1.9 + log 3.15),
    # Lindley 5, sums 3
    assert abs(bench.mm1_slots_per_customer() - (31.2 + 2 * 9.05 + 8)) < 1e-9
    assert abs(bench.ff_slots_per_cell() - (15.6 + 2 + 0.25)) < 1e-9
    assert abs(bench.rw_slots_per_step() - (62.4 / 64 + 8)) < 1e-9
    assert abs(bench.pi_slots_per_point() - (31.2 + 4 + 4.24 + 2)) < 1e-9
    assert bench.taus88_output_slots() == 19.0
    r = bench.alu_roofline(1e12, 10.0)
    assert r["bound"] == "alu" and abs(r["frac"] - 1e13 / bench.PEAK_LANE_OPS) < 1e-12


def test_defaults_and_split_choice(monkeypatch):
    # the default run warms up in the pipelined form before timing; the
    # headline's wavefronts per replication are one of the split kernels'
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.gpus, a.steps, a.warmup, a.split) == (1, 200, 300, bench.SPLIT)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--split", "8", "--steps", "5"])
    a = bench.parse()
    assert (a.split, a.steps) == (8, 5)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--split", "3"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr

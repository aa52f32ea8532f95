"""Helpers shared by the GPU parity tests."""
import numpy as np

from paper_1501_01405_amd import mrip

SIMT, WAVE, LANE0 = mrip.MRIP_MAP_SIMT, mrip.MRIP_MAP_WAVE, mrip.MRIP_MAP_LANE0


def rel_err(got, ref, floor=1e-6):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def announce(*what):
    """Name the case on stdout before a GPU step (a fault may end the process)."""
    print("[gpu case]", *what, flush=True)

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import core
    return core.lib()


@pytest.fixture(scope="session")
def philox_ref():
    """Independent Philox engines (PyTorch, rocRAND), compiled from their headers."""
    import ctypes as C

    import numpy as np
    import torch
    src = os.path.join(ROOT, "tests", "pins", "philox_ref.cpp")
    out = os.path.join(ROOT, "tests", "pins", "libphilox_ref.so")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        inc = os.path.join(os.path.dirname(torch.__file__), "include")
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I" + inc, src, "-o", out + ".tmp%d" % os.getpid()], check=True)
        os.replace(out + ".tmp%d" % os.getpid(), out)
    lib = C.CDLL(out)
    p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    for fn in (lib.torch_philox_batch, lib.rocrand_philox_batch):
        fn.argtypes = [C.c_uint64, p, p, p]
        fn.restype = None
    return lib


@pytest.fixture(scope="session")
def gpu():
    """The built GPU library on a real device; fails loudly when it is absent."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1501_01405_amd import mrip
    mrip.load()  # raises if libmrip.so was not built
    return mrip

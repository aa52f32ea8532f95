"""CPU oracle for the MRIP hot path -- TEST INFRASTRUCTURE ONLY.

A slow, sequential, obviously correct implementation of every computation
the GPU library performs, written from the paper and the model definitions,
sharing no code with the GPU library. Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product never does.

  core   Philox4x32-10, variates, random walk, M/M/1, forest fire (C, ctypes)
  stats  mean / unbiased variance / Student-t interval
  mlp    bf16-operand MLP forward, backward and Adam
  cv     control-variate estimator and the host steps of its training

Parity status of each function is recorded with its tests; every function
here has at least one pin independent of itself.
"""
from . import core, cv, mlp, stats  # noqa: F401

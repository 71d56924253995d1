"""CPU oracle for the homomorphic-convolution hot path -- TEST INFRASTRUCTURE.

A plain, slow, obviously correct CPU implementation of what the HIP path
computes, written from the paper (SecONNds, arXiv 2506.11586) before any
kernel.  Only `tests/`, the smoke check and the benchmark's CPU-baseline leg
may import it; the product package never does, and the two share no code
(only the seeded input generators in `synth.py`, which hold none of the
method's arithmetic).

Modules:
  heoracle.c  exact integer core (u128 products, `%` reduction)
  core.py     ctypes binding of the core, parameters, packing, planner,
              BFV client side, layer references, decode
  mirror.py   pure-Python big-integer mirror for tiny N (independent check)

Parity pins for every function live in tests/test_oracle_*.py.  Parts with no
pin are marked "parity unpinned" in their docstrings.
"""
from .core import *  # noqa: F401,F403

"""CPU FP64 oracle for the accelerated FBP method (Dolmatova, Chukalina, Nikolaev 2020).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this; only the test suite,
the smoke check and the benchmark's CPU-baseline leg may call it.  It shares no code with the
HIP path: the two meet only at the seeded input generators in ``fbp_inputs``.

Every function is written in plain PyTorch CPU ops in float64, following the paper's
definitions and notation; see ``oracle.fbp_oracle`` for the per-function citations.
"""
from .fbp_oracle import *  # noqa: F401,F403

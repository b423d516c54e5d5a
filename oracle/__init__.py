"""CPU oracle for the GFORS hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, FP64 / exact-integer restatement of the
method (PDHG on the penalised saddle problem, Bernoulli sampling, exact
candidate evaluation, incumbent update).  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path (the HIP library and its Python binding) never does.  It shares no code
with the GPU path.
"""
from .gfors_oracle import *  # noqa: F401,F403

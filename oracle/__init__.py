"""FP64 CPU oracle for the GS^3 triple-splatting path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package's smoke check and
the benchmark's CPU-baseline leg may import this package. The HIP library
never calls it and shares no code, headers, tables or constants with it.

Every function follows the paper (Bi et al., "GS^3: Efficient Relighting
with Triple Gaussian Splatting", SIGGRAPH Asia 2024) step by step, in torch
float64 on the CPU, and is differentiable with torch autograd so that the
same code yields the reference gradients.
"""
from .gs3_oracle import *  # noqa: F401,F403
from .gs3_oracle import __all__  # noqa: F401

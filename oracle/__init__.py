"""Plain FP64 CPU reference of the D3Q19 lattice-Boltzmann update.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the product path never does.  It shares no
code with the HIP library.  See ``lb_oracle`` for the formulas and the
reading of the paper behind each of them.
"""

from . import lb_oracle  # noqa: F401

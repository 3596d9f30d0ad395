"""Plain FP64 CPU oracle of the HMCSC lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY.  Imported by the test-suite, by the smoke check and by
the CPU-baseline leg of the benchmark to check the GPU library; the product path
never imports it.  See ``hmcsc_oracle.c`` for the steps it follows and the
readings of the paper it takes.
"""
from .ref import Oracle, build, lattice, params_struct  # noqa: F401

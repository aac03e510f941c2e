"""FP64 CPU oracle of the fourth-order BGK lattice Boltzmann model.

Test infrastructure only: imported by the tests, by the package smoke check and
by the CPU-baseline leg of the benchmark, never by the product path.
"""
from .lbm_oracle import *  # noqa: F401,F403

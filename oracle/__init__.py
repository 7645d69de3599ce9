"""CPU FP64 oracle for screened orbital-space VMC.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product library.  It shares
no code with the GPU path.

* ``oracle.core``   -- ctypes wrapper of the plain C oracle (``vmc_oracle.c``):
  screened local energy, CTMC move, gradient ratios, Philox.
* ``oracle.brute``  -- numpy brute force over a whole (N_alpha, N_beta) sector
  for tiny systems: the Hamiltonian matrix from second-quantised operators,
  exact energies, exact diagonalisation.
* ``oracle.optim``  -- energy/gradient estimators and AMSGrad.

Parity is pinned as documented in each module and in the CPU tests.
"""
from .core import OracleSystem, build_oracle_library, philox4x64_10, uniform  # noqa: F401

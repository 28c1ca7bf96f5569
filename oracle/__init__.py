"""FP64 CPU oracle for the coupled TRT-LBM / FFT-Poisson electroconvection step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
C ABI or the Python binding) imports, links or calls this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark do.  It shares
no code with the GPU path: the only input both sides agree on is the seeded
charge noise, which each side generates from the published SplitMix64
definition independently.

The oracle follows Guan & Novosselov, "Two Relaxation Time Lattice Boltzmann
Method Coupled to Fast Fourier Transform Poisson Solver: Application to
Electroconvective Flow" (arXiv:1812.05711):

  lattice.py      D2Q9 set (section IV.2) and the TRT parameters (Eq. 16-17)
                  mapped from the nondimensional groups (Eq. 26)
  hydrostatic.py  closed-form hydrostatic charge / field profile (Eq. 27-28)
  splitmix.py     SplitMix64 generator for the seeded initial charge noise
  poisson.py      spectral-x / finite-difference-y Poisson solve (Eq. 18-25)
  lbm.py          moments, equilibria, forcing, TRT collision (Eq. 5-15)
                  and streaming with the wall conditions (Table I)
  solver.py       the time loop and the nondimensional output fields
  diagnostics.py  mass, charge, boundary fluxes, error metrics

Every function is plain FP64 NumPy, unblocked and unfused, in the order the
paper gives the steps.  Pins that tie it to the paper and to mathematics
live in tests/test_oracle_*.py.
"""

from .lattice import Params, LatticeConstants, lattice_constants, CI, WI, OPP, CS2
from .solver import Oracle

__all__ = [
    "Params",
    "LatticeConstants",
    "lattice_constants",
    "CI",
    "WI",
    "OPP",
    "CS2",
    "Oracle",
]

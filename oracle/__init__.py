"""FP64 CPU oracle of the multicomponent thread-safe lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU library never does.  Two independent
routes live here:

* ``Oracle`` -- ctypes binding of ``tslb_oracle.c``: populations, A/B arrays,
  push streaming (the plain scheme the thread-safe step rewrites).
* ``moment_route`` -- a numpy route that stores only moments and rebuilds
  populations from the neighbours (the rewrite itself, Methodology Eqs. 6 and 8),
  used to check the C oracle and the equivalence the paper claims.
"""
from .oracle import (Oracle, OrcParams, build_oracle, library_path, lattice, collide, collide_vd,  # noqa: F401
                     phase_collide, noise)

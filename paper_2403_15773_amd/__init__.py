"""MI355X-native multicomponent thread-safe lattice Boltzmann (TSLB) step.

The GPU library (``libtslb.so``: hand-written HIP kernels for gfx950 behind the
C-ABI declared in ``include/tslb.h``) is loaded lazily by
``paper_2403_15773_amd.tslb``; importing the package itself loads nothing.
"""

"""MI355X-native axisymmetric cascaded central-moment lattice Boltzmann time
step (arXiv 1806.10241, Section 2): HIP kernels for gfx950 behind the C-ABI
library ``libaxlb.so`` (declared in ``include/axlb.h``); ``axlb`` is the thin
ctypes binding, ``inputs`` builds seeded synthetic workloads."""

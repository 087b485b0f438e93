"""MI355X-native REXI propagation step for the time-dependent Schroedinger equation.

Modules
-------
inputs   seeded synthetic grids, potentials, packets and workloads
poles    host (FP64) Faber-CF poles and weights
rexi     ctypes binding of the HIP library librexi.so (C ABI in include/rexi.h)
autograd torch.autograd.Function around the step and its adjoint
build    compiles librexi.so for gfx950

``rexi`` and ``autograd`` load the HIP library on import and raise if it
has not been built.
"""

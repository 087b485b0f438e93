"""FP64 CPU oracle for the REXI propagation step (test infrastructure).

This package is test infrastructure: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import or call it. The GPU
path never does, and this package imports nothing from the GPU path.

Contents
--------
faber_cf   Faber-Caratheodory-Fejer construction of poles and weights
           (Section 3.2, Algorithms 1 and 2, conformal map eq.
           ``map-to-imaginary``).
hamiltonian  The finite-difference Hamiltonian H = -(hbar^2/2m) Lap_h + V
           of eq. ``schroedinger`` with zero Dirichlet values (Section 1).
step       The REXI step of eq. ``rational-evaluation`` by direct solves,
           by eigendecomposition (Section 3.1), by the free-particle DST
           closed form and by separable (Kronecker) eigendecomposition;
           the adjoint step; certificates.
krylov     A plain restarted GMRES (modified Gram-Schmidt), used only to
           time a CPU Krylov step where a direct solve is infeasible.

Parity unpinned: none of the functions above; every one is checked by
the oracle tests against a closed form, a library routine or an invariant.
"""

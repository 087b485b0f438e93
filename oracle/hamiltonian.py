"""The finite-difference Hamiltonian (oracle, FP64, test infrastructure).

H = -(hbar^2 / 2m) Lap_h + diag(V): the semi-discrete form of eq.
``schroedinger`` (Section 1) on a tensor grid of interior points with zero
Dirichlet values on the boundary (Section 1). With finite differences the
two bilinear forms of Section 2 become A = H and B = hbar I, so the IVP of
eq. ``ode-system`` reads  i hbar u' = H u.

The discrete Laplacian is the Kronecker sum of the 1D second-difference
matrices  T_a = h_a^{-2} tridiag(1, -2, 1)  (one per axis, C order: the last
axis is the fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def kinetic_1d(n, h, hbar=1.0, mass=1.0):
    """``-(hbar^2/2m) d^2/dx^2`` on ``n`` interior points, sparse tridiagonal."""
    c = hbar * hbar / (2.0 * mass * h * h)
    main = np.full(n, 2.0 * c)
    off = np.full(n - 1, -c)
    return sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="csr")


def hamiltonian(n, h, V, hbar=1.0, mass=1.0):
    """Sparse H (CSR, float64) for grid sizes ``n`` and spacings ``h``."""
    n = tuple(int(k) for k in n)
    d = len(n)
    N = int(np.prod(n))
    Hm = sp.csr_matrix((N, N))
    for a in range(d):
        left = sp.identity(int(np.prod(n[:a])), format="csr")
        right = sp.identity(int(np.prod(n[a + 1:])), format="csr")
        Hm = Hm + sp.kron(sp.kron(left, kinetic_1d(n[a], h[a], hbar, mass)), right, format="csr")
    return (Hm + sp.diags(np.asarray(V, dtype=np.float64).ravel(), 0)).tocsr()


def apply_shifted(n, h, V, x, shift, hbar=1.0, mass=1.0):
    """``y = (H - shift I) x`` via the sparse matrix (complex128 in and out)."""
    H = hamiltonian(n, h, V, hbar, mass)
    x = np.asarray(x, dtype=np.complex128).ravel()
    return H @ x - shift * x


def laplacian_eigenvalues_1d(n, h, hbar=1.0, mass=1.0):
    """Eigenvalues of ``kinetic_1d``: (hbar^2/2m)(4/h^2) sin^2(k pi / (2(n+1))), k=1..n.

    The eigenvectors are the DST-I vectors sin(i k pi / (n+1)).
    """
    k = np.arange(1, n + 1)
    return hbar * hbar / (2.0 * mass) * 4.0 / (h * h) * np.sin(k * np.pi / (2.0 * (n + 1))) ** 2


def gershgorin(n, h, V, hbar=1.0, mass=1.0):
    """An interval containing spec(H): [min V, (hbar^2/2m) sum_a 4/h_a^2 + max V]."""
    V = np.asarray(V)
    return float(V.min()), float(hbar * hbar / (2.0 * mass) * sum(4.0 / (hh * hh) for hh in h) + V.max())

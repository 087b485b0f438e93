"""The mass-matrix form of the REXI step (oracle, FP64, test infrastructure).

Section 2 discretises the weak form with finite elements: the IVP
i B u' = A u of eq. ``ode-system`` with A_jk = a(chi_j, chi_k),
B_jk = b(chi_j, chi_k), a(phi, psi) = int (hbar^2/2m) grad phi . grad psi
+ V phi psi, b = hbar int phi psi. Here the elements are tensor-product
linear (Q1) elements on the same grid of interior nodes as the finite
differences (zero Dirichlet values on the boundary), so with the 1D mass and
stiffness matrices
    M_a = (h_a / 6) tridiag(1, 4, 1),   K_a = (1 / h_a) tridiag(-1, 2, -1)
the consistent mass matrix is M = M_0 x M_1 x M_2 (Kronecker product, C
order) and the stiffness matrix is K = sum_a (.. x K_a x ..) with M_b on
the other axes. The potential term int V phi_j phi_k is taken with nodal
quadrature, V_j int phi_j delta_jk = h^d V_j delta_jk (a reading: the
consistent product of three basis functions would make the operator depend
on V at up to 27 nodes per entry). So
    A = (hbar^2/2m) K + h^d diag(V),   B = hbar M,
and eq. ``rational-evaluation`` becomes
    u_1 = sum_j w_j (A - s_j M)^{-1} M u_0,   s_j = i hbar sigma_j / tau,
    w_j = i hbar beta_j / tau
(the same shifts and weights as with finite differences). Centering solves
with A - c M and multiplies by exp(-i tau c / hbar).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .step import rational, shifts_and_weights, step_factor


def mass_1d(n, h):
    """(h/6) tridiag(1, 4, 1) on n interior nodes."""
    return sp.diags([np.full(n - 1, h / 6.0), np.full(n, 4.0 * h / 6.0), np.full(n - 1, h / 6.0)],
                    [-1, 0, 1], shape=(n, n), format="csr")


def stiffness_1d(n, h):
    """(1/h) tridiag(-1, 2, -1) on n interior nodes."""
    return sp.diags([np.full(n - 1, -1.0 / h), np.full(n, 2.0 / h), np.full(n - 1, -1.0 / h)],
                    [-1, 0, 1], shape=(n, n), format="csr")


def _kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return out


def matrices(n, h, V, hbar=1.0, mass=1.0):
    """(A, M): A = (hbar^2/2m) K + h^d diag(V), M the consistent mass matrix."""
    n = tuple(int(k) for k in n)
    Ms = [mass_1d(n[a], h[a]) for a in range(len(n))]
    M = _kron_all(Ms)
    K = None
    for a in range(len(n)):
        mats = [stiffness_1d(n[b], h[b]) if b == a else Ms[b] for b in range(len(n))]
        term = _kron_all(mats)
        K = term if K is None else K + term
    vol = float(np.prod(h))
    A = hbar * hbar / (2.0 * mass) * K + sp.diags(vol * np.asarray(V, dtype=np.float64).ravel(), 0)
    return A.tocsr(), M.tocsr()


def p1_eigenvalues_1d(n, h, hbar=1.0, mass=1.0):
    """Generalised eigenvalues of ((hbar^2/2m) K_1, M_1) with V = 0, closed form:
    (hbar^2/2m)(6/h^2)(1 - cos t_k)/(2 + cos t_k), t_k = k pi/(n+1), eigenvectors
    the DST-I vectors sin(i t_k)."""
    t = np.arange(1, n + 1) * np.pi / (n + 1)
    return hbar * hbar / (2.0 * mass) * 6.0 / (h * h) * (1.0 - np.cos(t)) / (2.0 + np.cos(t))


def spectrum_bound(n, h, V, hbar=1.0, mass=1.0):
    """An interval containing the generalised eigenvalues of (A, M).

    Rayleigh quotients: the kinetic part lies in [0, sum_a (hbar^2/2m) 12/h_a^2]
    (per axis the 1D closed form is below 12/h^2); the potential part
    h^d sum V |x|^2 / x^H M x lies between V_min and V_max scaled by the
    eigenvalue range of M / h^d, [3^-d, 1].
    """
    V = np.asarray(V)
    d = len(n)
    lo_v, hi_v = float(V.min()), float(V.max())
    lo = min(lo_v, lo_v * 3.0 ** d)
    hi = hbar * hbar / (2.0 * mass) * sum(12.0 / (hh * hh) for hh in h) + max(hi_v, hi_v * 3.0 ** d)
    return lo, hi


class FemDirectStepper:
    """Step by exact sparse LU solves of (A - s_j M) x = M psi, one factorisation per pole."""

    def __init__(self, n, h, V, sigma, beta, dt, hbar=1.0, mass=1.0, center=0.0, stab_eps=0.0):
        self.n = tuple(n)
        self.s, self.w = shifts_and_weights(sigma, beta, dt, hbar)
        self.w = self.w * step_factor(dt, hbar, center, stab_eps)
        self.A, self.M = matrices(n, h, V, hbar, mass)
        Ac = (self.A - center * self.M).astype(np.complex128).tocsc()
        Mc = self.M.astype(np.complex128).tocsc()
        self.facs = [spla.splu((Ac - sj * Mc).tocsc()) for sj in self.s]

    def step(self, psi):
        b = self.M @ np.asarray(psi, dtype=np.complex128).ravel()
        out = np.zeros(b.size, dtype=np.complex128)
        for wj, f in zip(self.w, self.facs):
            out += wj * f.solve(b)
        return out.reshape(self.n)


class FemEigStepper:
    """Step by the generalised eigendecomposition A Q = M Q diag(lam), Q^T M Q = I
    (dense, tiny grids): r(tau M) applies r(-i tau lam / hbar) to the
    coefficients Q^T M psi."""

    def __init__(self, n, h, V, hbar=1.0, mass=1.0):
        self.n = tuple(n)
        self.hbar = hbar
        A, M = matrices(n, h, V, hbar, mass)
        self.Mdense = M.toarray()
        self.lam, self.Q = sla.eigh(A.toarray(), self.Mdense)

    def apply(self, psi, fvals):
        c = self.Q.T @ (self.Mdense @ np.asarray(psi, dtype=np.complex128).ravel())
        return (self.Q @ (fvals * c)).reshape(self.n)

    def step(self, psi, sigma, beta, dt, center=0.0, stab_eps=0.0):
        f = step_factor(dt, self.hbar, center, stab_eps)
        return self.apply(psi, f * rational(-1j * dt * (self.lam - center) / self.hbar, sigma, beta))

    def exact(self, psi, t):
        return self.apply(psi, np.exp(-1j * t * self.lam / self.hbar))

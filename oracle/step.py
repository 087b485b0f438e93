"""The REXI propagation step (oracle, FP64, test infrastructure).

Definition (eq. ``rational-evaluation``, Section 3.1): with poles and weights
(sigma_j, beta_j) of r(z) = sum_j beta_j/(z - sigma_j) ~ exp(z) and step tau,
    u_1 = sum_j beta_j (tau A - sigma_j iB)^{-1} (iB) u_0 .
For finite differences A = H and B = hbar I, so
    psi_1 = sum_j w_j (H - s_j I)^{-1} psi_0,
    s_j = i hbar sigma_j / tau,   w_j = i hbar beta_j / tau .
The step is the matrix function r(tau M) with M = (iB)^{-1} A (eq.
``matrix-exp-solution``); for symmetric H = Q diag(lam) Q^T this is
Q diag(r(-i tau lam / hbar)) Q^T (Section 3.1, matrix functions by
diagonalisation). Every routine below computes that one result by a
different exact route; none iterates.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.fft as sfft

from .hamiltonian import hamiltonian, laplacian_eigenvalues_1d


def shifts_and_weights(sigma, beta, dt, hbar=1.0):
    """(s_j, w_j) = (i hbar sigma_j / dt, i hbar beta_j / dt)."""
    sigma = np.asarray(sigma, dtype=np.complex128)
    beta = np.asarray(beta, dtype=np.complex128)
    return 1j * hbar * sigma / dt, 1j * hbar * beta / dt


def step_factor(dt, hbar=1.0, center=0.0, stab_eps=0.0):
    """Scalar that multiplies every weight.

    Stabilisation (Section 3.4): the coefficients beta_j are multiplied by
    1 - eps, eps slightly above the approximation error, so that |r(iy)| <= 1.
    Centering (not in the paper): exp(-i dt H / hbar) = exp(-i dt c / hbar)
    exp(-i dt (H - c) / hbar), so the step may solve with H - c I and multiply
    by the scalar phase; with c the midpoint of the spectrum the interval the
    approximation must cover halves.
    """
    return (1.0 - stab_eps) * np.exp(-1j * dt * center / hbar)


def rational(z, sigma, beta):
    """r(z) = sum_j beta_j / (z - sigma_j) (eq. ``partial-fraction-decomposition``)."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.zeros(z.shape, dtype=np.complex128)
    for sj, bj in zip(sigma, beta):
        out = out + bj / (z - sj)
    return out


class DirectStepper:
    """Step by exact sparse LU solves, one factorisation per pole (reused).

    1D grids use the banded (tridiagonal) LU of LAPACK, the rest SuperLU.
    """

    def __init__(self, n, h, V, sigma, beta, dt, hbar=1.0, mass=1.0, center=0.0, stab_eps=0.0):
        self.n = tuple(n)
        self.s, self.w = shifts_and_weights(sigma, beta, dt, hbar)
        self.w = self.w * step_factor(dt, hbar, center, stab_eps)
        self.H = hamiltonian(n, h, V, hbar, mass)
        if center != 0.0:
            self.H = (self.H - center * sp.identity(self.H.shape[0], format="csr")).tocsr()
        N = self.H.shape[0]
        self.N = N
        self.banded = len(self.n) == 1
        self.facs = []
        if self.banded:
            diag = self.H.diagonal()
            off = self.H.diagonal(1)
            self.ab = []
            for sj in self.s:
                ab = np.zeros((3, N), dtype=np.complex128)
                ab[0, 1:] = off
                ab[1, :] = diag - sj
                ab[2, :-1] = off
                self.ab.append(ab)
        else:
            I = sp.identity(N, dtype=np.complex128, format="csc")
            for sj in self.s:
                self.facs.append(spla.splu((self.H.astype(np.complex128) - sj * I).tocsc()))

    def solve(self, j, b, conjugate=False):
        """x = (H - s_j I)^{-1} b, or (H - conj(s_j) I)^{-1} b if ``conjugate``.

        H is real, so (H - conj s)^{-1} b = conj((H - s)^{-1} conj b).
        """
        b = np.asarray(b, dtype=np.complex128).ravel()
        if conjugate:
            return np.conj(self.solve(j, np.conj(b)))
        if self.banded:
            return sla.solve_banded((1, 1), self.ab[j], b)
        return self.facs[j].solve(b)

    def step(self, psi):
        psi = np.asarray(psi, dtype=np.complex128).ravel()
        out = np.zeros(self.N, dtype=np.complex128)
        for j, wj in enumerate(self.w):
            out += wj * self.solve(j, psi)
        return out.reshape(self.n)

    def solutions(self, psi):
        """The K per-pole solutions x_j = (H - s_j)^{-1} psi, shape [K, N]."""
        psi = np.asarray(psi, dtype=np.complex128).ravel()
        return np.stack([self.solve(j, psi) for j in range(len(self.s))])

    def adjoint(self, psi_n, gbar_next):
        """One backward step of L(psi_N) through psi_{n+1} = R psi_n.

        With R = sum_j w_j (H - s_j)^{-1} and the conjugate-Wirtinger
        gradient gbar = dL/d conj(psi):
          gbar_n  = R^H gbar_{n+1} = sum_j conj(w_j) (H - conj s_j)^{-1} gbar_{n+1}
          dL/dV_k = -2 Re sum_j w_j conj(y_j[k]) x_j[k],
        x_j = (H - s_j)^{-1} psi_n, y_j = (H - conj s_j)^{-1} gbar_{n+1}
        (H real symmetric, so (H - s)^H = H - conj s).
        """
        psi_n = np.asarray(psi_n, dtype=np.complex128).ravel()
        g = np.asarray(gbar_next, dtype=np.complex128).ravel()
        gout = np.zeros(self.N, dtype=np.complex128)
        dV = np.zeros(self.N, dtype=np.float64)
        for j, wj in enumerate(self.w):
            x = self.solve(j, psi_n)
            y = self.solve(j, g, conjugate=True)
            gout += np.conj(wj) * y
            dV += -2.0 * np.real(wj * np.conj(y) * x)
        return gout.reshape(self.n), dV.reshape(self.n)


def step_dense(n, h, V, psi, sigma, beta, dt, hbar=1.0, mass=1.0):
    """One step by dense LU per pole (tiny grids)."""
    s, w = shifts_and_weights(sigma, beta, dt, hbar)
    H = hamiltonian(n, h, V, hbar, mass).toarray().astype(np.complex128)
    N = H.shape[0]
    psi = np.asarray(psi, dtype=np.complex128).ravel()
    out = np.zeros(N, dtype=np.complex128)
    for sj, wj in zip(s, w):
        out += wj * sla.solve(H - sj * np.eye(N), psi)
    return out.reshape(tuple(n))


class EigStepper:
    """Step by the eigendecomposition H = Q diag(lam) Q^T (dense, tiny grids).

    ``step`` applies r(-i dt lam / hbar); ``exact`` applies exp(-i dt lam / hbar),
    the exact propagator of eq. ``matrix-exp-solution``.
    """

    def __init__(self, n, h, V, hbar=1.0, mass=1.0):
        self.n = tuple(n)
        self.hbar = hbar
        H = hamiltonian(n, h, V, hbar, mass).toarray()
        self.lam, self.Q = np.linalg.eigh(H)

    def apply(self, psi, fvals):
        c = self.Q.T @ np.asarray(psi, dtype=np.complex128).ravel()
        return (self.Q @ (fvals * c)).reshape(self.n)

    def step(self, psi, sigma, beta, dt, center=0.0, stab_eps=0.0):
        f = step_factor(dt, self.hbar, center, stab_eps)
        return self.apply(psi, f * rational(-1j * dt * (self.lam - center) / self.hbar, sigma, beta))

    def exact(self, psi, t):
        return self.apply(psi, np.exp(-1j * t * self.lam / self.hbar))


class SeparableStepper:
    """Step for V(r) = sum_a V_a(x_a): H = sum_a I x .. x H_a x .. x I.

    Each 1D H_a = kinetic_1d + diag(V_a) is diagonalised (dense eigh); the
    step multiplies the coefficients by r(-i dt (lam_1 + .. + lam_d) / hbar).
    With every V_a = 0 this is the free particle, whose eigenvectors are DST-I
    vectors (see ``FreeParticleStepper``).
    """

    def __init__(self, n, h, V_parts, hbar=1.0, mass=1.0):
        self.n = tuple(n)
        self.hbar = hbar
        self.Q, lam = [], []
        for a in range(len(n)):
            Ha = hamiltonian((n[a],), (h[a],), V_parts[a], hbar, mass).toarray()
            la, Qa = np.linalg.eigh(Ha)
            self.Q.append(Qa)
            lam.append(la)
        self.lam = lam[0]
        for la in lam[1:]:
            self.lam = np.add.outer(self.lam, la)

    def _fwd(self, x):
        for a, Qa in enumerate(self.Q):
            x = np.moveaxis(np.tensordot(Qa.T, np.moveaxis(x, a, 0), axes=1), 0, a)
        return x

    def _bwd(self, x):
        for a, Qa in enumerate(self.Q):
            x = np.moveaxis(np.tensordot(Qa, np.moveaxis(x, a, 0), axes=1), 0, a)
        return x

    def apply(self, psi, fvals):
        c = self._fwd(np.asarray(psi, dtype=np.complex128).reshape(self.n))
        return self._bwd(fvals * c)

    def step(self, psi, sigma, beta, dt):
        return self.apply(psi, rational(-1j * dt * self.lam / self.hbar, sigma, beta))

    def exact(self, psi, t):
        return self.apply(psi, np.exp(-1j * t * self.lam / self.hbar))


class FreeParticleStepper:
    """V = 0: H is diagonal in the DST-I basis with the closed-form eigenvalues
    (hbar^2/2m) sum_a (4/h_a^2) sin^2(k_a pi / (2(n_a+1)))."""

    def __init__(self, n, h, hbar=1.0, mass=1.0):
        self.n = tuple(n)
        self.hbar = hbar
        lam = laplacian_eigenvalues_1d(n[0], h[0], hbar, mass)
        for a in range(1, len(n)):
            lam = np.add.outer(lam, laplacian_eigenvalues_1d(n[a], h[a], hbar, mass))
        self.lam = lam

    def apply(self, psi, fvals):
        x = np.asarray(psi, dtype=np.complex128).reshape(self.n)
        c = sfft.dstn(x, type=1, norm="ortho")
        return sfft.idstn(fvals * c, type=1, norm="ortho")

    def step(self, psi, sigma, beta, dt):
        return self.apply(psi, rational(-1j * dt * self.lam / self.hbar, sigma, beta))

    def exact(self, psi, t):
        return self.apply(psi, np.exp(-1j * t * self.lam / self.hbar))


def certificate(n, h, V, psi, x, shift, lam_interval, hbar=1.0, mass=1.0):
    """Forward-error bound of one approximate shifted solve.

    H is real symmetric, so H - s I is normal and
    ||x - x*||_2 <= ||psi - (H - s)x||_2 / dist(s, [lam_min, lam_max]).
    Returns (residual norm, bound).
    """
    H = hamiltonian(n, h, V, hbar, mass)
    psi = np.asarray(psi, dtype=np.complex128).ravel()
    x = np.asarray(x, dtype=np.complex128).ravel()
    r = psi - (H @ x - shift * x)
    lo, hi = lam_interval
    re = min(max(shift.real, lo), hi)
    dist = abs(complex(re, 0.0) - shift)
    rn = float(np.linalg.norm(r))
    return rn, rn / dist


def rel_err(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))

"""A plain CPU GMRES step (oracle, FP64, test infrastructure).

Where a direct solve of (H - s_j I) x = psi is infeasible (a 128^3 grid),
the oracle solves each pole's system with textbook restarted GMRES
(modified Gram-Schmidt Arnoldi, Givens rotations, x0 = 0) on the sparse H
to a tight relative residual, then forms the weighted sum of eq.
``rational-evaluation``. The normality of H - s I turns the final residual
into a forward-error bound (``oracle.step.certificate``), which is what
makes an iterative result usable as a reference.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .hamiltonian import hamiltonian
from .step import shifts_and_weights


def gmres(matvec, b, tol=1e-14, m=60, max_restarts=50):
    """Solve A x = b, A given by ``matvec``; returns (x, iterations, rel. residual)."""
    b = np.asarray(b, dtype=np.complex128)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    its = 0
    r = b.copy()
    for _ in range(max_restarts):
        beta = np.linalg.norm(r)
        if beta <= tol * bn:
            break
        Vb = [r / beta]
        Hh = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            w = matvec(Vb[j])
            for i in range(j + 1):
                Hh[i, j] = np.vdot(Vb[i], w)
                w = w - Hh[i, j] * Vb[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            Vb.append(w / Hh[j + 1, j] if Hh[j + 1, j] != 0 else w)
            # rotation i maps (a, b) -> (conj(c) a + conj(s) b, -s a + c b)
            for i in range(j):
                t = np.conj(cs[i]) * Hh[i, j] + np.conj(sn[i]) * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            a, bb = Hh[j, j], Hh[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j] = a / den if den else 1.0
            sn[j] = bb / den if den else 0.0
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            its += 1
            k = j + 1
            if abs(g[j + 1]) <= tol * bn:
                break
        y = np.linalg.solve(np.triu(Hh[:k, :k]), g[:k])
        x = x + np.stack(Vb[:k], axis=1) @ y
        r = b - matvec(x)
    return x, its, float(np.linalg.norm(b - matvec(x)) / bn)


class KrylovStepper:
    """REXI step with one GMRES solve per pole on the sparse Hamiltonian."""

    def __init__(self, n, h, V, sigma, beta, dt, hbar=1.0, mass=1.0, tol=1e-14, m=60):
        self.n = tuple(n)
        self.s, self.w = shifts_and_weights(sigma, beta, dt, hbar)
        self.H = hamiltonian(n, h, V, hbar, mass)
        self.tol, self.m = tol, m

    def solve(self, j, b):
        sj = self.s[j]
        return gmres(lambda x: self.H @ x - sj * x, np.asarray(b, np.complex128).ravel(), self.tol, self.m)

    def step(self, psi, poles=None):
        """The weighted sum over ``poles`` (default all); returns (psi_out, iterations)."""
        poles = range(len(self.s)) if poles is None else poles
        out = np.zeros(int(np.prod(self.n)), dtype=np.complex128)
        its = []
        for j in poles:
            x, k, _ = self.solve(j, psi)
            out += self.w[j] * x
            its.append(k)
        return out.reshape(self.n), its


def host_threads():
    """The CPU cores this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def step_threads(n, h, V, sigma, beta, dt, psi, tols, hbar=1.0, mass=1.0, m=60, workers=None):
    """One REXI step (eq. ``rational-evaluation``) with one ``gmres`` solve per
    pole, the poles spread over ``workers`` threads (default: every core this
    process may use; the sparse products and vector operations release the
    interpreter lock, and BLAS runs one thread per solve).

    ``tols[j]`` is pole j's target relative residual. The weighted sum is
    formed in the fixed pole order. Returns (psi_out, iterations[K], rho[K])
    with rho the final explicit relative residuals ||psi - (H - s_j)x_j|| / ||psi||.
    """
    from threadpoolctl import threadpool_limits

    s, w = shifts_and_weights(sigma, beta, dt, hbar)
    # complex CSR: the same products as the real matrix times a complex vector
    # (a zero imaginary part adds exact zeros), without converting on every call
    H = hamiltonian(n, h, V, hbar, mass).astype(np.complex128)
    b = np.asarray(psi, dtype=np.complex128).ravel()
    workers = workers or host_threads()

    def solve(j):
        return gmres(lambda x: H @ x - s[j] * x, b, float(tols[j]), m)

    with threadpool_limits(limits=1):
        with ThreadPoolExecutor(max_workers=workers) as ex:
            res = list(ex.map(solve, range(len(s))))
    out = np.zeros_like(b)
    for j, (x, _, _) in enumerate(res):
        out += w[j] * x
    return out.reshape(tuple(n)), np.array([r[1] for r in res]), np.array([r[2] for r in res])

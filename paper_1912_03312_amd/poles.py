"""Host setup: Faber-CF poles and weights of r(z) ~ exp(z) on i[-R1, R1].

Computed once per (K, R1), in FP64, on the host (Section 3.1: the shifts
and coefficients do not depend on the initial value or the step). The
construction follows Section 3.2 (Algorithms 1 and 2 with the conformal map
eta(z) = (R1/2)(z - 1/z) of eq. ``map-to-imaginary``), with these choices:

* Faber coefficients of exp: a_j = J_j(R1) (Bessel values), because
  exp(eta(e^{it})) = exp(i R1 sin t) = sum_n J_n(R1) e^{int} (Jacobi-Anger).
* The Hankel matrix of Theorem 1 is real symmetric, so its SVD comes from
  an eigendecomposition: singular values |lambda|, U = Q, V = Q sign(Lambda).
* q(z) = sum_k v_{L-k} z^k from the (K+1)-st right singular vector; its K
  roots outside the unit disc give the poles sigma_j = eta(z_j).
* Weights by linear least squares of sum_j beta_j/(iy - sigma_j) against
  exp(iy) at Chebyshev points y of [-R1, R1] (same residues as Algorithm 2
  in exact arithmetic; well posed where the K x K system of Algorithm 2 is
  numerically singular).
"""
from __future__ import annotations

import numpy as np
from scipy.special import jv


def _truncation(K: int, R1: float) -> int:
    L = int(np.ceil(max(R1 + 40.0, K + 30.0)))
    while abs(jv(L, R1)) >= 1e-18:
        L += 1
    return L


def faber_cf_poles(K: int, R1: float, L: int | None = None, npts: int = 8000):
    """Poles ``sigma`` (complex128[K]) and weights ``beta`` with
    ``sum_j beta_j / (z - sigma_j) ~ exp(z)`` for z in i[-R1, R1].

    Returns ``(sigma, beta, info)``; raises ``ValueError`` when the CF step
    does not yield exactly K poles (degenerate choice of K and R1).
    Poles are ordered by ascending imaginary part, then real part.
    """
    if K < 1 or not (R1 > 0):
        raise ValueError("need K >= 1 and R1 > 0")
    L = L or _truncation(K, R1)
    a = jv(np.arange(L + 1), R1)
    i = np.arange(L + 1)
    s = i[:, None] + i[None, :]
    H = np.where(s <= L, a[np.minimum(s, L)], 0.0)
    lam, Q = np.linalg.eigh(H)
    order = np.argsort(-np.abs(lam))
    lam, Q = lam[order], Q[:, order]
    sv = np.abs(lam)
    v = Q[:, K] * np.sign(lam[K])          # (K+1)-st right singular vector
    q_asc = v[::-1]                        # q(z) = sum_k v_{L-k} z^k
    roots = np.roots(q_asc[::-1])
    zk = roots[np.abs(roots) > 1.0]
    if zk.size != K:
        raise ValueError(f"CF gave {zk.size} exterior roots for K={K}, R1={R1}: "
                         f"sigma_(K+1)/sigma_1 = {sv[K] / sv[0]:.2e}")
    sigma = 0.5 * R1 * (zk - 1.0 / zk)
    sigma = sigma[np.lexsort((sigma.real, sigma.imag))]
    # weights: least squares at Chebyshev points of [-R1, R1]
    th = (np.arange(npts) + 0.5) * np.pi / npts
    y = R1 * np.cos(th)
    A = 1.0 / (1j * y[:, None] - sigma[None, :])
    beta, *_ = np.linalg.lstsq(A, np.exp(1j * y), rcond=None)
    yy = np.linspace(-R1, R1, 40001)
    r = (1.0 / (1j * yy[:, None] - sigma[None, :])) @ beta
    info = dict(L=L, sigma_next=float(sv[K]), err_inf=float(np.max(np.abs(r - np.exp(1j * yy)))),
                amplification=float(np.sum(np.abs(beta) / sigma.real)))
    return sigma.astype(np.complex128), beta.astype(np.complex128), info


def select_poles(dt: float, lam_lo: float, lam_hi: float, err_target: float, hbar: float = 1.0,
                 centered: bool = False, Ks=(10, 16, 24, 32, 48, 64, 96, 128), margin: float = 1.02):
    """Per-configuration choice of (K, R1) for a step ``dt`` on a spectrum of
    H inside [lam_lo, lam_hi] (e.g. ``rexi_estimate_spectrum`` or Gershgorin
    bounds).

    The step is exact up to the approximation error when the eigenvalues of
    tau M lie in i[-R1, R1] (Section "Step-Size Requirements", eq.
    ``convergence-condition``: tau sr(M) <= R1, sr(M) = max |lambda| / hbar), so
    R1 = margin * dt * w / hbar, where w is max(|lam_lo|, |lam_hi|), or the
    half-width (lam_hi - lam_lo) / 2 for a step on H - cI with c the midpoint
    (``center`` option). Returns the smallest K of ``Ks`` whose Faber-CF
    approximation has err_inf <= err_target, as a dict with K, R1, sigma,
    beta and the construction's info; (K, R1) pairs for which the CF step is
    degenerate are skipped. Raises ValueError when no K of ``Ks`` qualifies.
    """
    if not (dt > 0 and hbar > 0 and lam_hi >= lam_lo and err_target > 0):
        raise ValueError("need dt > 0, hbar > 0, lam_hi >= lam_lo and err_target > 0")
    w = 0.5 * (lam_hi - lam_lo) if centered else max(abs(lam_lo), abs(lam_hi))
    R1 = max(margin * dt * w / hbar, 1e-3)
    tried = []
    for K in sorted(Ks):
        try:
            sigma, beta, info = faber_cf_poles(K, R1)
        except ValueError:
            tried.append((K, None))
            continue
        tried.append((K, info["err_inf"]))
        if info["err_inf"] <= err_target:
            return dict(K=K, R1=R1, sigma=sigma, beta=beta, info=info)
    raise ValueError(f"no K in {tuple(Ks)} reaches err_inf <= {err_target:g} at R1 = {R1:g}: {tried}")

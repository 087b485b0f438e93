"""Faber-Caratheodory-Fejer poles and weights (oracle, FP64, test infrastructure).

Follows Section 3.2 of the paper:

* Faber coefficients of ``f = exp`` for the conformal map
  ``eta(z) = (R1/2)(z - 1/z)`` (eq. ``map-to-imaginary``), from the contour
  integral of eq. ``faber-series`` sampled on the unit circle (the FFT route
  the paper names for Maclaurin coefficients).
* Algorithm 1 (CF): Hankel matrix of the coefficients, its SVD, the
  (n+1)-st singular triplet, the best approximation ``r~*`` of Theorem 1, the
  exterior roots of ``q``, the Laurent sequence of ``q_out r~*`` and the CF
  approximant with the negative-index terms dropped.
* Algorithm 2 (FaberCF): poles ``sigma_j = eta(z_j)``, Faber sequences of
  ``w -> 1/(w - sigma_k)``, Maclaurin coefficients of ``r_cf`` and the K x K
  linear system for the weights ``beta``.

Readings where the text is garbled (index typos in Theorem 1 and
Algorithm 1): the Hankel matrix is (L+1) x (L+1) with entries ``a_{i+j}``
(zero beyond L); ``p(z) = sum_k u_k z^k`` and ``q(z) = sum_k v_{L-k} z^k``
(0-based), ``u, v`` the (n+1)-st columns of ``U`` and ``V`` in
``H = U S V^H``; the Laurent sequence is that of ``q_out * r~*``.

Reading for the weights: the K x K system of Algorithm 2 becomes
numerically singular as K grows (its condition number passes 1e15 near
K = 24). When its condition number exceeds ``cond_max`` the weights are
instead the linear least-squares fit of ``sum_k beta_k/(iy - sigma_k)`` to
``exp(iy)`` on ``y`` in ``[-R1, R1]`` -- same poles, a different but
well-posed route to the residues. ``info['weights']`` records which route
was taken.
"""
from __future__ import annotations

import numpy as np


def eta(z, R1):
    """The conformal map of eq. ``map-to-imaginary``: unit circle -> i[-R1, R1]."""
    return 0.5 * R1 * (z - 1.0 / z)


def eta_prime(z, R1):
    return 0.5 * R1 * (1.0 + 1.0 / (z * z))


def laurent_coefficients(fun, nmax, M, radius=1.0):
    """Laurent coefficients ``c_0..c_nmax`` of ``fun`` on the circle ``|z| = radius``.

    ``c_n = (1/2 pi i) \\oint fun(z) z^{-n-1} dz``, sampled with the
    trapezoidal rule at ``M`` equispaced points (an FFT).
    """
    theta = 2.0 * np.pi * np.arange(M) / M
    z = radius * np.exp(1j * theta)
    c = np.fft.fft(fun(z)) / M
    n = np.arange(nmax + 1)
    return c[: nmax + 1] / radius ** n


def faber_sequence_exp(R1, L, M=None):
    """Faber coefficients ``a_0..a_L`` of ``exp`` on ``i[-R1, R1]`` (eq. ``faber-series``)."""
    M = M or max(4096, 8 * (L + 1))
    return laurent_coefficients(lambda z: np.exp(eta(z, R1)), L, M)


def default_L(K, R1):
    """Truncation degree of the Faber series: the smallest ``L >= max(R1 + 40,
    K + 30)`` beyond which the coefficients (Bessel values ``J_L(R1)``) fall
    below 1e-18 -- the paper asks only that the truncation error be
    negligible."""
    from scipy.special import jv
    L = int(np.ceil(max(R1 + 40.0, K + 30.0)))
    while abs(jv(L, R1)) >= 1e-18:
        L += 1
    return L


def cf(a, n, M=None):
    """Algorithm 1: CF approximation of ``h(z) = sum_{j<=L} a_j z^j`` with
    numerator degree ``n - 1`` and denominator degree ``n``.

    Returns ``(num, zk, info)``: ``num`` the coefficients ``d_0..d_{K-1}`` of the
    numerator (ascending), ``zk`` the K roots of ``q`` outside the unit disc (so
    ``r_cf = num(z) / prod_k (z - zk)``) and diagnostics.
    """
    a = np.asarray(a, dtype=np.complex128)
    L = a.size - 1
    # Hankel matrix of Theorem 1 / Algorithm 1: H[i, j] = a_{i+j}, zero past L
    idx = np.add.outer(np.arange(L + 1), np.arange(L + 1))
    H = np.where(idx <= L, a[np.minimum(idx, L)], 0.0)
    U, S, Vh = np.linalg.svd(H)
    s = S[n]                       # (n+1)-st singular value
    u = U[:, n]                    # (n+1)-st column of U
    v = np.conj(Vh[n, :])          # (n+1)-st column of V, H = U S V^H
    p = u                          # p(z) = sum_k u_k z^k           (ascending)
    q = v[::-1]                    # q(z) = sum_k v_{L-k} z^k      (ascending)

    def h_of(z):
        return np.polyval(a[::-1], z)

    def rtilde(z):
        return h_of(z) - s * z ** L * np.polyval(p[::-1], z) / np.polyval(q[::-1], z)

    roots = np.roots(q[::-1])
    zk = roots[np.abs(roots) > 1.0]
    K = zk.size
    M = M or max(4096, 8 * (L + n))

    def qout(z):
        out = np.ones_like(z)
        for r in zk:
            out = out * (z - r)
        return out

    d = laurent_coefficients(lambda z: qout(z) * rtilde(z), n - 1, M)
    num = d[:K]
    info = dict(L=L, sigma_next=float(s), singular_values=S, exterior_roots=K,
                n=n, p=p, q=q, h_fun=h_of, rtilde=rtilde)
    return num, zk, info


def faber_cf(K, R1, L=None, M=None, cond_max=1e10, ls_points=20001):
    """Algorithm 2: poles ``sigma`` and weights ``beta`` of
    ``r(w) = sum_k beta_k / (w - sigma_k) ~ exp(w)`` on ``i[-R1, R1]``.

    Returns ``(sigma, beta, info)``. ``info`` holds the CF data, the condition
    number of the K x K system and which route produced the weights.
    """
    L = L or default_L(K, R1)
    a = faber_sequence_exp(R1, L, M)
    num, zk, info = cf(a, K, M)
    Kf = zk.size
    sigma = eta(zk, R1)
    # Faber sequences of w -> 1/(w - sigma_k): Laurent coefficients of
    # 1/(eta(z) - sigma_k) on a circle between 1/|z_k| and |z_k| (the unit circle)
    Mb = M or max(4096, 8 * (L + K))
    B = np.empty((Kf, Kf), dtype=np.complex128)
    for k in range(Kf):
        B[:, k] = laurent_coefficients(lambda z: 1.0 / (eta(z, R1) - sigma[k]), Kf - 1, Mb)

    # Maclaurin coefficients of r_cf (analytic in the closed unit disc)
    def rcf(z):
        den = np.ones_like(z)
        for r in zk:
            den = den * (z - r)
        return np.polyval(num[::-1], z) / den

    c = laurent_coefficients(rcf, Kf - 1, Mb)
    condB = float(np.linalg.cond(B))
    if condB <= cond_max:
        beta = np.linalg.solve(B, c)
        route = "algorithm2"
    else:
        beta = least_squares_weights(sigma, R1, ls_points)
        route = "least_squares"
    info.update(R1=R1, condB=condB, weights=route, zk=zk, num=num, rcf=rcf, Kfound=Kf)
    return sigma, beta, info


def least_squares_weights(sigma, R1, npts=20001):
    """Weights minimising ``|| sum_k beta_k/(iy - sigma_k) - exp(iy) ||_2`` over
    ``npts`` equispaced ``y`` in ``[-R1, R1]`` (the fallback reading)."""
    y = np.linspace(-R1, R1, npts)
    C = 1.0 / (1j * y[:, None] - sigma[None, :])
    beta, *_ = np.linalg.lstsq(C, np.exp(1j * y), rcond=None)
    return beta


def r_eval(z, sigma, beta):
    """``r(z) = sum_k beta_k / (z - sigma_k)`` (eq. ``partial-fraction-decomposition``)."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.zeros(z.shape, dtype=np.complex128)
    for s, b in zip(sigma, beta):
        out += b / (z - s)
    return out


def diagnostics(sigma, beta, R1, npts=100001, far=50.0):
    """Error, amplification and stability numbers of a pole set.

    * ``err_inf``: max over ``npts`` points of ``|r(iy) - exp(iy)|`` on ``[-R1, R1]``
      (the paper's ``||e||_inf``, Table 1);
    * ``amplification``: ``A = sum_k |beta_k| / Re sigma_k`` -- the factor by which
      per-pole relative solve errors can add up in the weighted sum;
    * ``max_abs_r_far``: ``max |r(iy)|`` for ``|y| <= far * R1`` (stability on the
      imaginary axis, Section 3.4);
    * ``conj_residual``: distance of the pole set from its conjugate.
    """
    y = np.linspace(-R1, R1, npts)
    err = float(np.max(np.abs(r_eval(1j * y, sigma, beta) - np.exp(1j * y))))
    yf = np.linspace(-far * R1, far * R1, 20 * npts + 1)
    rf = float(np.max(np.abs(r_eval(1j * yf, sigma, beta))))
    A = float(np.sum(np.abs(beta) / sigma.real))
    # conjugate symmetry: {sigma} == {conj sigma}, beta matched alike
    order = np.argsort(sigma.imag)
    rev = order[::-1]
    conj_res = float(np.max(np.abs(sigma[order] - np.conj(sigma[rev]))) / np.max(np.abs(sigma))
                     + np.max(np.abs(beta[order] - np.conj(beta[rev]))) / np.max(np.abs(beta)))
    return dict(err_inf=err, amplification=A, min_re_sigma=float(sigma.real.min()),
                max_re_sigma=float(sigma.real.max()), max_abs_r_far=rf,
                conj_residual=conj_res, max_abs_beta=float(np.abs(beta).max()))

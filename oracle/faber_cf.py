"""Faber-Caratheodory-Fejer poles and weights (oracle, FP64, test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use this module; it shares nothing with the GPU path.

What is computed (Section 3.2). A rational function
r(w) = sum_k beta_k / (w - sigma_k) with K poles is sought that approximates
exp(w) on the segment i[-R1, R1]. The construction works in the disc:

* The map eta(z) = (R1/2)(z - 1/z) (eq. ``map-to-imaginary``) takes the unit
  circle onto the segment, and exp(eta(e^{it})) = exp(i R1 sin t). The Faber
  coefficients of exp (eq. ``faber-series``) are therefore the Fourier
  coefficients of that function: the Bessel values a_j = J_j(R1), real. They
  are sampled here by an FFT on the circle.
* Theorem 1 (Caratheodory-Fejer): how well the truncated series
  h(z) = sum_{j<=L} a_j z^j can be matched on the circle by functions with K
  poles outside the disc is read off the Hankel matrix [a_{i+j}]. Its
  entries are real, so it is real symmetric and its singular values are the
  moduli of its eigenvalues. With lam the (K+1)-st eigenvalue in modulus and
  v its (real) eigenvector, read as the polynomial v(z) = sum_j v_j z^j, the
  best approximation r~* satisfies
      h(z) - r~*(z) = lam v(z) / v(1/z),
  which has modulus |lam| all round the circle (v(1/z) is the conjugate of
  v(z) there). Its poles outside the disc are z_k = 1/zeta_k for the roots
  zeta_k of v inside the disc; there must be exactly K of them.
* The CF approximant keeps those K poles: r_cf = N(z) / prod_k (z - z_k) with
  N the part of degree below K of the Laurent series of
  prod_k (z - z_k) r~*(z) on the circle.
* Back on the segment the poles are sigma_k = eta(z_k). The Faber transform
  is linear and takes 1/(w - sigma_k) to 1/(eta'(z_k) (z - z_k)) on the disc
  (its Maclaurin coefficients are -z_k^{-n-1} / eta'(z_k)), so the weights
  solve "transform of r = r_cf". Section 3.2 imposes this on the first K
  Maclaurin coefficients; that K x K system becomes numerically singular as
  K grows (condition number past 1e15 near K = 24); beyond ``cond_max`` = 1e9
  (where the system's rounding, about cond * 1e-16, reaches the size of the
  approximation error itself: K = 16, R1 = 28 has 7.8e9) the weights are the
  linear least-squares fit of r to exp on the segment instead (same poles).
  ``info['weights']`` says which route was taken.

Readings where the text is garbled (the index typos of Theorem 1): the
Hankel matrix is (L+1) x (L+1) with entries a_{i+j}, zero beyond L, and the
(n+1)-st singular pair is the one of index K (0-based).
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


def _poly(c, z):
    """sum_j c_j z^j for ascending coefficients ``c``."""
    return np.polyval(np.asarray(c)[::-1], z)


def hankel_spectrum(a):
    """Eigen-decomposition of the real symmetric Hankel matrix [a_{i+j}]
    (zero past L), ordered by decreasing eigenvalue modulus: returns the
    signed eigenvalues (their moduli are the singular values) and the
    eigenvectors as columns."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        if np.max(np.abs(a.imag)) > 1e-13 * np.max(np.abs(a)):
            raise ValueError("the Faber coefficients of exp on i[-R1, R1] are real")
        a = a.real
    L = a.size - 1
    i = np.arange(L + 1)
    idx = i[:, None] + i[None, :]
    Hk = np.where(idx <= L, a[np.minimum(idx, L)], 0.0)
    lam, vec = np.linalg.eigh(Hk)
    order = np.argsort(-np.abs(lam), kind="stable")
    return lam[order], vec[:, order]


def cf(a, K, M=None):
    """Caratheodory-Fejer approximation of type (K-1, K) of
    ``h(z) = sum_{j<=L} a_j z^j`` on the unit circle (Theorem 1).

    Returns ``(num, zk, info)``: ``num`` the ascending coefficients of the
    numerator N of r_cf, ``zk`` its poles outside the disc (so
    ``r_cf = N(z) / prod_k (z - zk)``) and diagnostics, among them ``h_fun``
    and ``rtilde`` (the best approximation r~*) for checking Theorem 1.
    """
    a = np.asarray(a)
    L = a.size - 1
    lam_all, vec = hankel_spectrum(a)
    lam, v = lam_all[K], vec[:, K]
    hc = a.real if np.iscomplexobj(a) else a

    def h_of(z):
        return _poly(hc, z)

    def rtilde(z):
        return h_of(z) - lam * _poly(v, z) / _poly(v, 1.0 / z)

    zeta = np.roots(v[::-1])             # the roots of v(z)
    zk = 1.0 / zeta[np.abs(zeta) < 1.0]  # poles of r~* outside the disc
    M = M or max(4096, 8 * (L + K))

    def qout(z):
        out = np.ones_like(z)
        for r in zk:
            out = out * (z - r)
        return out

    num = laurent_coefficients(lambda z: qout(z) * rtilde(z), K - 1, M)[: zk.size]
    info = dict(L=L, sigma_next=float(abs(lam)), lam=float(lam), singular_values=np.abs(lam_all),
                exterior_roots=int(zk.size), n=K, v=v, h_fun=h_of, rtilde=rtilde)
    return num, zk, info


def faber_cf(K, R1, L=None, M=None, cond_max=1e9, ls_points=20001):
    """Poles ``sigma`` and weights ``beta`` of ``r(w) = sum_k beta_k / (w - sigma_k)
    ~ exp(w)`` on ``i[-R1, R1]`` (Section 3.2).

    Returns ``(sigma, beta, info)``; ``info`` holds the CF data, the condition
    number of the Maclaurin matching system and which route gave the weights.
    """
    L = L or default_L(K, R1)
    a = faber_sequence_exp(R1, L, M)
    num, zk, info = cf(a, K, M)
    Kf = zk.size
    sigma = eta(zk, R1)

    def rcf(z):
        den = np.ones_like(z)
        for r in zk:
            den = den * (z - r)
        return _poly(num, z) / den

    # transform of r = r_cf on the first Kf Maclaurin coefficients: the
    # transform of 1/(w - sigma_k) contributes -z_k^{-n-1} / eta'(z_k) to
    # coefficient n; r_cf is analytic on the closed disc
    n = np.arange(Kf)[:, None]
    B = -zk[None, :] ** (-n - 1.0) / eta_prime(zk, R1)[None, :]
    c = laurent_coefficients(rcf, Kf - 1, M or max(4096, 8 * (L + K)))
    condB = float(np.linalg.cond(B)) if Kf else np.inf
    if condB <= cond_max:
        beta = np.linalg.solve(B, c)
        route = "maclaurin"
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

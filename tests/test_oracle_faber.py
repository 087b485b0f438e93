"""Pins of the oracle's Faber-CF construction (Section 3.2, Theorem 1).

Each test checks the oracle against something other than itself: a closed
form (Jacobi-Anger Bessel coefficients, the Laurent series of the resolvent
of the conformal map), an invariant of Theorem 1 (constant-modulus error of
the best extended approximation), the paper's printed Table 1, or the
stability statements of Section 3.4.
"""
import os

import numpy as np
import pytest
from scipy.special import jv

from oracle import faber_cf as fcf

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_faber_cf.txt")

CASES = [(10, 10.0), (10, 10.5), (16, 28.0), (16, 32.0), (32, 80.0), (64, 180.0)]


@pytest.fixture(scope="module")
def polesets():
    return {c: fcf.faber_cf(*c) for c in CASES}


@pytest.mark.parametrize("R1", [10.0, 28.0, 180.0])
def test_faber_coefficients_are_bessel(R1):
    # exp(eta(e^{it})) = exp(i R1 sin t) = sum_n J_n(R1) e^{int}  (Jacobi-Anger)
    L = fcf.default_L(16, R1)
    a = fcf.faber_sequence_exp(R1, L)
    assert np.max(np.abs(a - jv(np.arange(L + 1), R1))) < 1e-14


def test_resolvent_faber_sequence_closed_form(polesets):
    # 1/(eta(z) - eta(zk)) = (2/R1) z/((z - zk)(z + 1/zk)); its z^n coefficient on
    # 1/|zk| < |z| < |zk| is -zk^{-n-1}/eta'(zk).
    s, b, info = polesets[(16, 28.0)]
    R1 = 28.0
    for zk, sk in zip(info["zk"][:4], s[:4]):
        c = fcf.laurent_coefficients(lambda z: 1.0 / (fcf.eta(z, R1) - sk), 20, 4096)
        n = np.arange(21)
        closed = -zk ** (-n - 1.0) / fcf.eta_prime(zk, R1)
        assert np.max(np.abs(c - closed)) < 1e-12 * np.max(np.abs(closed))


def _hankel_singular_values(a):
    # the Hankel matrix of Theorem 1 from its definition, its singular values by SVD
    L = a.size - 1
    idx = np.add.outer(np.arange(L + 1), np.arange(L + 1))
    return np.linalg.svd(np.where(idx <= L, a[np.minimum(idx, L)], 0.0), compute_uv=False)


@pytest.mark.parametrize("case", CASES)
def test_theorem1_singular_values_and_constant_modulus_error(polesets, case):
    # Theorem 1: the approximation number of h with K exterior poles is the
    # (K+1)-st Hankel singular value; the oracle reads it off a symmetric
    # eigenproblem, checked here against an SVD of the same matrix, and the
    # error of the best approximation has that modulus all round the circle
    s, b, info = polesets[case]
    K, R1 = case
    sv = _hankel_singular_values(fcf.faber_sequence_exp(R1, info["L"]))
    assert np.allclose(info["singular_values"][:K + 3], sv[:K + 3], rtol=1e-9, atol=1e-15 * sv[0])
    assert info["sigma_next"] == pytest.approx(sv[K], rel=1e-9)
    th = np.exp(2j * np.pi * np.arange(997) / 997)
    e = np.abs(info["h_fun"](th) - info["rtilde"](th))
    assert np.allclose(e / info["sigma_next"], 1.0, atol=1e-6)


@pytest.mark.parametrize("case", [(10, 10.0), (10, 10.5), (16, 28.0), (16, 32.0)])
def test_cf_approximant_is_near_best_on_the_circle(polesets, case):
    # dropping the negative-index tail of r~* keeps the CF approximant within
    # a few per cent of the best error sigma_{K+1} on the circle (while its
    # numerator-denominator form is well conditioned; for larger K the pole
    # set is checked through r on the segment instead)
    s, b, info = polesets[case]
    th = np.exp(2j * np.pi * np.arange(4001) / 4001)
    e = np.max(np.abs(info["h_fun"](th) - info["rcf"](th)))
    assert info["sigma_next"] <= e * (1 + 1e-6) and e <= 1.1 * info["sigma_next"]


@pytest.mark.parametrize("case", CASES)
def test_pole_set_invariants(polesets, case):
    K, R1 = case
    s, b, info = polesets[case]
    d = fcf.diagnostics(s, b, R1)
    assert info["Kfound"] == K                       # exactly K exterior roots
    assert np.all(np.abs(info["zk"]) > 1.0)
    assert d["conj_residual"] < 1e-6                 # real Faber coefficients
    assert d["min_re_sigma"] > 0.0                   # poles off the imaginary axis
    # Faber transform of a CF approximant: error about twice sigma_{K+1}
    assert d["err_inf"] <= 2.5 * info["sigma_next"]
    assert d["err_inf"] >= 1.0 * info["sigma_next"]
    # Section 3.4: |r| exceeds one by at most about ||e||_inf on the axis, and
    # decays away from the interval (deg p < deg q)
    assert d["max_abs_r_far"] <= 1.0 + 2.0 * d["err_inf"]
    assert abs(fcf.r_eval(1e6j, s, b)) < 1e-3


def test_maclaurin_weights_agree_with_least_squares_when_well_conditioned(polesets):
    for case in [(10, 10.0), (10, 10.5)]:
        s, b, info = polesets[case]
        assert info["weights"] == "maclaurin"
        bl = fcf.least_squares_weights(s, case[1])
        assert np.max(np.abs(bl - b)) / np.max(np.abs(b)) < 1e-6


def test_table1_order_of_magnitude():
    vals = {}
    with open(GOLD) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    K, R1, err = int(vals["K"]), vals["R1"], vals["err_inf"]
    # With K = 16 at R1 = 10 the 17th Hankel singular value lies below the FP64
    # noise floor: the printed choice is degenerate in double precision.
    a = fcf.faber_sequence_exp(R1, fcf.default_L(K, R1))
    S = np.linalg.svd(np.where(np.add.outer(np.arange(a.size), np.arange(a.size)) < a.size,
                               a[np.minimum(np.add.outer(np.arange(a.size), np.arange(a.size)), a.size - 1)], 0))[1]
    assert S[K] / S[0] < 1e-16
    # The accuracy the table prints on i[-10, 10] is reached by the largest
    # non-degenerate pole count at the same R1 (K = 10): same order of magnitude.
    s, b, info = fcf.faber_cf(10, R1)
    d = fcf.diagnostics(s, b, R1)
    assert err / 4 < d["err_inf"] < err * 4
    # and |r(iy)| - 1 is of the order the paper states (Section 3.4)
    y = np.linspace(-R1, R1, 20001)
    excess = np.max(np.abs(fcf.r_eval(1j * y, s, b))) - 1.0
    assert excess < 4 * vals["stability_excess"]

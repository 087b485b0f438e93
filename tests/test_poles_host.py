"""Host setup of the poles (the package's Faber-CF construction) against the
oracle's construction of the same approximation (Section 3.2), and the
per-configuration choice of (K, R1) (Section "Step-Size Requirements")."""
import numpy as np
import pytest

from oracle import faber_cf as fcf
from oracle import hamiltonian as ham
from paper_1912_03312_amd import inputs
from paper_1912_03312_amd.poles import faber_cf_poles, select_poles


def _r(sigma, beta, y):
    return (1.0 / (1j * y[:, None] - sigma[None, :])) @ beta


@pytest.mark.parametrize("K,R1", [(10, 10.5), (16, 28.0), (32, 80.0), (64, 180.0)])
def test_poles_match_oracle(K, R1):
    # the same poles (roots of the CF polynomial through the conformal map);
    # the package fits the weights by least squares, so its error on
    # i[-R1, R1] is at most the oracle's
    s1, b1, info = faber_cf_poles(K, R1)
    s2, b2, d2 = fcf.faber_cf(K, R1)
    o1, o2 = np.lexsort((s1.real, s1.imag)), np.lexsort((s2.real, s2.imag))
    assert np.max(np.abs(s1[o1] - s2[o2]) / np.abs(s2[o2])) <= 1e-8
    y = np.linspace(-R1, R1, 20001)
    e1 = np.max(np.abs(_r(s1, b1, y) - np.exp(1j * y)))
    e2 = np.max(np.abs(_r(s2, b2, y) - np.exp(1j * y)))
    assert e1 <= 1.05 * e2
    assert abs(info["err_inf"] - e1) <= 0.05 * e1
    # poles off the imaginary axis: the shifts s_j = i hbar sigma_j / dt then
    # have Im s_j != 0 and every (H - s_j) with Hermitian H is nonsingular
    assert np.all(np.abs(s1.real) > 1e-3 * R1)


def test_select_poles_meets_the_step_size_condition():
    # 1D harmonic spectrum: R1 covers dt * max|lambda| (or the half-width when
    # centered), the returned K meets the target and no smaller K of the list does
    wl = inputs.workload("1d_harmonic")
    lo, hi = ham.gershgorin(wl.grid.n, wl.grid.h, wl.V)
    dt, target = 0.05, 1e-6
    Ks = (10, 16, 24, 32, 48)
    for centered in (False, True):
        sel = select_poles(dt, lo, hi, target, centered=centered, Ks=Ks)
        w = 0.5 * (hi - lo) if centered else max(abs(lo), abs(hi))
        assert sel["R1"] >= dt * w
        assert sel["info"]["err_inf"] <= target
        for K in Ks:
            if K >= sel["K"]:
                break
            try:
                _, _, info = faber_cf_poles(K, sel["R1"])
                assert info["err_inf"] > target
            except ValueError:
                pass
    # centering halves R1, so it never needs more poles
    assert select_poles(dt, lo, hi, target, centered=True, Ks=Ks)["K"] <= select_poles(dt, lo, hi, target, Ks=Ks)["K"]
    with pytest.raises(ValueError):
        select_poles(dt, lo, hi, 1e-30, Ks=(10, 16))

"""Identities of the finite-difference stencil that the tiled Lanczos pass
relies on (CPU; the sparse H of the oracle against a direct evaluation).

1. Energy form. For H = -(hbar^2/2m) Lap_h + diag(V) with zero Dirichlet
   values outside the grid (Section 1) and c_a = hbar^2 / (2 m h_a^2),
     <u, H u> = sum_i V_i |u_i|^2
              + sum_a c_a sum_i (|u_i - u_{i+e_a}|^2 + [i_a = 0] |u_i|^2),
   with u = 0 past the last point of every axis. The pass forms
   alpha_{j+1} = c_{j+1}^2 <u_{j+1}, H u_{j+1}> from this sum, which needs
   forward neighbours only.
2. Relabelling. A 2D grid (ny, nx) in C order is the same vector as a 3D
   grid (ny, 1, nx) with no middle axis: its H is the same matrix (the
   tiled pass marches along the rows of 2D instances in this form).
"""
import numpy as np
import pytest

from oracle import hamiltonian as ham


def energy_form(u, V, c):
    u = u.reshape(V.shape)
    e = float(np.sum(V * np.abs(u) ** 2))
    for a in range(u.ndim):
        if c[a] == 0.0:
            continue
        pad = [(0, 0)] * u.ndim
        pad[a] = (0, 1)
        up = np.pad(u, pad)  # u = 0 past the last point of axis a
        fwd = np.take(up, np.arange(1, u.shape[a] + 1), axis=a)
        first = np.take(u, [0], axis=a)
        e += c[a] * (float(np.sum(np.abs(u - fwd) ** 2)) + float(np.sum(np.abs(first) ** 2)))
    return e


@pytest.mark.parametrize("shape,h", [((5, 7, 9), (0.3, 0.2, 0.25)), ((1, 1, 13), (1.0, 1.0, 0.1)),
                                     ((6, 11), (0.15, 0.4)), ((17,), (0.05,)), ((2, 3, 2), (1.0, 0.5, 2.0))])
def test_energy_form_equals_quadratic_form(shape, h):
    rng = np.random.default_rng(sum(shape))
    V = rng.random(shape) * 5.0 - 1.0
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    H = ham.hamiltonian(shape, h, V, hbar=1.3, mass=0.7)
    quad = np.vdot(u.ravel(), H @ u.ravel())
    c = [1.3 ** 2 / (2 * 0.7 * x * x) for x in h]
    e = energy_form(u, V, c)
    assert abs(quad.imag) <= 1e-12 * abs(quad.real)  # H is Hermitian
    assert abs(e - quad.real) <= 1e-12 * abs(quad.real), (e, quad)
    # a dropped boundary term or a wrong coefficient is visible
    assert abs(energy_form(u, V, [0.0] + c[1:]) - quad.real) > 1e-6 * abs(quad.real)


def test_rows_as_planes_relabelling():
    rng = np.random.default_rng(3)
    ny, nx = 9, 14
    hy, hx = 0.2, 0.3
    V = rng.random((ny, nx))
    u = rng.standard_normal(ny * nx) + 1j * rng.standard_normal(ny * nx)
    H2 = ham.hamiltonian((ny, nx), (hy, hx), V)
    # the (ny, 1, nx) form: the stencil with the middle axis absent
    cy, cx = 1.0 / (2 * hy * hy), 1.0 / (2 * hx * hx)
    u3 = u.reshape(ny, 1, nx)
    p = np.pad(u3, ((1, 1), (0, 0), (1, 1)))
    nb0 = p[:-2, :, 1:-1] + p[2:, :, 1:-1]
    nb2 = p[1:-1, :, :-2] + p[1:-1, :, 2:]
    Hu3 = (2 * (cy + cx) + V.reshape(ny, 1, nx)) * u3 - (cx * nb2 + cy * nb0)
    assert np.allclose(Hu3.ravel(), H2 @ u, rtol=0, atol=1e-12 * np.abs(H2 @ u).max())
    assert abs(energy_form(u3, V.reshape(ny, 1, nx), [cy, 0.0, cx]) - np.vdot(u, H2 @ u).real) <= \
        1e-12 * abs(np.vdot(u, H2 @ u).real)

"""Seeded synthetic inputs for the REXI propagation step.

This module is shared by the GPU path, the CPU oracle, the tests and the
benchmark. It holds grids, potentials, initial wave packets and the five
workload descriptions, and none of the method's arithmetic: no Hamiltonian,
no shifted solve, no pole sum and no pole construction.

Conventions (readings of the paper, stated once here):

* Grid: ``n[a]`` interior unknowns per axis on ``[lo[a], hi[a]]``; the zero
  Dirichlet values of Section 1 sit on the boundary and are not stored, so
  ``h[a] = (hi[a] - lo[a]) / (n[a] + 1)`` and ``x[a][i] = lo[a] + (i + 1) h[a]``.
* Storage: C order, last axis contiguous, complex values interleaved
  (the layout of ``numpy.complex128`` / ``torch.complex128``).
* Inner product: ``<phi, psi>_h = h^d sum conj(phi) psi``; an L2-normalised
  state has ``h^d sum |psi|^2 = 1`` (the discrete form of the normalisation
  of the Gaussian wave packet, eq. ``wave-package``, Section 4).
* Gaussian packet (eq. ``wave-package``) with ``Sigma = width^2 I`` and mean
  momentum ``p = hbar k``.
* Units: Hartree atomic units, ``hbar = m = 1`` (Section 4).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Grid:
    """A d-dimensional tensor grid of interior points (d = 1, 2 or 3)."""

    n: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]

    def __post_init__(self):
        if not (1 <= len(self.n) <= 3) or len(self.lo) != len(self.n) or len(self.hi) != len(self.n):
            raise ValueError("grid must have 1..3 axes with matching lo/hi")
        if any(int(k) < 1 for k in self.n):
            raise ValueError("every axis needs at least one interior point")
        if any(not (b > a) for a, b in zip(self.lo, self.hi)):
            raise ValueError("need lo < hi on every axis")

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def size(self) -> int:
        return int(np.prod(self.n))

    @property
    def h(self) -> Tuple[float, ...]:
        return tuple((b - a) / (k + 1) for k, a, b in zip(self.n, self.lo, self.hi))

    @property
    def cell_volume(self) -> float:
        return float(np.prod(self.h))

    def axes(self):
        return [a + (np.arange(k) + 1.0) * hh for k, a, hh in zip(self.n, self.lo, self.h)]

    def mesh(self):
        return np.meshgrid(*self.axes(), indexing="ij")


def cube(n: int, L: float, ndim: int) -> Grid:
    """The grid ``n^ndim`` on ``[-L, L]^ndim``."""
    return Grid((n,) * ndim, (-L,) * ndim, (L,) * ndim)


# ---------------------------------------------------------------- potentials

def harmonic(grid: Grid, omega: float = 1.0, mass: float = 1.0) -> np.ndarray:
    """``V = m omega^2 |r|^2 / 2`` sampled at the interior points (float64)."""
    r2 = sum(x * x for x in grid.mesh())
    return (0.5 * mass * omega * omega * r2).astype(np.float64)


def double_well_2d(grid: Grid) -> np.ndarray:
    """``V = 0.05 (x^2 - 16)^2 + 0.5 y^2`` (separable in x and y)."""
    if grid.ndim != 2:
        raise ValueError("double well is a 2D potential")
    x, y = grid.mesh()
    return (0.05 * (x * x - 16.0) ** 2 + 0.5 * y * y).astype(np.float64)


def double_well_parts(grid: Grid):
    """The two 1D factors of :func:`double_well_2d`: ``V = Vx(x) + Vy(y)``."""
    x, y = grid.axes()
    return 0.05 * (x * x - 16.0) ** 2, 0.5 * y * y


def gaussian_bumps(grid: Grid, seed: int, nbumps: int = 20,
                   amp: Tuple[float, float] = (-2.0, 2.0),
                   width: Tuple[float, float] = (0.5, 2.0)) -> np.ndarray:
    """Sum of ``nbumps`` Gaussian bumps ``A exp(-|r - c|^2 / (2 w^2))``.

    Draw order from ``numpy.random.default_rng(seed)``: all centres (uniform
    in the box, shape ``[nbumps, d]``), then amplitudes ``U(amp)``, then
    widths ``U(width)``.
    """
    rng = np.random.default_rng(seed)
    d = grid.ndim
    lo = np.asarray(grid.lo, dtype=np.float64)
    hi = np.asarray(grid.hi, dtype=np.float64)
    centres = lo + (hi - lo) * rng.random((nbumps, d))
    amps = rng.uniform(amp[0], amp[1], nbumps)
    widths = rng.uniform(width[0], width[1], nbumps)
    mesh = grid.mesh()
    V = np.zeros(grid.n, dtype=np.float64)
    for b in range(nbumps):
        r2 = sum((mesh[a] - centres[b, a]) ** 2 for a in range(d))
        V += amps[b] * np.exp(-r2 / (2.0 * widths[b] ** 2))
    return V


def step_barrier_1d(grid: Grid, vmax: float = 15.0, cbarr: float = 0.005) -> np.ndarray:
    """The tunnelling barrier of Section 4.1: ``vmax`` where ``|x| <= cbarr/2``."""
    (x,) = grid.axes()
    return np.where(np.abs(x) <= cbarr / 2.0, vmax, 0.0).astype(np.float64)


# ----------------------------------------------------------- wave packets

def gaussian_packet(grid: Grid, centre: Sequence[float], width: float,
                    momentum: Sequence[float], hbar: float = 1.0) -> np.ndarray:
    """Gaussian wave packet of eq. ``wave-package`` with ``Sigma = width^2 I``.

    ``momentum`` is the mean momentum ``p``; the phase is ``<p, r - c>/hbar``.
    The result is complex128, normalised so that ``h^d sum |psi|^2 = 1``.
    """
    mesh = grid.mesh()
    r2 = sum((mesh[a] - centre[a]) ** 2 for a in range(grid.ndim))
    phase = sum(momentum[a] * (mesh[a] - centre[a]) for a in range(grid.ndim)) / hbar
    psi = np.exp(-0.5 * r2 / (width * width)) * np.exp(1j * phase)
    nrm = np.sqrt(grid.cell_volume * np.sum(np.abs(psi) ** 2))
    return (psi / nrm).astype(np.complex128)


def seeded_packet(grid: Grid, seed: int, centre: Sequence[float], jitter: float,
                  width: float = 1.0, pmax: float = 1.0, hbar: float = 1.0) -> np.ndarray:
    """Packet at ``centre + U(-jitter, jitter)^d`` with ``p ~ U(-pmax, pmax)^d``.

    Draw order from ``default_rng(seed)``: the centre offset, then the momentum.
    """
    rng = np.random.default_rng(seed)
    d = grid.ndim
    c = np.asarray(centre, dtype=np.float64) + rng.uniform(-jitter, jitter, d)
    p = rng.uniform(-pmax, pmax, d)
    return gaussian_packet(grid, c, width, p, hbar)


def random_state(n: int, seed: int) -> np.ndarray:
    """A complex normal vector of length ``n`` (unit 2-norm), for unit tests."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return (z / np.linalg.norm(z)).astype(np.complex128)


# ------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    """One REXI workload: a grid, a potential, an initial state and a step plan.

    ``R1`` is the half-length of the approximation interval ``i[-R1, R1]`` of
    the conformal map (eq. ``map-to-imaginary``); the workloads themselves do
    not fix it and the values below are the parity-first choices (small
    pole-sum amplification).
    """

    name: str
    grid: Grid
    V: np.ndarray
    psi0: np.ndarray
    dt: float
    steps: int
    K: int
    R1: float
    tol: float
    m: int = 30
    hbar: float = 1.0
    mass: float = 1.0
    precision: str = "c128"
    center: bool = False
    note: str = ""


def workload(name: str, scale: Optional[int] = None) -> Workload:
    """Build one of the named workloads.

    ``scale`` replaces the points per axis (same domain and physics) to get a
    smaller instance of the same workload for parity tests.

    * ``1d_harmonic``  -- 256 points on [-10, 10], V = x^2/2, packet at -2,
      width 1, k = 1; dt 0.1, 10 steps, K = 16, tol 1e-12.
    * ``2d_double_well`` -- 512^2 on [-20, 20]^2, V = 0.05(x^2-16)^2 + y^2/2,
      packet near (-4, 0) (seed 2); dt 0.5, 20 steps, K = 32, GMRES(30),
      tol 1e-10.
    * ``3d_bumps`` -- 128^3 on [-15, 15]^3, 20 Gaussian bumps (seed 3),
      packet near the origin (seed 30); dt 1.0, 10 steps, K = 64,
      complex64 inner solves refined in FP64 to 1e-10.
    * ``2d_adjoint`` -- 256^2 on [-10, 10]^2, 20 bumps (seed 5), packet
      (seed 50), target packet (seed 51); dt 0.5, 20 steps, K = 32.
    * ``1d_tunnel`` -- the tunnelling problem of Section 4.1 (Table 2) in
      finite differences: 8001 points (the paper's degrees of freedom) on
      [-20.005, 20.005], so h = 0.005 = C_barr and the barrier of height 15 is
      one grid point of the same integrated strength; packet at -3 with
      Sigma = 4 I (width 2) and momentum 5; dt 2e-4 for T = 0.2 (1000 steps);
      K = 10 poles on i[-10, 10] (the largest K that is not degenerate in FP64
      at R1 = 10). dt lam_max = 16 exceeds R1, so the step is centered
      (half-width 8).
    """
    if name == "1d_harmonic":
        g = cube(scale or 256, 10.0, 1)
        return Workload(name, g, harmonic(g), gaussian_packet(g, (-2.0,), 1.0, (1.0,)),
                        dt=0.1, steps=10, K=16, R1=28.0, tol=1e-12)
    if name == "2d_double_well":
        g = cube(scale or 512, 20.0, 2)
        return Workload(name, g, double_well_2d(g), seeded_packet(g, 2, (-4.0, 0.0), 0.5),
                        dt=0.5, steps=20, K=32, R1=80.0, tol=1e-10, m=30)
    if name == "3d_bumps":
        g = cube(scale or 128, 15.0, 3)
        return Workload(name, g, gaussian_bumps(g, 3), seeded_packet(g, 30, (0.0, 0.0, 0.0), 2.0),
                        dt=1.0, steps=10, K=64, R1=180.0, tol=1e-10, m=30, precision="c64")
    if name == "2d_adjoint":
        g = cube(scale or 256, 10.0, 2)
        return Workload(name, g, gaussian_bumps(g, 5), seeded_packet(g, 50, (-2.0, 0.0), 1.0),
                        dt=0.5, steps=20, K=32, R1=80.0, tol=1e-12)
    if name == "1d_tunnel":
        g = Grid((scale or 8001,), (-20.005,), (20.005,))
        return Workload(name, g, step_barrier_1d(g, 15.0, 0.005), gaussian_packet(g, (-3.0,), 2.0, (5.0,)),
                        dt=2e-4, steps=1000, K=10, R1=10.0, tol=1e-12, m=100, center=True)
    raise KeyError(name)


def adjoint_target(grid: Grid) -> np.ndarray:
    """The target packet of the ``2d_adjoint`` workload (seed 51)."""
    return seeded_packet(grid, 51, (2.0, 0.0), 1.0)


def batch_instances(count: int = 256, seed: int = 4000,
                    sides: Sequence[int] = tuple(range(64, 513, 32)),
                    Ks: Sequence[int] = (16, 24, 32, 48),
                    max_side: Optional[int] = None):
    """The uneven-size batch: ``count`` independent 2D instances.

    Instance ``i`` draws, from ``default_rng(seed + i)`` in this order: its side
    (uniform over ``sides``), its time step ``U(0.2, 1.0)`` and its pole count
    (uniform over ``Ks``). Its potential is 20 bumps (seed ``seed + i``) and its
    packet is seeded likewise, on ``[-10, 10]^2``. ``max_side`` caps the side
    (for small parity runs of the same recipe).
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        side = int(rng.choice(np.asarray(sides)))
        dt = float(rng.uniform(0.2, 1.0))
        K = int(rng.choice(np.asarray(Ks)))
        if max_side is not None:
            side = min(side, max_side)
        g = cube(side, 10.0, 2)
        out.append(dict(grid=g, V=gaussian_bumps(g, seed + i),
                        psi0=seeded_packet(g, seed + i, (-4.0, 0.0), 0.5),
                        dt=dt, K=K))
    return out


#: parity-first half-widths R1 of the approximation interval per pole count
#: (pole-sum amplification of order 1e4..1e5)
R1_PARITY = {10: 10.5, 16: 28.0, 24: 54.0, 32: 80.0, 48: 130.0, 64: 180.0}
